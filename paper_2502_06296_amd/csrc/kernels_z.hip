// Wall-normal solves (paper Sec. 2.2.3 steps 4-6, Sec. 2.2.4, Algorithm 2).
//
// Both the Poisson z solve and the Helmholtz apply use the partition method
// of the paper inside one workgroup: each column of N_z unknowns is cut into
// P chunks, one thread per chunk holds its m = N_z/P values in registers,
// reduces them to the two boundary rows of the chunk, the 2P boundary rows of
// every column form a tridiagonal system that is solved by parallel cyclic
// reduction in LDS, and each thread rebuilds its interior. Where the paper
// exchanges the boundary rows between GPUs with an all-to-all, here they only
// cross the LDS of one compute unit.
//
// All rows are sign-normalised M-matrix rows
//   -alpha x[k-1] + (alpha + gamma + eps) x[k] - gamma x[k+1] = d,
// alpha, gamma, eps >= 0, and every elimination keeps each diagonal as a sum
// of non-negative parts (a forward excess, a backward excess), so no pivot is
// ever formed by subtraction.
#include "pf_internal.hpp"

#include <algorithm>
#include <type_traits>

namespace pf {

// ------------------------------------------------------- Poisson z solve
// Thread (col, ch): column i = ib*TI + col of plane j, rows [ch*M, ch*M+M)
// of the column. Columns are padded to P*M rows with identity rows (alpha =
// gamma = 0, excess = 1), which decouple exactly because the last real row
// has gamma = 0; the padding keeps every loop and register index a compile-
// time constant. The chunk's Step 1 coefficients depend on the column's
// shift lambda = sx[i] + sy[j] (the modified wavenumbers; sy holds the
// packed-slot values for the x slots 0 and 1 and, from index ny on, the
// values of the natural-order complex y modes of the other slot pairs), so
// they are
// rebuilt in registers: an upward sweep gives the reduced first row, a
// downward sweep (Algorithm 2, Step 1 and the forward half of Step 2, fused)
// gives the reduced last row and leaves the forward-reduced d and the pivots
// 1/b. After the reduced solve the interior follows from one forward and one
// backward substitution with the chunk's end values as Dirichlet data.
// 1/b for the positive, normal pivots of the eliminations: the hardware
// reciprocal refined by two Newton steps (about 1 ulp), a third of the
// instructions of an IEEE division.
__device__ __forceinline__ double rcp64(double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  return __builtin_fma(r, e, r);
}
// A compiler memory fence every fourth row of an unrolled sweep: the
// compiler would otherwise issue every table and field read of the sweep up
// front and run out of registers. It emits no instruction.
__device__ __forceinline__ void sched_fence(int q) {
  if ((q & 3) == 3) asm volatile("" ::: "memory");
}

template <bool FAST>
__device__ __forceinline__ double qdiv(double a, double b) {
  if constexpr (FAST) return a * rcp64(b);
  else return a / b;
}

template <typename TS, int M, int TI, int WAVES, bool FAST>
__global__ __launch_bounds__(512, WAVES) void k_zsolve(TS *__restrict__ data, int nx, int ny, int nz, int P,
                                                 const double *__restrict__ zal,
                                                 const double *__restrict__ zga,
                                                 const double *__restrict__ zex,
                                                 const double *__restrict__ sx,
                                                 const double *__restrict__ sy, size_t sp) {
  extern __shared__ double red[];  // [4][2P][TI]: alpha, gamma, eps, d of the reduced rows
  const int nr = 2 * P;
  double *RA = red, *RG = red + nr * TI, *RE = red + 2 * nr * TI, *RD = red + 3 * nr * TI;
  const int nib = nx / TI;
  const int blk = (int)xcd_block(blockIdx.x, gridDim.x);
  const int ib = blk % nib;
  const int j = blk / nib;
  const int col = threadIdx.x % TI;
  const int ch = threadIdx.x / TI;
  const int i = ib * TI + col;
  const int r0 = ch * M;
  const size_t plane = sp;
  TS *cp = data + (size_t)j * nx + i + (size_t)r0 * plane;
  // the singular column is the one with no shift at all (Poisson's (0,0);
  // the 3-D Helmholtz has 1/s in every entry of sx)
  const double lam0 = sx[i] + sy[(i >= 2 ? ny : 0) + j];
  const bool zero_col = lam0 == 0.0;
  const double lam = zero_col ? 1.0 : lam0;
  const double *al = zal + r0, *ga = zga + r0, *ex = zex + r0;

  double d[M], ib_[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    d[q] = (r0 + q < nz) ? -(double)cp[(size_t)q * plane] : 0.0;
    ib_[q] = 0.0;
  }

  // upward sweep: the first row reduced to couple x_{-1}, x_0, x_{M-1}
  double uc = ga[M - 2];
  double ue = ex[M - 2] + lam;
  double ud = d[M - 2];
  double ub = al[M - 2] + uc + ue;
#pragma unroll
  for (int q = M - 3; q >= 0; --q) {
    const double tq = qdiv<FAST>(ga[q], ub);
    uc = tq * uc;
    ue = (ex[q] + lam) + tq * ue;
    ud = d[q] + tq * ud;
    ub = al[q] + uc + ue;
  }
  // downward sweep: pivots b_q = gamma_q + |a_q| + e'_q, forward-reduced d
  double fa = al[1];
  double fe = ex[1] + lam;
  ib_[1] = qdiv<FAST>(1.0, ga[1] + fa + fe);
#pragma unroll
  for (int q = 2; q < M; ++q) {
    const double tq = al[q] * ib_[q - 1];
    fa = tq * fa;
    fe = (ex[q] + lam) + tq * fe;
    d[q] = d[q] + tq * d[q - 1];
    ib_[q] = qdiv<FAST>(1.0, ga[q] + fa + fe);
  }

  // reduced rows 2ch (first) and 2ch+1 (last) of this column
  double ra0 = al[0], rg0 = uc, re0 = ue, rd0 = ud;
  double ra1 = fa, rg1 = ga[M - 1], re1 = fe, rd1 = d[M - 1];
  const int w0 = (2 * ch) * TI + col, w1 = (2 * ch + 1) * TI + col;
  // parallel cyclic reduction over the 2P rows: after the step of stride s
  // every row couples only to rows 2s away; the sums stay subtraction-free
  for (int s = 1; s < nr; s *= 2) {
    RA[w0] = ra0; RG[w0] = rg0; RE[w0] = re0; RD[w0] = rd0;
    RA[w1] = ra1; RG[w1] = rg1; RE[w1] = re1; RD[w1] = rd1;
    __syncthreads();
    double na[2], ng[2], ne[2], nd[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = 2 * ch + h;
      const double a = h ? ra1 : ra0, g = h ? rg1 : rg0, e = h ? re1 : re0, dd = h ? rd1 : rd0;
      double k1 = 0.0, k2 = 0.0, am = 0.0, em = 0.0, dm = 0.0, gp = 0.0, ep = 0.0, dp = 0.0;
      if (r - s >= 0) {
        const int o = (r - s) * TI + col;
        am = RA[o]; em = RE[o]; dm = RD[o];
        k1 = qdiv<FAST>(a, am + RG[o] + em);
      }
      if (r + s < nr) {
        const int o = (r + s) * TI + col;
        gp = RG[o]; ep = RE[o]; dp = RD[o];
        k2 = qdiv<FAST>(g, RA[o] + gp + ep);
      }
      na[h] = k1 * am;
      ng[h] = k2 * gp;
      ne[h] = e + k1 * em + k2 * ep;
      nd[h] = dd + k1 * dm + k2 * dp;
    }
    __syncthreads();
    ra0 = na[0]; rg0 = ng[0]; re0 = ne[0]; rd0 = nd[0];
    ra1 = na[1]; rg1 = ng[1]; re1 = ne[1]; rd1 = nd[1];
  }
  const double x0 = qdiv<FAST>(rd0, ra0 + rg0 + re0);
  const double xl = qdiv<FAST>(rd1, ra1 + rg1 + re1);

  // interior: y_q = (d_q + |a_q| x0) / b_q forward, x_q = y_q + gamma_q x_{q+1} / b_q backward
  double a = al[1];
#pragma unroll
  for (int q = 1; q < M - 1; ++q) {
    if (q >= 2) a = al[q] * ib_[q - 1] * a;
    d[q] = (d[q] + a * x0) * ib_[q];
  }
  d[M - 1] = xl;
#pragma unroll
  for (int q = M - 2; q >= 1; --q) d[q] = d[q] + ga[q] * ib_[q] * d[q + 1];
  d[0] = x0;
#pragma unroll
  for (int q = 0; q < M; ++q)
    if (r0 + q < nz) cp[(size_t)q * plane] = (TS)(zero_col ? 0.0 : d[q]);
}

// Paired variant: each thread takes two adjacent slot columns (i, i+1), i
// even. Slots 2q and 2q+1 carry the real and imaginary parts of the same x
// mode, so the two columns share the shift lambda and the whole Step 1
// (pivots, reciprocals, reduced-row coefficients, the cyclic-reduction
// multipliers): only the right-hand sides are doubled. The one pair whose
// slots differ in mode (slots 0 and 1: the mean and the Nyquist mode) lives
// in the workgroups with ib == 0; those run two passes, pass p solving
// column p of every pair with that column's own shift.
template <int NR>
__device__ __forceinline__ double rcpn(double b) {
  double r = __builtin_amdgcn_rcp(b);
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const double e = __builtin_fma(-b, r, 1.0);
    r = __builtin_fma(r, e, r);
  }
  return r;
}

// The z tables are deliberately not restrict-qualified: the workgroup
// barriers then force them to be re-read (from L1) after the reduced solve
// instead of being held in registers through it.
// LDS slot of reduced row `row` of thread pair pc: consecutive pairs are
// adjacent, and with fewer than 8 pairs per workgroup every row pair is
// followed by a gap of TP slots, so the 8 lanes of one 128-bit LDS access
// (two chunks) fall in different banks.
__host__ __device__ constexpr int zskew(int tp, bool sk) { return sk && tp < 8 ? tp : 0; }
template <int TP, bool SK>
__device__ __forceinline__ int zslot(int row, int pc) {
  return (row >> 1) * (2 * TP + zskew(TP, SK)) + (row & 1) * TP + pc;
}

template <typename TS, int M, int TP, int NR, int WAVES, bool SK>
__global__ __launch_bounds__(512, WAVES) void k_zsolve2(TS *data, int nx, int ny, int nz, int P,
                                               const double *zal, const double *zga,
                                               const double *zex, const double *sx,
                                               const double *sy, size_t sp, int xr) {
  using V = cplx<TS>;  // the pair (column i, column i+1) of one row
  // LDS: the z tables of the column, (alpha, gamma) and eps of row
  // ch*M + q at [q*P + ch] (the chunks of one wave read consecutive
  // entries), then three double2 arrays of the 2P reduced rows (zslot)
  extern __shared__ double red[];
  using D2 = cplx<double>;
  const int nr = 2 * P;
  D2 *tag = reinterpret_cast<D2 *>(red);
  double *tex = reinterpret_cast<double *>(tag + P * M);
  for (int e = threadIdx.x; e < P * M; e += blockDim.x) {
    const int o = (e % M) * P + e / M;
    tag[o] = mkc<double>(zal[e], zga[e]);
    tex[o] = zex[e];
  }
  const int nib = nx / (2 * TP);
  const int blk = (int)xcd_block(blockIdx.x, gridDim.x);
  const int ib = blk % nib;
  const int j = blk / nib;
  const int pc = threadIdx.x % TP;
  const int ch = threadIdx.x / TP;
  const int i = 2 * (ib * TP + pc);
  const int r0 = ch * M;
  const size_t plane = sp;
  V *cp = reinterpret_cast<V *>(data + (size_t)j * nx + i + (size_t)r0 * plane);
  const size_t vplane = plane / 2;
  const D2 *agc = tag + ch;
  const double *exc = tex + ch;
  auto al = [&](int q) { return agc[q * P].x; };
  auto ga = [&](int q) { return agc[q * P].y; };
  auto ex = [&](int q) { return exc[q * P]; };
  __syncthreads();
  // xr (x walls): every slot is its own real x mode, so the two columns of
  // a pair have different shifts and every pair takes both passes
  const int npass = ib == 0 || xr ? 2 : 1;  // uniform per workgroup
  for (int pass = 0; pass < npass; ++pass) {
    // pass 1 exists only for the pair of slots 0 and 1; other lanes redo
    // pass 0's work on already solved data and store nothing
    const int ci = i + pass;
    const double lam0 = sx[ci] + sy[(ci >= 2 ? ny : 0) + j];
    const bool zero_col = lam0 == 0.0;  // Poisson's (0,0) only
    const double lam = zero_col ? 1.0 : lam0;
    // pass 0 stores both columns of every pair except column 1 of the pair
    // (0, 1); pass 1 stores only that column (with xr: pass 0 column 0 and
    // pass 1 column 1 of every pair)
    const bool st0 = pass == 0;
    const bool st1 = xr ? pass == 1
                        : (pass == 0 && (npass == 1 || i != 0)) || (pass == 1 && i == 0);

    double d0[M], d1[M], ib_[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      V v = V{};
      if (r0 + q < nz) v = cp[(size_t)q * vplane];
      d0[q] = -(double)v.x;
      d1[q] = -(double)v.y;
    }
    // upward sweep (reduced first row) and downward sweep (pivots, reduced last row)
    double uc = ga(M - 2);
    double ue = ex(M - 2) + lam;
    double ud0 = d0[M - 2], ud1 = d1[M - 2];
    double ub = al(M - 2) + uc + ue;
#pragma unroll
    for (int q = M - 3; q >= 0; --q) {
      const double tq = ga(q) * rcpn<NR>(ub);
      uc = tq * uc;
      ue = (ex(q) + lam) + tq * ue;
      ud0 = d0[q] + tq * ud0;
      ud1 = d1[q] + tq * ud1;
      ub = al(q) + uc + ue;
    }
    double fa = al(1);
    double fe = ex(1) + lam;
    ib_[1] = rcpn<NR>(ga(1) + fa + fe);
#pragma unroll
    for (int q = 2; q < M; ++q) {
      const double tq = al(q) * ib_[q - 1];
      fa = tq * fa;
      fe = (ex(q) + lam) + tq * fe;
      d0[q] = d0[q] + tq * d0[q - 1];
      d1[q] = d1[q] + tq * d1[q - 1];
      ib_[q] = rcpn<NR>(ga(q) + fa + fe);
    }
    // The reduced rows 2ch (first row of the chunk) and 2ch+1 (last row),
    // each kept divided by its own diagonal: coupling below A, above G,
    // excess E (A + G + E = 1) and the right-hand sides D0, D1. A cyclic-
    // reduction step on normalised rows needs no division by a neighbour's
    // pivot: row r takes A' D[r-s] and G' D[r+s] into its parts, sums its
    // new diagonal from non-negative terms and divides once. A row with no
    // neighbour at distance s already has A (or G) exactly zero, so the
    // clamped read contributes nothing.
    D2 *X1 = reinterpret_cast<D2 *>(tex + P * M);  // (A, E)
    const int span = (nr / 2) * (2 * TP + zskew(TP, SK));
    D2 *X2 = X1 + span;                    // (D0, D1)
    D2 *X3 = X2 + span;                    // (G, E)
    double A[2], G[2], E[2], D0[2], D1[2];
    {
      const double b0 = rcpn<NR>(al(0) + uc + ue), b1 = rcpn<NR>(fa + ga(M - 1) + fe);
      A[0] = al(0) * b0; G[0] = uc * b0; E[0] = ue * b0; D0[0] = ud0 * b0; D1[0] = ud1 * b0;
      A[1] = fa * b1; G[1] = ga(M - 1) * b1; E[1] = fe * b1; D0[1] = d0[M - 1] * b1; D1[1] = d1[M - 1] * b1;
    }
    for (int s = 1; s < nr; s *= 2) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int o = zslot<TP, SK>(2 * ch + h, pc);
        X1[o] = mkc<double>(A[h], E[h]);
        X2[o] = mkc<double>(D0[h], D1[h]);
        X3[o] = mkc<double>(G[h], E[h]);
      }
      __syncthreads();
      double na[2], ng[2], ne[2], n0[2], n1[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = 2 * ch + h;
        const int lo = zslot<TP, SK>(r - s < 0 ? 0 : r - s, pc);
        const int hi = zslot<TP, SK>(r + s >= nr ? nr - 1 : r + s, pc);
        const D2 ae = X1[lo], dl = X2[lo], ge = X3[hi], dh = X2[hi];
        na[h] = A[h] * ae.x;
        ng[h] = G[h] * ge.x;
        ne[h] = E[h] + A[h] * ae.y + G[h] * ge.y;
        n0[h] = D0[h] + A[h] * dl.x + G[h] * dh.x;
        n1[h] = D1[h] + A[h] * dl.y + G[h] * dh.y;
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double ib = rcpn<NR>(na[h] + ng[h] + ne[h]);
        A[h] = na[h] * ib; G[h] = ng[h] * ib; E[h] = ne[h] * ib;
        D0[h] = n0[h] * ib; D1[h] = n1[h] * ib;
      }
    }
    // decoupled: every diagonal is 1
    const double x00 = D0[0], x01 = D1[0], xl0 = D0[1], xl1 = D1[1];
    // interior: forward y_q = (d_q + |a_q| x0) / b_q, backward x_q = y_q + gamma_q x_{q+1} / b_q
    double a = al(1);
#pragma unroll
    for (int q = 1; q < M - 1; ++q) {
      if (q >= 2) a = al(q) * ib_[q - 1] * a;
      d0[q] = (d0[q] + a * x00) * ib_[q];
      d1[q] = (d1[q] + a * x01) * ib_[q];
    }
    d0[M - 1] = xl0;
    d1[M - 1] = xl1;
#pragma unroll
    for (int q = M - 2; q >= 1; --q) {
      const double c = ga(q) * ib_[q];
      d0[q] = d0[q] + c * d0[q + 1];
      d1[q] = d1[q] + c * d1[q + 1];
    }
    d0[0] = x00;
    d1[0] = x01;
    if (st0 || st1) {
#pragma unroll
      for (int q = 0; q < M; ++q) {
        if (r0 + q < nz) {
          TS *e = reinterpret_cast<TS *>(cp + (size_t)q * vplane);
          if (st0 && st1) {
            cp[(size_t)q * vplane] = V{(TS)(zero_col ? 0.0 : d0[q]), (TS)d1[q]};
          } else if (st0) {
            e[0] = (TS)(zero_col ? 0.0 : d0[q]);
          } else {
            e[1] = (TS)d1[q];
          }
        }
      }
    }
  }
}

// Separator form of the paired solve. The last row of every chunk is a
// separator; the other M-1 rows of the chunk are interior to it. A downward
// sweep from the chunk's first row (which couples to the previous separator
// by its alpha) reduces the chunk to its separator row; an upward sweep over
// the interior rows reduces the chunk's first row to its couplings with the
// previous and the own separator. The separator row then eliminates the
// next chunk's first row (read from LDS), which leaves one tridiagonal row
// per chunk in the separators alone: P rows instead of the 2P of the first-
// and-last-row reduction, one row per thread, and one cyclic-reduction step
// fewer. Every pivot is still a sum of non-negative parts:
//   separator row:  -SA x[s-1] + (SA + SG + SE) x[s] - SG x[s+1] = SD,
//   SA = fa, SG = t ug', SE = fe + t ue', SD = D + t U', t = gamma / C',
// with (fa, fe, D) from the downward sweep and (ug', ue', U', C') the next
// chunk's reduced first row.
//
// TILE: the workgroup's R*2*TP columns (128 bytes of every row) are staged
// through LDS: the whole column tile is read row by row with 16-byte loads
// (whole 128-byte lines, instead of 2*TP*sizeof(TS) bytes per row and
// thread group), every thread takes its rows from LDS, and the results go
// back the same way, after the last round. The threads take the tile's
// columns in R rounds of 2*TP; each round's columns are a region of their
// own, [P*M rows][2*TP], whose first bytes the reduced-row arrays share
// once every thread holds its rows. Only single-pass workgroups tile; the
// two-pass ones (the pair of slots 0 and 1, x walls) read and write their
// columns directly.
// DB: the three reduced-row arrays are doubled, and the steps of the cyclic
// reduction alternate between the two sets: a step writes one set while the
// previous step's reads of the other may still be in flight, so a step
// takes one barrier instead of two.
template <typename TS, int M, int TP, int NR, int WAVES, int MAXT = 512, bool TILE = false, int R = 1,
          bool DB = false>
__device__ __forceinline__ void zsolve3_body(TS *data, int nx, int ny, int nz, int P,
                                                      const double *zal, const double *zga,
                                                      const double *zex, const double *sx,
                                                      const double *sy, size_t sp, int xr,
                                             unsigned bx_, unsigned gx_) {
  static_assert(M >= 3, "a chunk needs interior rows");
  static_assert(TILE || R == 1, "rounds need the tile");
  using V = cplx<TS>;
  using D2 = cplx<double>;
  // LDS: the z tables as in k_zsolve2, then three double2 arrays [P][TP]
  // (TILE: then R tile regions, the first bytes of the current one shared
  // with the three arrays)
  extern __shared__ double red[];
  D2 *tag = reinterpret_cast<D2 *>(red);
  double *tex = reinterpret_cast<double *>(tag + P * M);
  for (int e = threadIdx.x; e < P * M; e += blockDim.x) {
    const int o = (e % M) * P + e / M;
    tag[o] = mkc<double>(zal[e], zga[e]);
    tex[o] = zex[e];
  }
  constexpr int TC = 2 * TP;  // columns of one round
  // one tile region: P*M rows of TC values, at least the three arrays
  constexpr int NX = DB ? 6 : 3;  // reduced-row arrays
  const size_t region = ((size_t)P * M * TC * sizeof(TS) > (size_t)NX * P * TP * sizeof(D2)
                             ? (size_t)P * M * TC * sizeof(TS)
                             : (size_t)NX * P * TP * sizeof(D2)) / sizeof(double);
  double *const reg0 = tex + P * M;
  D2 *X1 = reinterpret_cast<D2 *>(reg0);
  D2 *X2 = X1 + P * TP;
  D2 *X3 = X2 + P * TP;
  TS *tile = reinterpret_cast<TS *>(reg0);
  const int nib = nx / (R * TC);
  const int blk = (int)xcd_block(bx_, gx_);
  const int ib = blk % nib;
  const int j = blk / nib;
  const int pc = threadIdx.x % TP;
  const int ch = threadIdx.x / TP;
  int i = 2 * (ib * R * TP + pc);
  const int r0 = ch * M;
  const size_t plane = sp;
  V *cp = reinterpret_cast<V *>(data + (size_t)j * nx + i + (size_t)r0 * plane);
  const size_t vplane = plane / 2;
  const D2 *agc = tag + ch;
  const double *exc = tex + ch;
  auto al = [&](int q) { return agc[q * P].x; };
  auto ga = [&](int q) { return agc[q * P].y; };
  auto ex = [&](int q) { return exc[q * P]; };
  const int me = ch * TP + pc;
  const int nch = ch + 1 < P ? ch + 1 : ch;  // the last chunk's gamma is 0
  const int nb = nch * TP + pc;
  const int npass = ib == 0 || xr ? 2 : 1;  // uniform per workgroup
  // 16-byte vectors of a round's row segment and of a tile row, and the
  // tile's first row in global memory
  constexpr int EPV = 16 / (int)sizeof(TS);
  constexpr int VPR = TC / EPV;
  static_assert(!TILE || TC % EPV == 0, "tile rows are whole 16-byte vectors");
  TS *const gt = data + (size_t)j * nx + (size_t)ib * R * TC;
  const bool tiled = TILE && npass == 1;
  auto tile_io = [&](bool load) {
    for (int e = threadIdx.x; e < nz * R * VPR; e += blockDim.x) {
      const int r = e / (R * VPR), c = e % (R * VPR);
      uint4 *l = reinterpret_cast<uint4 *>(reinterpret_cast<TS *>(reg0 + (c / VPR) * region) + r * TC +
                                           (c % VPR) * EPV);
      uint4 *g = reinterpret_cast<uint4 *>(gt + (size_t)r * plane + c * EPV);
      if (load)
        *l = *g;
      else
        *g = *l;
    }
  };
  if (tiled) tile_io(true);
  __syncthreads();
  // the tiled and the direct path as separate instances of the pass loop,
  // so that neither keeps the other's addresses live
  auto passes = [&](auto tl) {
  constexpr bool TL = decltype(tl)::value;
  for (int pass = 0; pass < npass; ++pass) {
    // as in k_zsolve2: pass 1 only for column 1 of the pair of slots 0, 1,
    // or (xr) for column 1 of every pair
    const int ci = i + pass;
    const double lam0 = sx[ci] + sy[(ci >= 2 ? ny : 0) + j];
    const bool zero_col = lam0 == 0.0;  // Poisson's (0,0) only
    const double lam = zero_col ? 1.0 : lam0;
    const bool st0 = pass == 0;
    const bool st1 = xr ? pass == 1
                        : (pass == 0 && (npass == 1 || i != 0)) || (pass == 1 && i == 0);

    double d0[M], d1[M], ib_[M];
    // the 1024-thread shapes have half the registers: compiler fences keep
    // their unrolled sweeps from issuing every read up front
    constexpr bool kFence = MAXT > 512 || M >= 32;
#pragma unroll
    for (int q = 0; q < M; ++q) {
      V v = V{};
      if (r0 + q < nz)
        v = TL ? *reinterpret_cast<const V *>(tile + (r0 + q) * TC + 2 * pc) : cp[(size_t)q * vplane];
      d0[q] = -(double)v.x;
      d1[q] = -(double)v.y;
    }
    // every thread holds its rows before the reduced-row arrays reuse the tile
    if constexpr (TL) __syncthreads();
    // upward sweep over the interior: the chunk's first row in terms of the
    // previous separator (alpha_0) and the own separator (ug)
    {
      double ug = ga(M - 2), ue = ex(M - 2) + lam, u0 = d0[M - 2], u1 = d1[M - 2];
      double cb = al(M - 2) + ug + ue;
#pragma unroll
      for (int q = M - 3; q >= 0; --q) {
        const double t = ga(q) * rcpn<NR>(cb);
        ug = t * ug;
        ue = (ex(q) + lam) + t * ue;
        u0 = d0[q] + t * u0;
        u1 = d1[q] + t * u1;
        cb = al(q) + ug + ue;
        if constexpr (kFence) sched_fence(q);
      }
      X1[me] = mkc<double>(ug, ue);
      X2[me] = mkc<double>(u0, u1);
    }
    // downward sweep from the first row (coupled to the previous separator)
    double fa = al(0), fe = ex(0) + lam;
    ib_[0] = rcpn<NR>(fa + ga(0) + fe);
#pragma unroll
    for (int q = 1; q < M; ++q) {
      const double t = al(q) * ib_[q - 1];
      fa = t * fa;
      fe = (ex(q) + lam) + t * fe;
      d0[q] = d0[q] + t * d0[q - 1];
      d1[q] = d1[q] + t * d1[q - 1];
      if (q < M - 1) ib_[q] = rcpn<NR>(fa + ga(q) + fe);
      if constexpr (kFence) sched_fence(q);
    }
    __syncthreads();
    double A, G, E, S0, S1;
    {
      const D2 gu = X1[nb], uu = X2[nb];
      const double t = ga(M - 1) * rcpn<NR>(tag[nch].x + gu.x + gu.y);
      const double sa = fa, sg = t * gu.x, se = fe + t * gu.y;
      const double s0 = d0[M - 1] + t * uu.x, s1 = d1[M - 1] + t * uu.y;
      const double b = rcpn<NR>(sa + sg + se);
      A = sa * b; G = sg * b; E = se * b; S0 = s0 * b; S1 = s1 * b;
    }
    __syncthreads();
    // cyclic reduction on the P separator rows (normalised, see k_zsolve2)
    D2 *F2 = X2;  // the set the separator values go to
    if constexpr (DB) {
      D2 *const Y1 = X3 + P * TP, *const Y2 = Y1 + P * TP, *const Y3 = Y2 + P * TP;
      bool odd = false;
      for (int s = 1; s < P; s *= 2) {
        D2 *const Z1 = odd ? Y1 : X1, *const Z2 = odd ? Y2 : X2, *const Z3 = odd ? Y3 : X3;
        Z1[me] = mkc<double>(A, E);
        Z2[me] = mkc<double>(S0, S1);
        Z3[me] = mkc<double>(G, E);
        __syncthreads();
        const int lo = (ch - s < 0 ? 0 : ch - s) * TP + pc;
        const int hi = (ch + s >= P ? P - 1 : ch + s) * TP + pc;
        const D2 ae = Z1[lo], dl = Z2[lo], ge = Z3[hi], dh = Z2[hi];
        const double na = A * ae.x, ng = G * ge.x, ne = E + A * ae.y + G * ge.y;
        const double n0 = S0 + A * dl.x + G * dh.x, n1 = S1 + A * dl.y + G * dh.y;
        const double b = rcpn<NR>(na + ng + ne);
        A = na * b; G = ng * b; E = ne * b; S0 = n0 * b; S1 = n1 * b;
        odd = !odd;
      }
      // the set the last step did not read
      F2 = odd ? Y2 : X2;
    } else {
      for (int s = 1; s < P; s *= 2) {
        X1[me] = mkc<double>(A, E);
        X2[me] = mkc<double>(S0, S1);
        X3[me] = mkc<double>(G, E);
        __syncthreads();
        const int lo = (ch - s < 0 ? 0 : ch - s) * TP + pc;
        const int hi = (ch + s >= P ? P - 1 : ch + s) * TP + pc;
        const D2 ae = X1[lo], dl = X2[lo], ge = X3[hi], dh = X2[hi];
        const double na = A * ae.x, ng = G * ge.x, ne = E + A * ae.y + G * ge.y;
        const double n0 = S0 + A * dl.x + G * dh.x, n1 = S1 + A * dl.y + G * dh.y;
        __syncthreads();
        const double b = rcpn<NR>(na + ng + ne);
        A = na * b; G = ng * b; E = ne * b; S0 = n0 * b; S1 = n1 * b;
      }
    }
    // separator values: the own one and the previous chunk's
    F2[me] = mkc<double>(S0, S1);
    __syncthreads();
    const D2 xl = ch > 0 ? F2[me - TP] : mkc<double>(0.0, 0.0);
    __syncthreads();
    // interior: forward y_q = (D_q + fa_q x_lo) / b_q, backward x_q = y_q + gamma_q x_{q+1} / b_q
    double a = al(0);
#pragma unroll
    for (int q = 0; q < M - 1; ++q) {
      if (q >= 1) a = al(q) * ib_[q - 1] * a;
      d0[q] = (d0[q] + a * xl.x) * ib_[q];
      d1[q] = (d1[q] + a * xl.y) * ib_[q];
      if constexpr (kFence) sched_fence(q);
    }
    d0[M - 1] = S0;
    d1[M - 1] = S1;
#pragma unroll
    for (int q = M - 2; q >= 0; --q) {
      const double c = ga(q) * ib_[q];
      d0[q] = d0[q] + c * d0[q + 1];
      d1[q] = d1[q] + c * d1[q + 1];
      if constexpr (kFence) sched_fence(q);
    }
    if constexpr (TL) {
      // single pass: both columns, into the round's region (its reduced-row
      // arrays are read by now); the tile goes out after the last round
      __syncthreads();
#pragma unroll
      for (int q = 0; q < M; ++q)
        if (r0 + q < nz)
          *reinterpret_cast<V *>(tile + (r0 + q) * TC + 2 * pc) = V{(TS)d0[q], (TS)d1[q]};
      __syncthreads();
    } else if (st0 || st1) {
#pragma unroll
      for (int q = 0; q < M; ++q) {
        if (r0 + q < nz) {
          TS *e = reinterpret_cast<TS *>(cp + (size_t)q * vplane);
          if (st0 && st1) {
            cp[(size_t)q * vplane] = V{(TS)(zero_col ? 0.0 : d0[q]), (TS)d1[q]};
          } else if (st0) {
            e[0] = (TS)(zero_col ? 0.0 : d0[q]);
          } else {
            e[1] = (TS)d1[q];
          }
        }
      }
    }
  }
  };
  for (int rd = 0; rd < R; ++rd) {
    if (rd > 0) {
      // the next round: its columns, its tile region (which the three
      // arrays share now)
      i += 2 * TP;
      cp += TP;
      X1 = reinterpret_cast<D2 *>(reg0 + rd * region);
      X2 = X1 + P * TP;
      X3 = X2 + P * TP;
      tile = reinterpret_cast<TS *>(reg0 + rd * region);
    }
    if (tiled)
      passes(std::true_type{});
    else
      passes(std::false_type{});
  }
  if (tiled) tile_io(false);
}
template <typename TS, int M, int TP, int NR, int WAVES, int MAXT = 512, bool TILE = false, int R = 1,
          bool DB = false>
__global__ __launch_bounds__(MAXT, WAVES) void k_zsolve3(TS *data, int nx, int ny, int nz, int P,
                                                      const double *zal, const double *zga,
                                                      const double *zex, const double *sx,
                                                      const double *sy, size_t sp, int xr) {
  zsolve3_body<TS, M, TP, NR, WAVES, MAXT, TILE, R, DB>(data, nx, ny, nz, P, zal, zga, zex, sx, sy, sp, xr,
                                                        blockIdx.x, gridDim.x);
}

// one z-solve shape for several problems with the same chunk count (see
// GJobs): float32 storage, periodic x
template <int M, int TP, int NR, int WAVES, int MAXT, bool TILE, int R, bool DB = false>
__global__ __launch_bounds__(MAXT, WAVES) void k_zsolve3_grp(const GJobs g) {
  const GJob &J = g.j[blockIdx.y];
  if (blockIdx.x >= J.nblk) return;  // uniform per block
  zsolve3_body<float, M, TP, NR, WAVES, MAXT, TILE, R, DB>(static_cast<float *>(J.out), J.nx, J.ny, J.nz,
                                                           J.P, J.zal, J.zga, J.zex, J.sx, J.sy, J.sp, 0,
                                                           blockIdx.x, J.nblk);
}

// Launch shapes of the z solve: rows per thread M, columns per workgroup
// TI, minimum waves per SIMD (0: none), fast reciprocals.
// Paired variants (two columns per thread sharing their shift) take TI
// columns per workgroup as TI/2 thread pairs; nr is the Newton-step count
// of their reciprocal.
struct ZVariant {
  int M, TI, waves;
  bool fast;
  bool paired;
  int nr;
  bool skew = true;  // paired: gaps between reduced row pairs in LDS
  bool sep = false;  // paired: separator form, P reduced rows
  int maxt = 512;    // threads per workgroup at most
  bool tile = false; // separator form with the column tile staged through LDS
  int rounds = 1;    // tiled: the threads take the TI columns in rounds of TI/rounds
  bool dbl = false;  // separator form: double-buffered reduced rows, one barrier per reduction step
};
static const ZVariant kZVariants[] = {
    {16, 16, 0, false, false, 2}, {16, 16, 4, true, false, 2}, {16, 16, 0, true, false, 2},
    {8, 8, 0, true, false, 2},    {16, 8, 0, true, false, 2},  {8, 16, 0, true, false, 2},
    {16, 32, 0, true, false, 2},  {8, 8, 4, true, false, 2},   {16, 16, 0, true, true, 1},
    {8, 16, 0, true, true, 1},    {16, 32, 0, true, true, 1},  {8, 32, 0, true, true, 1},
    {16, 16, 0, true, true, 2},   {8, 8, 0, true, true, 1},    {8, 8, 4, true, true, 1},
    {8, 16, 4, true, true, 1},    {8, 8, 4, true, true, 1, false}, {8, 16, 4, true, true, 1, false},
    // separator form (k_zsolve3)
    {8, 8, 4, true, true, 1, false, true},   {8, 16, 4, true, true, 1, false, true},
    {16, 16, 0, true, true, 1, false, true}, {16, 32, 0, true, true, 1, false, true},
    {8, 32, 4, true, true, 1, false, true},
    // wide separator shapes for short columns (few chunks per column)
    {8, 64, 4, true, true, 1, false, true},  {8, 128, 4, true, true, 1, false, true},
    {16, 64, 1, true, true, 1, false, true}, {16, 128, 1, true, true, 1, false, true},
    // separator form in 1024-thread workgroups: wider rows for the long
    // columns (8 rows per thread; 16 spilled)
    {8, 32, 1, true, true, 1, false, true, 1024}, {8, 16, 1, true, true, 1, false, true, 1024},
    // separator form with 128-byte row tiles through LDS (32 float32 or 16
    // float64 columns), the 32 float32 columns of 1024-row tiles in two
    // rounds of 16: one workgroup per compute unit at 1024 rows
    {8, 32, 1, true, true, 1, false, true, 1024, true, 2},  {16, 32, 1, true, true, 1, false, true, 512, true, 2},
    {8, 16, 1, true, true, 1, false, true, 1024, true, 1},  {16, 16, 1, true, true, 1, false, true, 512, true, 1},
    {16, 32, 1, true, true, 1, false, true, 512, true, 1},  {8, 32, 1, true, true, 1, false, true, 1024, true, 1},
    {8, 16, 1, true, true, 1, false, true, 512, true, 1},   {8, 32, 1, true, true, 1, false, true, 512, true, 2},
    // 1024-thread separator shapes with double-buffered reduced rows (LDS
    // room for the second set): the 16-column float32 tile and the direct form
    {8, 16, 1, true, true, 1, false, true, 1024, true, 1, true},
    {8, 16, 1, true, true, 1, false, true, 1024, false, 1, true},
    // the 512-thread defaults of 512-row columns with double-buffered reduced rows
    {8, 16, 1, true, true, 1, false, true, 512, true, 1, true},
    {16, 32, 0, true, true, 1, false, true, 512, false, 1, true},
};
constexpr int kZVariantCount = sizeof(kZVariants) / sizeof(kZVariants[0]);

int zsolve_variant_count() { return kZVariantCount; }

// LDS bytes of a launch: paired variants hold the column's z tables and
// three double2 arrays of the reduced rows, unpaired ones four double arrays;
// tiled ones the tables and the larger of the reduced-row arrays and the
// column tile (elements of esize bytes).
static size_t zsolve_lds(const ZVariant &z, int P, int esize) {
  const int tp = z.TI / 2;
  const size_t tables = (size_t)3 * P * z.M * sizeof(double);
  const size_t nxa = z.dbl ? 6 : 3;  // reduced-row arrays
  if (z.tile) {
    const int tpr = tp / z.rounds;  // thread pairs of a round
    return tables + z.rounds * std::max(nxa * P * tpr * 2 * sizeof(double),
                                        (size_t)P * z.M * 2 * tpr * esize);
  }
  if (z.paired && z.sep) return tables + nxa * P * tp * 2 * sizeof(double);
  return z.paired ? (size_t)3 * P * (2 * tp + zskew(tp, z.skew)) * 2 * sizeof(double) + tables
                  : (size_t)4 * 2 * P * z.TI * sizeof(double);
}

bool zsolve_variant_fits(int v, int nx, int nz, int esize) {
  if (v < 0 || v >= kZVariantCount) return false;
  const ZVariant &z = kZVariants[v];
  const int P = (nz + z.M - 1) / z.M;
  const int threads = z.paired ? P * z.TI / 2 / z.rounds : P * z.TI;
  // a tiled launch needs whole 16-byte vectors per round's row segment and
  // at least two chunks
  if (z.tile && (z.TI / z.rounds * esize % 16 != 0 || P < 2)) return false;
  return threads <= z.maxt && nx % z.TI == 0 && P * z.M <= (nz + 15) / 16 * 16 &&
         zsolve_lds(z, P, esize) <= (z.maxt > 512 || z.tile ? 160 * 1024 : 65536);
}

int zsolve_default_variant(int nx, int nz, bool fp64) {
  // fastest measured on MI355X at 1024x512x512: float64 storage 40 (1.037
  // ms: separator form, 16 rows, 32 columns, double-buffered reduced rows),
  // 21 (1.050, the same with one set), 10 (1.11); float32 storage (padded
  // planes) 39 (0.711 ms: separator form, 8 rows, 16-column tiles through
  // LDS, double-buffered reduced rows), 35 (0.752, one set), 31, 18 (0.84:
  // 8 rows, 8 columns, direct); the unpaired 4
  // and 3 as fall-backs where the LDS or thread budget excludes the paired
  // shapes. At 1024 rows float64 storage takes 38 (11.06 ms at
  // 2048x1024x1024: 28 with double-buffered reduced rows; 28 11.30, 20
  // 11.52, the tiled 31 12.8, 4 22.2) and float32 storage the tiled 37 (8.01
  // ms: 16-column tiles, double-buffered reduced rows; 29 8.20, 31 8.38, 18
  // 8.9). Short
  // columns (few chunks) would leave those shapes with tiny workgroups, so
  // the first fitting shape with at least 128 threads wins, widened by the
  // 64- and 128-column shapes.
  static const int f64[] = {40, 21, 10, 19, 38, 26, 25, 24, 23, 20, 8, 4, 3},
                   f32[] = {39, 35, 37, 29, 31, 18, 19, 16, 13, 24, 23, 26, 25, 8, 4, 3};
  const int *list = fp64 ? f64 : f32;
  const int len = fp64 ? (int)(sizeof(f64) / sizeof(int)) : (int)(sizeof(f32) / sizeof(int));
  auto threads = [&](int v) {
    const ZVariant &z = kZVariants[v];
    const int P = (nz + z.M - 1) / z.M;
    return z.paired ? P * z.TI / 2 / z.rounds : P * z.TI;
  };
  for (int k = 0; k < len; ++k)
    if (zsolve_variant_fits(list[k], nx, nz, fp64 ? 8 : 4) && threads(list[k]) >= 128) return list[k];
  for (int k = 0; k < len; ++k)
    if (zsolve_variant_fits(list[k], nx, nz, fp64 ? 8 : 4)) return list[k];
  return -1;
}

template <typename TS>
hipError_t launch_zsolve(int nx, int ny, int nz, TS *data, size_t sp, const double *zal,
                         const double *zga, const double *zex, const double *sx, const double *sy,
                         int variant, hipStream_t st, bool xr) {
  // the z tables hold whole 16-row chunks (identity padding past nz)
  if (!zsolve_variant_fits(variant, nx, nz, (int)sizeof(TS))) return hipErrorInvalidValue;
  const ZVariant &z = kZVariants[variant];
  const int P = (nz + z.M - 1) / z.M;
  const size_t shm = zsolve_lds(z, P, (int)sizeof(TS));
  dim3 g((unsigned)((long)(nx / z.TI) * ny)), b(z.paired ? P * z.TI / 2 / z.rounds : P * z.TI);
#define PF_ZV(ID, M_, TI_, W_, F_)                                                                \
  case ID:                                                                                        \
    hipLaunchKernelGGL((k_zsolve<TS, M_, TI_, W_, F_>), g, b, shm, st, data, nx, ny, nz, P, zal, \
                       zga, zex, sx, sy, sp);                                                         \
    break;
  switch (variant) {
    PF_ZV(0, 16, 16, 0, false)
    PF_ZV(1, 16, 16, 4, true)
    PF_ZV(2, 16, 16, 0, true)
    PF_ZV(3, 8, 8, 0, true)
    PF_ZV(4, 16, 8, 0, true)
    PF_ZV(5, 8, 16, 0, true)
    PF_ZV(6, 16, 32, 0, true)
    PF_ZV(7, 8, 8, 4, true)
#define PF_ZP(ID, M_, TI_, NR_, W_, SK_)                                                         \
  case ID:                                                                                       \
    hipLaunchKernelGGL((k_zsolve2<TS, M_, TI_ / 2, NR_, W_, SK_>), g, b, shm, st, data, nx, ny,  \
                       nz, P, zal, zga, zex, sx, sy, sp, (int)xr);                                   \
    break;
    PF_ZP(8, 16, 16, 1, 1, true)
    PF_ZP(9, 8, 16, 1, 1, true)
    PF_ZP(10, 16, 32, 1, 1, true)
    PF_ZP(11, 8, 32, 1, 1, true)
    PF_ZP(12, 16, 16, 2, 1, true)
    PF_ZP(13, 8, 8, 1, 1, true)
    PF_ZP(14, 8, 8, 1, 4, true)
    PF_ZP(15, 8, 16, 1, 4, true)
    PF_ZP(16, 8, 8, 1, 4, false)
    PF_ZP(17, 8, 16, 1, 4, false)
#define PF_ZS(ID, M_, TI_, W_)                                                                   \
  case ID:                                                                                       \
    hipLaunchKernelGGL((k_zsolve3<TS, M_, TI_ / 2, 1, W_>), g, b, shm, st, data, nx, ny, nz, P,  \
                       zal, zga, zex, sx, sy, sp, (int)xr);                                          \
    break;
    PF_ZS(18, 8, 8, 4)
    PF_ZS(19, 8, 16, 4)
    PF_ZS(20, 16, 16, 1)
    PF_ZS(21, 16, 32, 1)
    PF_ZS(22, 8, 32, 4)
    PF_ZS(23, 8, 64, 4)
    PF_ZS(24, 8, 128, 4)
    PF_ZS(25, 16, 64, 1)
    PF_ZS(26, 16, 128, 1)
#define PF_ZW(ID, M_, TI_)                                                                       \
  case ID:                                                                                       \
    hipLaunchKernelGGL((k_zsolve3<TS, M_, TI_ / 2, 1, 1, 1024>), g, b, shm, st, data, nx, ny, nz, \
                       P, zal, zga, zex, sx, sy, sp, (int)xr);                                   \
    break;
    PF_ZW(27, 8, 32)
    PF_ZW(28, 8, 16)
#define PF_ZT(ID, M_, TI_, MAXT_, R_)                                                            \
  case ID:                                                                                       \
    hipLaunchKernelGGL((k_zsolve3<TS, M_, TI_ / 2 / R_, 1, 1, MAXT_, true, R_>), g, b, shm, st,   \
                       data, nx, ny, nz, P, zal, zga, zex, sx, sy, sp, (int)xr);                 \
    break;
    PF_ZT(29, 8, 32, 1024, 2)
    PF_ZT(30, 16, 32, 512, 2)
    PF_ZT(31, 8, 16, 1024, 1)
    PF_ZT(32, 16, 16, 512, 1)
    PF_ZT(33, 16, 32, 512, 1)
    PF_ZT(34, 8, 32, 1024, 1)
    PF_ZT(35, 8, 16, 512, 1)
    PF_ZT(36, 8, 32, 512, 2)
  case 37:
    hipLaunchKernelGGL((k_zsolve3<TS, 8, 8, 1, 1, 1024, true, 1, true>), g, b, shm, st, data, nx, ny, nz, P,
                       zal, zga, zex, sx, sy, sp, (int)xr);
    break;
  case 38:
    hipLaunchKernelGGL((k_zsolve3<TS, 8, 8, 1, 1, 1024, false, 1, true>), g, b, shm, st, data, nx, ny, nz, P,
                       zal, zga, zex, sx, sy, sp, (int)xr);
    break;
  case 39:
    hipLaunchKernelGGL((k_zsolve3<TS, 8, 8, 1, 1, 512, true, 1, true>), g, b, shm, st, data, nx, ny, nz, P,
                       zal, zga, zex, sx, sy, sp, (int)xr);
    break;
  case 40:
    hipLaunchKernelGGL((k_zsolve3<TS, 16, 16, 1, 1, 512, false, 1, true>), g, b, shm, st, data, nx, ny, nz,
                       P, zal, zga, zex, sx, sy, sp, (int)xr);
    break;
#undef PF_ZT
#undef PF_ZW
#undef PF_ZS
#undef PF_ZP
    default:
      return hipErrorInvalidValue;
  }
#undef PF_ZV
  return hipGetLastError();
}
bool zsolve_variant_groups(int variant) { return variant >= 18 && variant < kZVariantCount; }
int zsolve_chunks(int variant, int nz) { return (nz + kZVariants[variant].M - 1) / kZVariants[variant].M; }

hipError_t launch_zsolve_grp(int variant, GJobs &g, hipStream_t st) {
  if (!zsolve_variant_groups(variant) || g.count < 1 || g.count > kMaxGroupJobs) return hipErrorInvalidValue;
  const ZVariant &z = kZVariants[variant];
  const int P = (g.j[0].nz + z.M - 1) / z.M;
  unsigned mb = 1;
  for (int k = 0; k < g.count; ++k) {
    GJob &J = g.j[k];
    if ((J.nz + z.M - 1) / z.M != P || J.P != P || !zsolve_variant_fits(variant, J.nx, J.nz, 4))
      return hipErrorInvalidValue;
    J.nblk = (unsigned)((long)(J.nx / z.TI) * J.ny);
    mb = J.nblk > mb ? J.nblk : mb;
  }
  const size_t shm = zsolve_lds(z, P, 4);
  const dim3 gr(mb, (unsigned)g.count), b(P * z.TI / 2 / z.rounds);
#define PF_G(ID, M_, TI_, W_, MAXT_, TILE_, R_)                                                     \
  case ID:                                                                                         \
    hipLaunchKernelGGL((k_zsolve3_grp<M_, TI_ / 2 / R_, 1, W_, MAXT_, TILE_, R_>), gr, b, shm, st, g); \
    break;
  switch (variant) {
    PF_G(18, 8, 8, 4, 512, false, 1)
    PF_G(19, 8, 16, 4, 512, false, 1)
    PF_G(20, 16, 16, 1, 512, false, 1)
    PF_G(21, 16, 32, 1, 512, false, 1)
    PF_G(22, 8, 32, 4, 512, false, 1)
    PF_G(23, 8, 64, 4, 512, false, 1)
    PF_G(24, 8, 128, 4, 512, false, 1)
    PF_G(25, 16, 64, 1, 512, false, 1)
    PF_G(26, 16, 128, 1, 512, false, 1)
    PF_G(27, 8, 32, 1, 1024, false, 1)
    PF_G(28, 8, 16, 1, 1024, false, 1)
    PF_G(29, 8, 32, 1, 1024, true, 2)
    PF_G(30, 16, 32, 1, 512, true, 2)
    PF_G(31, 8, 16, 1, 1024, true, 1)
    PF_G(32, 16, 16, 1, 512, true, 1)
    PF_G(33, 16, 32, 1, 512, true, 1)
    PF_G(34, 8, 32, 1, 1024, true, 1)
    PF_G(35, 8, 16, 1, 512, true, 1)
    PF_G(36, 8, 32, 1, 512, true, 2)
  case 37:
    hipLaunchKernelGGL((k_zsolve3_grp<8, 8, 1, 1, 1024, true, 1, true>), gr, b, shm, st, g);
    break;
  case 38:
    hipLaunchKernelGGL((k_zsolve3_grp<8, 8, 1, 1, 1024, false, 1, true>), gr, b, shm, st, g);
    break;
  case 39:
    hipLaunchKernelGGL((k_zsolve3_grp<8, 8, 1, 1, 512, true, 1, true>), gr, b, shm, st, g);
    break;
  case 40:
    hipLaunchKernelGGL((k_zsolve3_grp<16, 16, 1, 1, 512, false, 1, true>), gr, b, shm, st, g);
    break;
#undef PF_G
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_zsolve<double>(int, int, int, double *, size_t, const double *, const double *,
                                          const double *, const double *, const double *, int,
                                          hipStream_t, bool);
template hipError_t launch_zsolve<float>(int, int, int, float *, size_t, const double *, const double *,
                                         const double *, const double *, const double *, int,
                                         hipStream_t, bool);

// ----------------------------------------------------------- zero mode
// The (0,0) slot of the transformed problem is the plane-mean profile of p.
// Plane means come from the float64 line sums, one workgroup per plane with
// a fixed-order tree reduction (bitwise reproducible).
__device__ __forceinline__ void plane_means_body(const double *__restrict__ sums, double *__restrict__ mean,
                                                 int ny, double inv_nxny, int k) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const double *s = sums + (size_t)k * ny;
  double a = 0.0;
  for (int j = tid; j < ny; j += 256) a += s[j];
  red[tid] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) mean[k] = red[0] * inv_nxny;
}
__global__ __launch_bounds__(256) void k_plane_means(const double *__restrict__ sums,
                                                     double *__restrict__ mean, int ny,
                                                     double inv_nxny) {
  plane_means_body(sums, mean, ny, inv_nxny, blockIdx.x);
}

// One thread: projection of the plane means fbar onto the range of L_z (zero
// dzf-weighted mean), the singular Neumann system solved with its last
// equation replaced by m[nz-1] = 0, then the shift to zero dzf-weighted mean.
// With p0mean (the iterate's plane means) it writes zm = m - p0mean instead.
__device__ __forceinline__ void zero_solve_body(const double *__restrict__ fbar, const double *__restrict__ dzf,
                                                const double *__restrict__ zal, const double *__restrict__ zga,
                                                double *__restrict__ m, int nz) {
  extern __shared__ double sh[];  // F, W, A, G, Y, RT: nz each
  double *F = sh, *W = sh + nz, *A = sh + 2 * nz, *G = sh + 3 * nz, *Y = sh + 4 * nz,
         *RT = sh + 5 * nz;
  for (int k = threadIdx.x; k < nz; k += blockDim.x) {
    F[k] = fbar[k];
    W[k] = dzf[k];
    A[k] = zal[k];
    G[k] = zga[k];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double wr = 0.0, w = 0.0;
  for (int k = 0; k < nz; ++k) { wr += W[k] * F[k]; w += W[k]; }
  const double c = wr / w;
  // rows 0..nz-2 of -L_z x = -(fbar - c), x[nz-1] = 0 (row nz-2 keeps its
  // gamma on the diagonal). No row has an excess, so the pivot of row k is
  // gamma_k + g_k with g_0 = 0 and g_k = alpha_k g_{k-1} / pivot_{k-1}.
  // pivots first (a chain of reciprocals only), then the right-hand side
  double g = 0.0, rp = 0.0;
  for (int k = 0; k < nz - 1; ++k) {
    g = A[k] * g * rp;
    rp = 1.0 / (G[k] + g);
    RT[k] = rp;
  }
  double y = 0.0;
  for (int k = 0; k < nz - 1; ++k) {
    y = (-(F[k] - c) + A[k] * y) * RT[k];
    Y[k] = y;
    RT[k] = G[k] * RT[k];
  }
  double x = 0.0, wm = 0.0;
  Y[nz - 1] = 0.0;
  for (int k = nz - 2; k >= 0; --k) {
    x = Y[k] + (k == nz - 2 ? 0.0 : RT[k] * x);
    Y[k] = x;
    wm += W[k] * x;
  }
  const double shift = wm / w;
  for (int k = 0; k < nz; ++k) m[k] = Y[k] - shift;
}
__global__ __launch_bounds__(256) void k_zero_solve(const double *__restrict__ fbar,
                                                    const double *__restrict__ dzf,
                                                    const double *__restrict__ zal,
                                                    const double *__restrict__ zga,
                                                    double *__restrict__ m, int nz) {
  zero_solve_body(fbar, dzf, zal, zga, m, nz);
}

__global__ __launch_bounds__(256) void k_sub(const double *__restrict__ a,
                                             const double *__restrict__ b, double *__restrict__ out,
                                             int n) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < n) out[k] = a[k] - b[k];
}

// grouped: blockIdx.y (means) or blockIdx.x (solve, difference) is the job
__global__ __launch_bounds__(256) void k_plane_means_grp(const GJobs g) {
  const GJob &J = g.j[blockIdx.y];
  if ((int)blockIdx.x >= J.nz) return;  // uniform per block
  plane_means_body(J.sums, static_cast<double *>(J.out), J.ny, 1.0 / ((double)J.nx * J.ny), blockIdx.x);
}
__global__ __launch_bounds__(256) void k_zero_solve_grp(const GJobs g) {
  const GJob &J = g.j[blockIdx.x];
  zero_solve_body(static_cast<const double *>(J.out), J.aux, J.zal, J.zga,
                  const_cast<double *>(static_cast<const double *>(J.in2)), J.nz);
}
__global__ __launch_bounds__(256) void k_sub_grp(const GJobs g) {
  const GJob &J = g.j[blockIdx.y];
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < J.nz)
    const_cast<double *>(J.zm)[k] = static_cast<const double *>(J.in2)[k] - static_cast<const double *>(J.out)[k];
}
hipError_t launch_zero_mode_grp(GJobs &g, hipStream_t st) {
  if (g.count < 1 || g.count > kMaxGroupJobs) return hipErrorInvalidValue;
  int mz = 1;
  for (int k = 0; k < g.count; ++k) mz = g.j[k].nz > mz ? g.j[k].nz : mz;
  hipLaunchKernelGGL(k_plane_means_grp, dim3(mz, g.count), dim3(256), 0, st, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_solve_grp, dim3(g.count), dim3(256), (size_t)6 * mz * sizeof(double), st, g);
  return hipGetLastError();
}
hipError_t launch_zero_shift_grp(GJobs &g, hipStream_t st) {
  if (g.count < 1 || g.count > kMaxGroupJobs) return hipErrorInvalidValue;
  int mz = 1;
  for (int k = 0; k < g.count; ++k) mz = g.j[k].nz > mz ? g.j[k].nz : mz;
  hipLaunchKernelGGL(k_plane_means_grp, dim3(mz, g.count), dim3(256), 0, st, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sub_grp, dim3((mz + 255) / 256, g.count), dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_zero_mode(int nx, int ny, int nz, const double *sums, const double *dzf,
                            const double *zal, const double *zga, double *fbar, double *m,
                            hipStream_t st) {
  const double inv = 1.0 / ((double)nx * (double)ny);
  hipLaunchKernelGGL(k_plane_means, dim3(nz), dim3(256), 0, st, sums, fbar, ny, inv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_solve, dim3(1), dim3(256), (size_t)6 * nz * sizeof(double), st, fbar,
                     dzf, zal, zga, m, nz);
  return hipGetLastError();
}

// zm = m - (plane means of the iterate p0), from its float64 line sums;
// p0mean is scratch of nz doubles.
hipError_t launch_zero_shift(int nx, int ny, int nz, const double *sums_p0, const double *m,
                             double *p0mean, double *zm, hipStream_t st) {
  const double inv = 1.0 / ((double)nx * (double)ny);
  hipLaunchKernelGGL(k_plane_means, dim3(nz), dim3(256), 0, st, sums_p0, p0mean, ny, inv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sub, dim3((nz + 255) / 256), dim3(256), 0, st, m, p0mean, zm, nz);
  return hipGetLastError();
}

// ------------------------------------------------------- Helmholtz apply
// Algorithm 2, Steps 2-4, with the Step 1 coefficients of pcr_prepare. One
// wave (64 consecutive columns) per chunk of M rows, so every coefficient
// address is uniform across the wave. Columns are padded to P*M rows with
// identity rows (see the Poisson z solve). The reduced 2P-row system is the
// same for all columns, so its eliminations are precomputed and only the
// right-hand sides cross LDS.
// Read-only tables through the constant address space: wave-uniform reads of
// them stay scalar loads even after the kernel has stored to LDS.
template <typename T>
using cptr = const T __attribute__((address_space(4))) *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const void *p) {
  return (cptr<T>)p;
}

// The rows of a Step 1 table that a lane's chunk uses, from row r0 on. With
// 64-column chunks r0 is wave-uniform and the tables are read through the
// constant address space as scalar loads (GRow); narrower chunks put two or
// four chunks in a wave, and their tables are read from a copy in LDS
// (LRow): per-lane vector loads of the tables in global memory spilled the
// 32-row shapes, and wave-uniform loads of every chunk of the wave with a
// per-lane select ran out of scalar registers.
template <typename T>
struct GRow {
  cptr<T> t;
  int r0;
  __device__ __forceinline__ T operator[](int q) const { return t[r0 + q]; }
};
// The rows of a global table for the CPW chunks that share a wave: one
// wave-uniform scalar load per chunk and a per-lane select (the sweeps that
// use it are fenced, so the scalar loads are not all issued at once).
template <typename T, int CPW>
struct SRow {
  cptr<T> t;
  int base[CPW];  // first row of each chunk of the wave (uniform)
  int slot;       // the lane's chunk within the wave
  __device__ __forceinline__ T operator[](int q) const {
    T v = t[base[0] + q];
#pragma unroll
    for (int k = 1; k < CPW; ++k) {
      const T o = t[base[k] + q];
      v = slot == k ? o : v;
    }
    return v;
  }
};
template <typename T>
struct LRow {
  const T *t;
  int r0;
  __device__ __forceinline__ T operator[](int q) const { return t[r0 + q]; }
};

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Steps 2-4 on the M rows d of one chunk. Step 3 is a twisted elimination:
// after one barrier every wave reads the 2P reduced right-hand sides of its
// columns and sweeps from the top down to its first reduced row and from the
// bottom up to its last, with the plan's multipliers; the two sweeps meet at
// the chunk's rows. With NBR it also returns the end values of the
// neighbouring chunks, x[2w-1] and x[2w+2] (0 past the walls), by extending
// its sweeps two rows. Those must equal bitwise what the neighbouring waves
// compute for their own rows (the residual has to see the values that are
// stored), so every sweep step is an explicit fused multiply-add: each
// y[r] and z[r] is then the same chain of roundings in every wave. RD holds
// 2P rows of CW values and is written once per call.
template <typename TC, int M, bool NBR, typename RW, typename CP>
__device__ __forceinline__ void helm_solve_regs(TC (&d)[M], RW fa, RW bg, RW ib, RW ra, RW rc, CP tf,
                                                CP tb, CP ti, int P, TC *RD, int w, int lane,
                                                bool active, int CW, TC &below, TC &above) {
  if (active) {
    // Step 2: forward and backward reduction of d
#pragma unroll
    for (int q = 2; q < M; ++q) {
      d[q] = d[q] + fa[q] * d[q - 1];
      sched_fence(q);
    }
#pragma unroll
    for (int q = M - 3; q >= 0; --q) {
      d[q] = d[q] + bg[q] * d[q + 1];
      sched_fence(q);
    }
    RD[(2 * w) * CW + lane] = d[0];
    RD[(2 * w + 1) * CW + lane] = d[M - 1];
  }
  __syncthreads();
  if (!active) return;
  // Step 3: forward sweep y[r] = D[r] + tf[r] y[r-1] down to row lo, backward
  // sweep z[r] = D[r] + tb[r] z[r+1] up to row hi = lo + 1
  const int nr = 2 * P, lo = 2 * w, hi = lo + 1;
  const TC *col = RD + lane;
  TC y = col[0], y1 = TC(0), y2 = TC(0);
#pragma unroll 8
  for (int r = 1; r <= lo; ++r) {
    y2 = y1;
    y1 = y;
    y = fmad(tf[r], y, col[r * CW]);
  }
  TC z = col[(nr - 1) * CW], z1 = TC(0), z2 = TC(0);
  const int nb = nr - 1 - hi;  // rows nr-2 down to hi
#pragma unroll 8
  for (int k = 0; k < nb; ++k) {
    const int r = nr - 2 - k;
    z2 = z1;
    z1 = z;
    z = fmad(tb[r], z, col[r * CW]);
  }
  // x[lo] = (y[lo] + tb z[hi]) ti[lo], x[hi] = (z[hi] + tf y[lo]) ti[hi]
  const TC x0 = fmad(tb[lo], z, y) * ti[lo];
  const TC xl = fmad(tf[hi], y, z) * ti[hi];
  if constexpr (NBR) {
    below = TC(0);
    above = TC(0);
    if (lo > 0) {  // extend the backward sweep by rows lo and lo-1
      const TC zl = fmad(tb[lo], z, col[lo * CW]);
      const TC zm = fmad(tb[lo - 1], zl, col[(lo - 1) * CW]);
      below = fmad(tf[lo - 1], y2, zm) * ti[lo - 1];
    }
    if (hi < nr - 1) {  // extend the forward sweep by rows hi and hi+1
      const TC yh = fmad(tf[hi], y, col[hi * CW]);
      const TC yp = fmad(tf[hi + 1], yh, col[(hi + 1) * CW]);
      above = fmad(tb[hi + 1], z2, yp) * ti[hi + 1];
    }
  }
  // Step 4: rebuild the interior in place
#pragma unroll
  for (int q = 1; q < M - 1; ++q) {
    d[q] = (d[q] + ra[q] * x0 + rc[q] * xl) * ib[q];
    sched_fence(q);
  }
  d[0] = x0;
  d[M - 1] = xl;
}

struct HelmArgs {
  HelmJob job[kMaxHelmJobs];
  int count;
};

// TS = TC = double (float64), TS = TC = float (float32 storage), or TS =
// double, TC = float with REFINE: a float32 solve, the float64 residual
// r - (I - s L_z) u in registers, a float32 solve for the correction.
// CW columns per chunk: 64 (one wave per chunk, wave-uniform coefficient
// addresses), 32 or 16 (two or four chunks per wave: smaller workgroups, so
// that several fit on a compute unit).
// Steps 2-4 for the chunk of one lane (see k_helm), with the Step 1 rows
// from RW sources (GRow or LRow) and the reduced system's multipliers from
// constant memory.
// Hides a per-lane column pointer from common-subexpression elimination:
// with chunks narrower than a wave the row addresses are per-lane 64-bit
// values, and keeping all of them from the loads to the stores of a sweep
// took as many registers as the column itself; they are recomputed instead.
template <typename TS>
__device__ __forceinline__ TS *fresh(TS *p) {
  uintptr_t a = reinterpret_cast<uintptr_t>(p);
  asm volatile("" : "+v"(a));
  return reinterpret_cast<TS *>(a);
}

// Rows of the float64 right-hand side that the refinement of a 32-row chunk
// narrower than a wave parks in LDS (the rest stay in registers): all 32 in
// registers spill, and reading them again from global memory doubled the
// HBM reads (the caches did not keep them). To make room, such a launch
// keeps one reduced-row array for both solves and reads the float64
// M-matrix rows from global memory.
template <int M, int CW>
constexpr int helm_parked_rows() { return CW < 64 && M > 16 ? 16 : 0; }

template <typename TS, typename TC, int M, bool REFINE, int CW, typename RW, typename DW>
__device__ __forceinline__ void helm_column(TS *cp, size_t plane, int r0, int n, RW fa, RW bg,
                                            RW ibv, RW ra, RW rc, DW mal, DW mga, DW mdg,
                                            cptr<TC> tf, cptr<TC> tb, cptr<TC> ti, int P, TC *RD,
                                            int w, int lane, bool active, double *park, TC *RD2) {
  TC below, above;
  if constexpr (!REFINE) {
    TC d[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      d[q] = (active && r0 + q < n) ? (TC)cp[(size_t)q * plane] : TC(0);
      if constexpr (CW < 64) sched_fence(q);
    }
    helm_solve_regs<TC, M, false>(d, fa, bg, ibv, ra, rc, tf, tb, ti, P, RD, w, lane, active, CW,
                                  below, above);
    if constexpr (CW < 64) cp = fresh(cp);
    if (active) {
#pragma unroll
      for (int q = 0; q < M; ++q) {
        if (r0 + q < n) cp[(size_t)q * plane] = (TS)d[q];
        if constexpr (CW < 64) sched_fence(q);
      }
    }
  } else {
    // The float64 right-hand side is held for the residual: in registers,
    // except KL rows parked in LDS (one slot per thread and row) when the
    // chunk is 32 rows and narrower than a wave
    constexpr int KL = helm_parked_rows<M, CW>();
    double r[M - KL];
    TC u[M], dd[M];
    const int tid = threadIdx.x, nt = blockDim.x;
    // every read of the column in flight before the first is used; then the
    // parked rows go to LDS
    double t[KL > 0 ? KL : 1];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const double v = (active && r0 + q < n) ? (double)cp[(size_t)q * plane] : 0.0;
      if (q < KL) t[q < KL ? q : 0] = v;
      else r[q < KL ? 0 : q - KL] = v;
    }
#pragma unroll
    for (int q = 0; q < KL; ++q) {
      park[q * nt + tid] = t[q];
      u[q] = (TC)t[q];
    }
#pragma unroll
    for (int q = KL; q < M; ++q) u[q] = (TC)r[q - KL];
    if constexpr (KL > 0) cp = fresh(cp);
    // the first solve also gives the neighbours across the chunk ends
    helm_solve_regs<TC, M, true>(u, fa, bg, ibv, ra, rc, tf, tb, ti, P, RD, w, lane, active, CW,
                                 below, above);
    if (active) {
#pragma unroll
      for (int q = 0; q < M; ++q) {
        const double al = mal[q], ga = mga[q], dg = mdg[q];
        const double um = q == 0 ? (double)below : (double)u[q == 0 ? 0 : q - 1];
        const double up = q == M - 1 ? (double)above : (double)u[q == M - 1 ? q : q + 1];
        const double rq = q < KL ? park[q * nt + tid] : r[q < KL ? 0 : q - KL];
        dd[q] = (TC)(rq - (dg * (double)u[q] - al * um - ga * up));
        if constexpr (KL > 0) {
          // row by row: left to itself the compiler reads every table row
          // of the loop first and spills them
          asm volatile("" : "+v"(dd[q]));
          sched_fence(q);
        }
      }
    }
    if (RD2 == RD) __syncthreads();  // every wave is done reading the first solve's rows
    helm_solve_regs<TC, M, false>(dd, fa, bg, ibv, ra, rc, tf, tb, ti, P, RD2, w, lane,
                                  active, CW, below, above);
    if constexpr (CW < 64) cp = fresh(cp);
    if (active) {
#pragma unroll
      for (int q = 0; q < M; ++q) {
        if (r0 + q < n) cp[(size_t)q * plane] = (TS)((double)u[q] + (double)dd[q]);
        if constexpr (CW < 64) sched_fence(q);
      }
    }
  }
}

// TS = TC = double (float64), TS = TC = float (float32 storage), or TS =
// double, TC = float with REFINE: a float32 solve, the float64 residual
// r - (I - s L_z) u in registers, a float32 solve for the correction.
// CW columns per chunk: 64 (one wave per chunk, wave-uniform coefficient
// addresses), 32 or 16 (two or four chunks per wave, so that a column of 32
// chunks fits a workgroup; the Step 1 tables are then copied to LDS after
// the reduced rows: 5 P M values of TC, and for REFINE 3 P M float64 rows).
template <typename TS, typename TC, int M, int CW, bool REFINE>
__global__ __launch_bounds__(1024) void k_helm(HelmArgs args) {
  extern __shared__ double shd[];
  const HelmJob &J = args.job[blockIdx.y];
  const HelmCoef &C = J.c;
  const int nib = J.nx / CW;
  const long nblk = (long)nib * J.ny;
  if ((long)blockIdx.x >= nblk) return;  // uniform per block
  // the 2P reduced rows of each solve (two solves with REFINE)
  TC *RD = reinterpret_cast<TC *>(shd);
  const int w = CW == 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / 64) : threadIdx.x / CW;
  const int lane = threadIdx.x % CW;
  const bool active = w < C.P;
  // narrow chunks (the long columns): every XCD walks a contiguous range of
  // column blocks (2048x1024x1024, three components: float64 27.4 -> 24.1 ms,
  // FP32+refine 34.9 -> 31.2 ms; the 64-column shapes lost up to 8 %). Only
  // when the launch has no spare blocks beyond this job's count.
  const unsigned bk = CW < 64 && gridDim.x == nblk ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int ib = bk % nib;
  const int j = bk / nib;
  const int r0 = active ? w * M : 0;
  const size_t plane = (size_t)J.nx * J.ny;
  TS *cp = reinterpret_cast<TS *>(J.field) + (size_t)j * J.nx + ib * CW + lane + (size_t)r0 * plane;
  const cptr<TC> tf = as_const<TC>(C.tf), tb = as_const<TC>(C.tb), ti = as_const<TC>(C.ti);
  if constexpr (CW == 64) {
    using R = GRow<TC>;
    using D = GRow<double>;
    helm_column<TS, TC, M, REFINE, CW>(
        cp, plane, r0, C.n, R{as_const<TC>(C.fa), r0}, R{as_const<TC>(C.bg), r0},
        R{as_const<TC>(C.ib), r0}, R{as_const<TC>(C.ra), r0}, R{as_const<TC>(C.rc), r0},
        D{as_const<double>(C.al), r0}, D{as_const<double>(C.ga), r0}, D{as_const<double>(C.dg), r0},
        tf, tb, ti, C.P, RD, w, lane, active, nullptr, RD + 2 * C.P * CW);
  } else {
    const int npad = C.P * M;
    constexpr bool kPark = REFINE && helm_parked_rows<M, CW>() > 0;
    if constexpr (kPark) {
      // one reduced-row array, then the five Step 1 tables, then the parked
      // rows of the right-hand side
      TC *T0 = RD + 2 * C.P * CW;
      TC *fa = T0, *bg = T0 + npad, *ibv = T0 + 2 * npad, *ra = T0 + 3 * npad, *rc = T0 + 4 * npad;
      // 8-byte aligned: 2 P CW and 5 P M float32 values are even counts;
      // plain pointer arithmetic from the LDS array keeps the stores in LDS
      // address space (through an integer the compiler lost it and used
      // flat stores with 64-bit addresses)
      double *park = reinterpret_cast<double *>(rc + npad);
      {
        const TC *sfa = (const TC *)C.fa, *sbg = (const TC *)C.bg, *sib = (const TC *)C.ib;
        const TC *sra = (const TC *)C.ra, *src = (const TC *)C.rc;
        for (int r = threadIdx.x; r < npad; r += blockDim.x) {
          fa[r] = sfa[r]; bg[r] = sbg[r]; ibv[r] = sib[r]; ra[r] = sra[r]; rc[r] = src[r];
        }
      }
      __syncthreads();
      using R = LRow<TC>;
      constexpr int CPW = 64 / CW;
      using D = SRow<double, CPW>;
      const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
      D dal{as_const<double>(C.al), {}, (int)(threadIdx.x % 64) / CW};
#pragma unroll
      for (int k = 0; k < CPW; ++k) dal.base[k] = (wave * CPW + k < C.P ? wave * CPW + k : 0) * M;
      D dga = dal, ddg = dal;
      dga.t = as_const<double>(C.ga);
      ddg.t = as_const<double>(C.dg);
      helm_column<TS, TC, M, REFINE, CW>(cp, plane, r0, C.n, R{fa, r0}, R{bg, r0}, R{ibv, r0},
                                         R{ra, r0}, R{rc, r0}, dal, dga, ddg, tf, tb, ti, C.P, RD, w,
                                         lane, active, park, RD);
    } else {
      double *D0 = shd + 2 * C.P * CW;  // past the reduced rows
      double *mal = D0, *mga = D0 + npad, *mdg = D0 + 2 * npad;
      TC *T0 = reinterpret_cast<TC *>(REFINE ? D0 + 3 * npad : D0);
      TC *fa = T0, *bg = T0 + npad, *ibv = T0 + 2 * npad, *ra = T0 + 3 * npad, *rc = T0 + 4 * npad;
      {
        const TC *sfa = (const TC *)C.fa, *sbg = (const TC *)C.bg, *sib = (const TC *)C.ib;
        const TC *sra = (const TC *)C.ra, *src = (const TC *)C.rc;
        for (int r = threadIdx.x; r < npad; r += blockDim.x) {
          fa[r] = sfa[r]; bg[r] = sbg[r]; ibv[r] = sib[r]; ra[r] = sra[r]; rc[r] = src[r];
          if (REFINE) { mal[r] = C.al[r]; mga[r] = C.ga[r]; mdg[r] = C.dg[r]; }
        }
      }
      __syncthreads();
      using R = LRow<TC>;
      using D = LRow<double>;
      helm_column<TS, TC, M, REFINE, CW>(cp, plane, r0, C.n, R{fa, r0}, R{bg, r0}, R{ibv, r0},
                                         R{ra, r0}, R{rc, r0}, D{mal, r0}, D{mga, r0}, D{mdg, r0},
                                         tf, tb, ti, C.P, RD, w, lane, active, nullptr,
                                         RD + 2 * C.P * CW);
    }
  }
}

// Same algorithm, coefficient tables staged in LDS. A persistent workgroup
// (CW columns per chunk, any CW) copies its job's Step 1 tables into LDS once
// and then walks column blocks; chunks that share a wave read their
// different coefficient rows from LDS instead of global memory, so CW = 32
// gives 512-thread workgroups that keep more than one resident per compute
// unit and overlap one block's loads with another's elimination.
template <typename TC, int M>
__device__ __forceinline__ void helm_solve_lds(TC (&d)[M], TC &x0, TC &xl, int r0, const TC *fa,
                                               const TC *bg, const TC *ib, const TC *ra,
                                               const TC *rc, const TC *k1, const TC *k2,
                                               const TC *invd, int P, int steps, TC *RD, int w,
                                               int lane, bool active, int CW) {
  if (active) {
#pragma unroll
    for (int q = 2; q < M; ++q) d[q] = d[q] + fa[r0 + q] * d[q - 1];
#pragma unroll
    for (int q = M - 3; q >= 0; --q) d[q] = d[q] + bg[r0 + q] * d[q + 1];
  }
  const int nr = 2 * P;
  x0 = d[0];
  xl = d[M - 1];
  for (int st = 0; st < steps; ++st) {
    const int s = 1 << st;
    if (active) {
      RD[(2 * w) * CW + lane] = x0;
      RD[(2 * w + 1) * CW + lane] = xl;
    }
    __syncthreads();
    if (active) {
      const int ra0 = 2 * w, ra1 = 2 * w + 1;
      TC n0 = x0, n1 = xl;
      if (ra0 - s >= 0) n0 += k1[st * nr + ra0] * RD[(ra0 - s) * CW + lane];
      if (ra0 + s < nr) n0 += k2[st * nr + ra0] * RD[(ra0 + s) * CW + lane];
      if (ra1 - s >= 0) n1 += k1[st * nr + ra1] * RD[(ra1 - s) * CW + lane];
      if (ra1 + s < nr) n1 += k2[st * nr + ra1] * RD[(ra1 + s) * CW + lane];
      x0 = n0;
      xl = n1;
    }
    __syncthreads();
  }
  if (active) {
    x0 = x0 * invd[2 * w];
    xl = xl * invd[2 * w + 1];
#pragma unroll
    for (int q = 1; q < M - 1; ++q) d[q] = (d[q] + ra[r0 + q] * x0 + rc[r0 + q] * xl) * ib[r0 + q];
    d[0] = x0;
    d[M - 1] = xl;
  }
}

template <typename TS, typename TC, int M, int CW, bool REFINE>
__global__ __launch_bounds__(512, 4) void k_helm_lds(HelmArgs args) {
  extern __shared__ double shd[];
  const HelmJob &J = args.job[blockIdx.y];
  const HelmCoef &C = J.c;
  const int P = C.P, steps = C.steps, nr = 2 * P, npad = P * M;
  // LDS layout (in TC units unless noted): fa bg ib ra rc [npad each],
  // k1 k2 [steps*nr], invd [nr], RD [nr*CW]; then float64: al ga ep [npad]
  // (refinement only), NB [nr*CW]
  TC *L = reinterpret_cast<TC *>(shd);
  TC *fa = L, *bg = fa + npad, *ibv = bg + npad, *ra = ibv + npad, *rc = ra + npad;
  TC *k1 = rc + npad, *k2 = k1 + steps * nr, *invd = k2 + steps * nr, *RD = invd + nr;
  double *D = reinterpret_cast<double *>(
      (reinterpret_cast<uintptr_t>(RD + nr * CW) + 7) & ~uintptr_t(7));
  double *mal = D, *mga = D + npad, *mdg = D + 2 * npad, *NB = D + 3 * npad;
  {
    const TC *sfa = (const TC *)C.fa, *sbg = (const TC *)C.bg, *sib = (const TC *)C.ib;
    const TC *sra = (const TC *)C.ra, *src = (const TC *)C.rc;
    for (int r = threadIdx.x; r < npad; r += blockDim.x) {
      fa[r] = sfa[r]; bg[r] = sbg[r]; ibv[r] = sib[r]; ra[r] = sra[r]; rc[r] = src[r];
      if (REFINE) { mal[r] = C.al[r]; mga[r] = C.ga[r]; mdg[r] = C.dg[r]; }
    }
    const TC *sk1 = (const TC *)C.k1, *sk2 = (const TC *)C.k2, *sinv = (const TC *)C.invd;
    for (int r = threadIdx.x; r < steps * nr; r += blockDim.x) { k1[r] = sk1[r]; k2[r] = sk2[r]; }
    for (int r = threadIdx.x; r < nr; r += blockDim.x) invd[r] = sinv[r];
  }
  __syncthreads();
  const int w = threadIdx.x / CW;
  const int lane = threadIdx.x % CW;
  const bool active = w < P;
  const int n = C.n;
  const int r0 = active ? w * M : 0;
  const int nib = J.nx / CW;
  const long nblk = (long)nib * J.ny;
  const size_t plane = (size_t)J.nx * J.ny;
  for (long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {   // uniform per block
    const int ibk = (int)(blk % nib);
    const long j = blk / nib;
    TS *cp = reinterpret_cast<TS *>(J.field) + (size_t)j * J.nx + (size_t)ibk * CW + lane +
             (size_t)r0 * plane;
    TC x0, xl;
    if constexpr (!REFINE) {
      TC d[M];
#pragma unroll
      for (int q = 0; q < M; ++q) d[q] = (active && r0 + q < n) ? (TC)cp[(size_t)q * plane] : TC(0);
      helm_solve_lds<TC, M>(d, x0, xl, r0, fa, bg, ibv, ra, rc, k1, k2, invd, P, steps, RD, w,
                            lane, active, CW);
      if (active) {
#pragma unroll
        for (int q = 0; q < M; ++q)
          if (r0 + q < n) cp[(size_t)q * plane] = (TS)d[q];
      }
    } else {
      double r[M];
      TC u[M], dd[M];
#pragma unroll
      for (int q = 0; q < M; ++q) {
        r[q] = (active && r0 + q < n) ? (double)cp[(size_t)q * plane] : 0.0;
        u[q] = (TC)r[q];
      }
      helm_solve_lds<TC, M>(u, x0, xl, r0, fa, bg, ibv, ra, rc, k1, k2, invd, P, steps, RD, w,
                            lane, active, CW);
      if (active) {
        NB[(2 * w) * CW + lane] = (double)u[0];
        NB[(2 * w + 1) * CW + lane] = (double)u[M - 1];
      }
      __syncthreads();
      double below = 0.0, above = 0.0;
      if (active) {
        if (w > 0) below = NB[(2 * w - 1) * CW + lane];
        if (w < P - 1) above = NB[(2 * w + 2) * CW + lane];
      }
      __syncthreads();
      if (active) {
#pragma unroll
        for (int q = 0; q < M; ++q) {
          const double al = mal[r0 + q], ga = mga[r0 + q], dg = mdg[r0 + q];
          const double um = q == 0 ? below : (double)u[q == 0 ? 0 : q - 1];
          const double up = q == M - 1 ? above : (double)u[q == M - 1 ? q : q + 1];
          dd[q] = (TC)(r[q] - (dg * (double)u[q] - al * um - ga * up));
        }
      }
      helm_solve_lds<TC, M>(dd, x0, xl, r0, fa, bg, ibv, ra, rc, k1, k2, invd, P, steps, RD, w,
                            lane, active, CW);
      if (active) {
#pragma unroll
        for (int q = 0; q < M; ++q)
          if (r0 + q < n) cp[(size_t)q * plane] = (TS)((double)u[q] + (double)dd[q]);
      }
    }
  }
}

size_t helm_lds_bytes(int precision, int M, int P, int steps, int CW) {
  const size_t tc = precision == 0 ? 8 : 4;
  const size_t npad = (size_t)P * M, nr = 2 * (size_t)P;
  size_t b = tc * (5 * npad + 2 * steps * nr + nr + nr * CW);
  b = (b + 7) & ~size_t(7);
  b += 8 * (3 * npad + nr * CW);
  return b;
}

int helm_default_cw(int P) { return P <= 16 ? 64 : 32; }

hipError_t launch_helm(int precision, int chunk_rows, int cw, bool staged, int count,
                       const HelmJob *jobs, hipStream_t st) {
  if (count < 1 || count > kMaxHelmJobs) return hipErrorInvalidValue;
  HelmArgs a;
  a.count = count;
  int maxP = 0;
  for (int t = 0; t < count; ++t) maxP = jobs[t].c.P > maxP ? jobs[t].c.P : maxP;
  const int CW = cw;
  if (maxP < 1 || maxP * CW > 1024 || (CW != 16 && CW != 32 && CW != 64)) return hipErrorInvalidValue;
  long maxblk = 0;
  for (int t = 0; t < count; ++t) {
    a.job[t] = jobs[t];
    if (jobs[t].nx % CW) return hipErrorInvalidValue;
    const long nb = (long)(jobs[t].nx / CW) * jobs[t].ny;
    if (nb > maxblk) maxblk = nb;
  }
  if (staged) {
    if (maxP * CW > 512) return hipErrorInvalidValue;
    int maxsteps = 0;
    for (int t = 0; t < count; ++t) maxsteps = jobs[t].c.steps > maxsteps ? jobs[t].c.steps : maxsteps;
    const size_t shm = helm_lds_bytes(precision, chunk_rows, maxP, maxsteps, CW);
    if (shm > 160 * 1024) return hipErrorInvalidValue;
    // persistent: a few workgroups per compute unit walk the column blocks
    const long gx = maxblk < 2048 ? maxblk : 2048;
    dim3 g((unsigned)gx, (unsigned)count), b(CW * maxP);
#define PF_HELMS_CW(M, CWV)                                                                      \
  if (precision == 0)                                                                            \
    hipLaunchKernelGGL((k_helm_lds<double, double, M, CWV, false>), g, b, shm, st, a);           \
  else if (precision == 1)                                                                       \
    hipLaunchKernelGGL((k_helm_lds<float, float, M, CWV, false>), g, b, shm, st, a);             \
  else                                                                                           \
    hipLaunchKernelGGL((k_helm_lds<double, float, M, CWV, true>), g, b, shm, st, a);
#define PF_HELMS(M)                   \
  case M:                             \
    if (CW == 64) {                   \
      PF_HELMS_CW(M, 64)              \
    } else if (CW == 32) {            \
      PF_HELMS_CW(M, 32)              \
    } else {                          \
      PF_HELMS_CW(M, 16)              \
    }                                 \
    break;
    switch (chunk_rows) {
      PF_HELMS(8)
      PF_HELMS(16)
      PF_HELMS(32)
      default:
        return hipErrorInvalidValue;
    }
#undef PF_HELMS
#undef PF_HELMS_CW
    return hipGetLastError();
  }
  dim3 g((unsigned)maxblk, (unsigned)count), b(CW * maxP);
  // the reduced rows: one float64 array, or two float32 arrays (refinement);
  // chunks narrower than a wave add the Step 1 tables (see k_helm)
  size_t shm = (size_t)2 * maxP * CW * sizeof(double);
  if (CW < 64) {
    const size_t npad = (size_t)maxP * chunk_rows;
    if (precision == 2 && chunk_rows > 16) {
      // one float32 reduced-row array, the five float32 tables, 16 parked rows
      shm = (size_t)2 * maxP * CW * 4 + npad * 5 * 4;
      shm = ((shm + 7) & ~size_t(7)) + (size_t)16 * CW * maxP * 8;
    } else {
      shm += npad * (5 * (precision == 0 ? 8 : 4) + (precision == 2 ? 24 : 0));
    }
  }
  if (shm > 160 * 1024) return hipErrorInvalidValue;
#define PF_HELM_CW(M, CWV)                                                                      \
  if (precision == 0)                                                                           \
    hipLaunchKernelGGL((k_helm<double, double, M, CWV, false>), g, b, shm, st, a);              \
  else if (precision == 1)                                                                      \
    hipLaunchKernelGGL((k_helm<float, float, M, CWV, false>), g, b, shm, st, a);                \
  else                                                                                          \
    hipLaunchKernelGGL((k_helm<double, float, M, CWV, true>), g, b, shm, st, a);
#define PF_HELM(M)                    \
  case M:                             \
    if (CW == 64) {                   \
      PF_HELM_CW(M, 64)               \
    } else if (CW == 32) {            \
      PF_HELM_CW(M, 32)               \
    } else {                          \
      PF_HELM_CW(M, 16)               \
    }                                 \
    break;
  switch (chunk_rows) {
    PF_HELM(8)
    PF_HELM(16)
    PF_HELM(32)
    default:
      return hipErrorInvalidValue;
  }
#undef PF_HELM
#undef PF_HELM_CW
  return hipGetLastError();
}

// ------------------------------------------- Algorithm 2, Step 1 on the device
// The Step 1 coefficients of (I - s L_z) for every chunk, the reduced
// system's twisted-elimination multipliers and its cyclic-reduction
// multipliers, recomputed from the rows of -L_z and s by one workgroup, so
// that a new s (one per Runge-Kutta substep) needs no host work, no copy and
// no synchronisation. Rows in sign-normalised form: row r of I - s L_z is
// -A x[r-1] + (A + G + E) x[r] - G x[r+1] with A = s alpha, G = s gamma,
// E = 1 + s excess; the padding rows (alpha = gamma = excess = 0) are
// identity rows.
//
// Per chunk of m rows (one thread each), eliminating the interior onto the
// two end rows keeps every pivot as a sum of non-negative parts: the forward
// elimination's pivot b = G + a + ef (a the coupling to the chunk's first
// row, ef the carried excess), the backward pass's couplings a, c and excess
// eta. The reduced 2P rows couple chunk ends; they are factored from both
// ends (twisted elimination) and by cyclic reduction, each with the excess
// carried instead of a diagonal formed by subtraction.
constexpr int kPrepRows = 32 * 32;  // P * M at most
__global__ __launch_bounds__(64) void k_pcr_prepare(PcrPrep t, double s) {
  __shared__ double sb[kPrepRows], sa[kPrepRows], sc[kPrepRows], sef[kPrepRows], seta[kPrepRows];
  __shared__ double RA[64], RG[64], RE[64], fe[64], be[64];
  const int tid = threadIdx.x, P = t.P, m = t.M, nr = 2 * P, np = P * m;
  double *T0 = t.d[0], *T1 = t.d[1], *T2 = t.d[2], *T3 = t.d[3], *T4 = t.d[4];
  if (tid < P) {
    const int r0 = tid * m;
    double *b = sb + r0, *a = sa + r0, *c = sc + r0, *ef = sef + r0, *eta = seta + r0;
    auto A = [&](int i) { return s * t.al[r0 + i]; };
    auto G = [&](int i) { return s * t.ga[r0 + i]; };
    auto E = [&](int i) { return 1.0 + s * t.ex[r0 + i]; };
    a[1] = A(1);
    ef[1] = E(1);
    b[1] = G(1) + A(1) + E(1);
    for (int i = 2; i < m; ++i) {
      const double q = A(i) / b[i - 1];
      a[i] = q * a[i - 1];
      ef[i] = E(i) + q * ef[i - 1];
      b[i] = G(i) + a[i] + ef[i];
    }
    c[m - 2] = G(m - 2);
    eta[m - 2] = ef[m - 2];
    for (int i = m - 3; i >= 1; --i) {
      const double q = G(i) / b[i + 1];
      a[i] = a[i] + q * a[i + 1];
      c[i] = q * c[i + 1];
      eta[i] = ef[i] + q * eta[i + 1];
    }
    const double q0 = G(0) / b[1];
    RA[2 * tid] = A(0);
    RG[2 * tid] = q0 * c[1];
    RE[2 * tid] = E(0) + q0 * eta[1];
    RA[2 * tid + 1] = a[m - 1];
    RG[2 * tid + 1] = G(m - 1);
    RE[2 * tid + 1] = ef[m - 1];
    for (int i = 0; i < m; ++i) {
      T0[r0 + i] = i >= 2 ? A(i) / b[i - 1] : 0.0;
      T1[r0 + i] = i <= m - 3 ? G(i) / b[i + 1] : 0.0;
      const bool in = i >= 1 && i <= m - 2;
      T2[r0 + i] = in ? 1.0 / b[i] : 0.0;
      T3[r0 + i] = in ? a[i] : 0.0;
      T4[r0 + i] = in ? c[i] : 0.0;
    }
  }
  __syncthreads();
  // twisted elimination of the reduced rows: forward pivots G + fe,
  // backward pivots A + be, both sums of non-negative parts
  if (tid == 0) {
    fe[0] = RA[0] + RE[0];
    for (int r = 1; r < nr; ++r) fe[r] = RE[r] + RA[r] * fe[r - 1] / (RG[r - 1] + fe[r - 1]);
    be[nr - 1] = RG[nr - 1] + RE[nr - 1];
    for (int r = nr - 2; r >= 0; --r) be[r] = RE[r] + RG[r] * be[r + 1] / (RA[r + 1] + be[r + 1]);
  }
  __syncthreads();
  if (tid < nr) {
    const int r = tid;
    const double fp = r > 0 ? RG[r - 1] + fe[r - 1] : 1.0;
    const double bp = r < nr - 1 ? RA[r + 1] + be[r + 1] : 1.0;
    const double lo = r > 0 ? RA[r] * fe[r - 1] / fp : RA[r];
    const double hi = r < nr - 1 ? RG[r] * be[r + 1] / bp : RG[r];
    t.d[8][r] = r > 0 ? RA[r] / fp : 0.0;
    t.d[9][r] = r < nr - 1 ? RG[r] / bp : 0.0;
    t.d[10][r] = 1.0 / (RE[r] + lo + hi);
  }
  // cyclic reduction of the reduced rows: step st couples rows 2^st apart;
  // the new excess is the old one plus the eliminated neighbours' excesses
  for (int st = 0; st < t.steps; ++st) {
    const int h = 1 << st;
    double nA = 0.0, nG = 0.0, nE = 0.0;
    if (tid < nr) {
      const int r = tid;
      double k1 = 0.0, k2 = 0.0, em = 0.0, ep2 = 0.0, am = 0.0, gp = 0.0;
      if (r - h >= 0) {
        k1 = RA[r] / (RA[r - h] + RG[r - h] + RE[r - h]);
        am = RA[r - h];
        em = RE[r - h];
      }
      if (r + h < nr) {
        k2 = RG[r] / (RA[r + h] + RG[r + h] + RE[r + h]);
        gp = RG[r + h];
        ep2 = RE[r + h];
      }
      t.d[5][st * nr + r] = k1;
      t.d[6][st * nr + r] = k2;
      nA = k1 * am;
      nG = k2 * gp;
      nE = RE[r] + k1 * em + k2 * ep2;
    }
    __syncthreads();
    if (tid < nr) {
      RA[tid] = nA;
      RG[tid] = nG;
      RE[tid] = nE;
    }
    __syncthreads();
  }
  if (tid < nr) t.d[7][tid] = 1.0 / (RA[tid] + RG[tid] + RE[tid]);
  // the float32 copies and the M-matrix rows of the refinement's residual
  __syncthreads();
  const int len[11] = {np, np, np, np, np, t.steps * nr, t.steps * nr, nr, nr, nr, nr};
  for (int k = 0; k < 11; ++k)
    for (int i = tid; i < len[k]; i += 64) t.f[k][i] = (float)t.d[k][i];
  for (int r = tid; r < np; r += 64) {
    const double a = s * t.al[r], g = s * t.ga[r], e = 1.0 + s * t.ex[r];
    t.mA[r] = a;
    t.mG[r] = g;
    t.mE[r] = e;
    t.mD[r] = a + g + e;
  }
}

hipError_t launch_pcr_prepare(const PcrPrep &p, double s, hipStream_t st) {
  if (p.P < 1 || p.P > 32 || p.P * p.M > kPrepRows || p.M < 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pcr_prepare, dim3(1), dim3(64), 0, st, p, s);
  return hipGetLastError();
}

// dst[i] = src[i] + kappa: the x-slot shifts of a 3-D Helmholtz plan for a
// new s (kappa = 1/s)
__global__ __launch_bounds__(256) void k_shift_add(const double *__restrict__ src, double *__restrict__ dst,
                                                   int n, double kappa) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i] + kappa;
}

hipError_t launch_shift_add(const double *src, double *dst, int n, double kappa, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shift_add, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n, kappa);
  return hipGetLastError();
}

// ------------------------------------------------------------ plain copy
// The fastest copy measured on MI355X (4 GiB: 5.6 TB/s, against 4.9 TB/s for
// one 16-byte element per thread and grid stride): four 16-byte nontemporal
// loads in flight per thread over a 16 KiB block tile, 16384 workgroups
// striding over the tiles, then the tail one element per thread.
typedef unsigned int pf_v4u __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(const pf_v4u *__restrict__ src, pf_v4u *__restrict__ dst,
                                              size_t n) {
  constexpr int U = 4;
  constexpr size_t kTile = (size_t)256 * U;
  const size_t full = n / kTile * kTile;
  for (size_t b = (size_t)blockIdx.x * kTile; b < full; b += (size_t)gridDim.x * kTile) {
    pf_v4u v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + b + u * 256 + threadIdx.x);
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], dst + b + u * 256 + threadIdx.x);
  }
  for (size_t i = full + (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    dst[i] = src[i];
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  size_t blocks = (n + 1023) / 1024;
  if (blocks > 16384) blocks = 16384;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const pf_v4u *)src,
                     (pf_v4u *)dst, n);
  return hipGetLastError();
}

}  // namespace pf
