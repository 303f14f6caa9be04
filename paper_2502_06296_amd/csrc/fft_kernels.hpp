// The line-transform kernels of the x and y directions and the refinement
// residual, as templates over the transform length, the launch shape
// (threads per line TPL, lines per workgroup LPW) and the radix order RO
// (0: radix 16 first; 1: radix 8 at most): the default shapes are
// instantiated by kernels_fft.hip, the alternatives the autotuner times by
// kernels_fft_alt.hip.
#pragma once
#include "pf_internal.hpp"

namespace pf {

// pairs of storage values (two adjacent slots) as float64
template <typename T>
__device__ __forceinline__ cplx<double> ld2(const T *p) {
  const cplx<T> v = *reinterpret_cast<const cplx<T> *>(p);
  return mkc<double>((double)v.x, (double)v.y);
}
template <typename T>
__device__ __forceinline__ void st2(T *p, double x, double y) {
  *reinterpret_cast<cplx<T> *>(p) = mkc<T>((T)x, (T)y);
}

// ----------------------------------------------------------- x forward
// XW = 0: periodic x, the packed real layout (App. A).
// XW = 1 (2): zero-gradient (value-zero) walls at both x ends: the cosine
// (sine) transform of every line, X_q = 2 sum_i x_i cos(pi q (2i + 1) / 2N)
// (Y_q = 2 sum_i x_i sin(pi (q + 1) (2i + 1) / 2N)), one real coefficient
// per slot in natural order (slot q holds mode q). Computed as along y for y
// walls: the line pair a + ib in Makhoul's order (even positions ascending,
// odd descending; for the sine the odd positions negated) through one
// complex FFT, then X_q = c_q Z_q + conj(c_q) Z_{N-q} (c_q = ctw[q] =
// exp(-i pi q / 2N), Z_N = Z_0) gives the two lines' coefficients as its
// real and imaginary parts (the transform has real coefficients); the sine
// takes the cosine coefficient of index N-1-q as its mode q. Z_0 is the sum
// of each line, as in the periodic case.
__device__ __forceinline__ int xw_src(int n, int N) { return n < N / 2 ? 2 * n : 2 * N - 1 - 2 * n; }
// XW = 3: a field on the x faces between value-zero walls (line positions
// 0..NL-2 hold the faces 1..NL-1, position NL-1 the east wall face): the
// type-I sine transform X_q = 2 sum_m x_m sin(pi q m / NL), q = 1..NL-1, of
// both lines of a pair at once, as one complex FFT of length N = 2 NL of the
// oddly extended pair (e_m = x_m, e_{N-m} = -x_m, e_0 = e_NL = 0): X_q = i E_q,
// its real and imaginary parts the two lines' coefficients; slot q - 1 holds
// mode q and the last slot is zero.
template <int XW>
__device__ __forceinline__ cplx<double> xface_src(int i, int NL, const double *a, const double *b) {
  if (i == 0 || i == NL) return mkc<double>(0.0, 0.0);
  if (i < NL) return mkc<double>(a[i - 1], b[i - 1]);
  return mkc<double>(-a[2 * NL - 1 - i], -b[2 * NL - 1 - i]);
}
template <typename T, int N, int TPL, int LPW, bool SUMS, int XW, int RO = 0>
__device__ __forceinline__ void xfwd_body(const double *__restrict__ in, T *__restrict__ out,
                                                   const cplx<double> *__restrict__ tw,
                                                   const cplx<double> *__restrict__ ctw,
                                                   double *__restrict__ sums, long ncl, int ny,
                                                   size_t sp,
                                          unsigned bx_, unsigned gx_) {
  using C = cplx<double>;
  __shared__ C lds[LPW * lds_len(N)];
  static_assert(N % TPL == 0, "every thread takes N / TPL positions");
  const int tid = threadIdx.x, l = tid / TPL, t = tid % TPL;
  const long c = (long)bx_ * LPW + l;
  const bool ok = c < ncl;
  C *buf = lds + l * lds_len(N);
  constexpr int NL = XW == 3 ? N / 2 : N;  // line length
  // the first pass reads the line pair straight from global memory
  const double *a = in + (ok ? (size_t)(2 * c) * NL : 0);
  const double *b = a + NL;
  auto src = [&](int i) {
    if constexpr (XW == 0) {
      return ok ? mkc<double>(a[i], b[i]) : mkc<double>(0.0, 0.0);
    } else if constexpr (XW == 3) {
      return ok ? xface_src<XW>(i, NL, a, b) : mkc<double>(0.0, 0.0);
    } else {
      const int x = xw_src(i, N);
      const double sg = (XW == 2 && (x & 1)) ? -1.0 : 1.0;
      return ok ? mkc<double>(sg * a[x], sg * b[x]) : mkc<double>(0.0, 0.0);
    }
  };
  fft_line_io<double, N, TPL, false, true, false, RO>(buf, tw, t, src, [](int, const C &) {});
  if (!ok) return;
  T *oa = out + (size_t)(2 * c / ny) * sp + (size_t)(2 * c % ny) * NL;
  T *ob = oa + NL;
  if constexpr (XW == 3) {
#pragma unroll
    for (int q = t; q < N; q += TPL) {
      if (q >= 1 && q < NL) {
        const C v = buf[lds_idx(q)];
        oa[q - 1] = (T)(-v.y);
        ob[q - 1] = (T)v.x;
      } else if (q == NL) {
        oa[NL - 1] = (T)0.0;
        ob[NL - 1] = (T)0.0;
      }
      if (SUMS && q == 0) {  // no zero mode: the faces field has no mean mode
        sums[2 * c] = 0.0;
        sums[2 * c + 1] = 0.0;
      }
    }
    return;
  }
  if constexpr (XW != 0) {
#pragma unroll
    for (int q = t; q < N; q += TPL) {
      const C v1 = buf[lds_idx(q)], v2 = buf[lds_idx(q == 0 ? 0 : N - q)], cq = ctw[q];
      const int slot = XW == 2 ? N - 1 - q : q;
      oa[slot] = (T)(cq.x * v1.x - cq.y * v1.y + cq.x * v2.x + cq.y * v2.y);
      ob[slot] = (T)(cq.x * v1.y + cq.y * v1.x + cq.x * v2.y - cq.y * v2.x);
      if (SUMS && q == 0) {
        // the sum of each line (a sign-alternated sum for the sine, unused)
        sums[2 * c] = v1.x;
        sums[2 * c + 1] = v1.y;
      }
    }
    return;
  }
#pragma unroll
  for (int q = t; q < N / 2; q += TPL) {
    C A, B;
    if (q == 0) {
      const C z0 = buf[lds_idx(0)], zh = buf[lds_idx(N / 2)];
      A = mkc<double>(z0.x, zh.x);
      B = mkc<double>(z0.y, zh.y);
      // the float64 zero mode of each line is its sum (a tree of exact
      // unit-twiddle butterflies)
      if (SUMS) {
        sums[2 * c] = z0.x;
        sums[2 * c + 1] = z0.y;
      }
    } else {
      split_pair<double>(buf[lds_idx(q)], buf[lds_idx(N - q)], A, B);
    }
    *reinterpret_cast<cplx<T> *>(oa + 2 * q) = mkc<T>((T)A.x, (T)A.y);
    *reinterpret_cast<cplx<T> *>(ob + 2 * q) = mkc<T>((T)B.x, (T)B.y);
  }
}
template <typename T, int N, int TPL, int LPW, bool SUMS, int XW, int RO = 0>
__global__ __launch_bounds__(TPL *LPW) void k_xfwd(const double *__restrict__ in, T *__restrict__ out,
                                                   const cplx<double> *__restrict__ tw,
                                                   const cplx<double> *__restrict__ ctw,
                                                   double *__restrict__ sums, long ncl, int ny,
                                                   size_t sp) {
  xfwd_body<T, N, TPL, LPW, SUMS, XW, RO>(in, out, tw, ctw, sums, ncl, ny, sp, blockIdx.x, gridDim.x);
}

// ------------------------------ residual of the correction in x-spectral space
// The first float32 solution is kept as its x spectrum W (after the y
// inverse; W = ny X(p0), X the unnormalised x transform), so the correction's
// right-hand side is formed without going back to real space:
//   R = X(f) - nx fbar[k] e_0 - (1/ny) L7^ W,
//   L7^ W = -sx[s] W + (W[j-1] - 2 W + W[j+1]) / dy^2
//           + alpha_k W[k-1] + gamma_k W[k+1] - (alpha_k + gamma_k + eps_k) W,
// (eps_k = 0 for the pressure rows; the 3-D Helmholtz passes its wall excess,
// 1/s folded into sx, and fbar = 0),
// slot by slot of the packed layout: the periodic x second difference is
// -sx[s] (its eigenvalue, the modified wavenumber of the slot) on each
// packed slot, and the y and z parts act on every slot alike. X(f) is the
// float64 transform of the float64 right-hand side; the iterate is exactly
// the stored float32 W, so R is the residual of that iterate (Neumann z rows:
// alpha_0 = 0, gamma_{nz-1} = 0, no excess). The float64 line sums of the
// iterate, W[slot 0] / ny, feed its plane means. The x inverse of the
// iterate disappears: the final pass transforms W + (correction) at once.
// Shape of k_xfwd; a workgroup takes LPW line pairs of one plane (2*LPW
// divides ny), in chunks of planes (see the block order below).
// XW = 1 (2): walls at both x ends: X(f) is k_xfwd's cosine (sine)
// transform, one real coefficient per slot, so a slot pair holds two x
// modes of the same line; the x second difference is still -sx[slot], and
// the cosine's zero mode of a constant f is 2 N f.
template <int N, int TPL, int LPW, int XW, int RO = 0>
__device__ __forceinline__ void resid_spec_body(
    const double *__restrict__ f, const double *__restrict__ fbar, const float *__restrict__ W,
    float *__restrict__ out, const cplx<double> *__restrict__ tw, const cplx<double> *__restrict__ ctw,
    double *__restrict__ sums_p, const double *__restrict__ sx, const double *__restrict__ zal,
    const double *__restrict__ zga, const double *__restrict__ zex, int ny, int nz, double idy2,
    double inv_ny, int ywalls, size_t sp,
                                                unsigned bx_, unsigned gx_) {
  using C = cplx<double>;
  static_assert(N % TPL == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * lds_len(N)];
  const int tid = threadIdx.x, l = tid / TPL, t = tid % TPL;
  // block order: chunks of kResidPlanes planes; within a chunk the planes
  // run fastest, then the row groups, so that the rows j-1 and j+2 (read
  // by the previous and the next row group of the same planes) and the
  // planes k-1 and k+1 are read by blocks close in time and come from L2
  const unsigned b = xcd_block(bx_, gx_);
  const int njg = ny / (2 * LPW);  // row groups of a plane
  const long per = (long)kResidPlanes * njg;
  const int k0 = (int)(b / per) * kResidPlanes;
  const int sz = nz - k0 < kResidPlanes ? nz - k0 : kResidPlanes;
  const long rem = (long)b - (long)(k0 / kResidPlanes) * per;
  const int k = k0 + (int)(rem % sz), j = (int)(rem / sz) * 2 * LPW + 2 * l;  // lines j, j+1
  C *buf = lds + l * lds_len(N);
  constexpr int NL = XW == 3 ? N / 2 : N;  // line length
  {
    // the first pass reads the line pair of f straight from global memory
    const double *fa = f + ((size_t)k * ny + j) * NL;
    const double *fb = fa + NL;
    auto src = [&](int i) {
      if constexpr (XW == 0) {
        return mkc<double>(fa[i], fb[i]);
      } else if constexpr (XW == 3) {
        return xface_src<XW>(i, NL, fa, fb);
      } else {
        const int x = xw_src(i, N);
        const double sg = (XW == 2 && (x & 1)) ? -1.0 : 1.0;
        return mkc<double>(sg * fa[x], sg * fb[x]);
      }
    };
    fft_line_io<double, N, TPL, false, true, false, RO>(buf, tw, t, src, [](int, const C &) {});
  }
  const double ak = zal[k], gk = zga[k], dk = ak + gk + zex[k];
  const double fk = (XW == 1 ? 2.0 : 1.0) * (double)N * fbar[k];
  const bool lo = k > 0, hi = k < nz - 1;
  // y neighbours of the line pair: periodic wrap, or the end row itself as
  // the ghost value beyond a wall, mirrored (ywalls 1, zero gradient) or
  // negated (ywalls 2, value zero on the wall)
  // ywalls 3: a field on the y faces: the wall face below row 0 is zero, row
  // ny - 1 is the top wall face (zero in the iterate; its residual row is
  // never read)
  const int jm = j == 0 ? (ywalls ? 0 : ny - 1) : j - 1;
  const int jp2 = j + 2 == ny ? (ywalls ? ny - 1 : 0) : j + 2;
  const double gm = j == 0 ? (ywalls == 2 ? -1.0 : ywalls == 3 ? 0.0 : 1.0) : 1.0;
  const double gp = j + 2 == ny ? (ywalls == 2 ? -1.0 : ywalls == 3 ? 0.0 : 1.0) : 1.0;
  const float *Wk = W + (size_t)k * sp;
  const float *w0 = Wk + (size_t)j * NL, *w1 = w0 + NL;        // lines j, j+1
  const float *wm = Wk + (size_t)jm * NL, *wp = Wk + (size_t)jp2 * NL;
  float *oa = out + (size_t)k * sp + (size_t)j * NL;
  float *ob = oa + NL;
#pragma unroll
  for (int q = t; q < N / 2; q += TPL) {
    if (XW == 3 && q >= NL / 2) continue;  // slot pairs of a line of NL
    C A, B;
    if constexpr (XW == 3) {
      // slots 2q and 2q+1 (modes 2q+1, 2q+2; the last slot is the wall)
      C v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int sl = 2 * q + h;
        const C e = sl < NL - 1 ? buf[lds_idx(sl + 1)] : mkc<double>(0.0, 0.0);
        v[h] = mkc<double>(-e.y, e.x);
      }
      A = mkc<double>(v[0].x, v[1].x);
      B = mkc<double>(v[0].y, v[1].y);
    } else if constexpr (XW != 0) {
      // slots 2q and 2q+1 of lines a (real parts) and b (imaginary parts)
      C v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int qc = XW == 2 ? N - 1 - (2 * q + h) : 2 * q + h;
        const C v1 = buf[lds_idx(qc)], v2 = buf[lds_idx(qc == 0 ? 0 : N - qc)], cq = ctw[qc];
        v[h] = mkc<double>(cq.x * v1.x - cq.y * v1.y + cq.x * v2.x + cq.y * v2.y,
                           cq.x * v1.y + cq.y * v1.x + cq.x * v2.y - cq.y * v2.x);
      }
      A = mkc<double>(v[0].x - (q == 0 ? fk : 0.0), v[1].x);
      B = mkc<double>(v[0].y - (q == 0 ? fk : 0.0), v[1].y);
    } else if (q == 0) {
      const C z0 = buf[lds_idx(0)], zh = buf[lds_idx(N / 2)];
      A = mkc<double>(z0.x - fk, zh.x);
      B = mkc<double>(z0.y - fk, zh.y);
    } else {
      split_pair<double>(buf[lds_idx(q)], buf[lds_idx(N - q)], A, B);
    }
    const C c0 = ld2<float>(w0 + 2 * q), c1 = ld2<float>(w1 + 2 * q);
    const C cm0 = ld2<float>(wm + 2 * q), cp0 = ld2<float>(wp + 2 * q);
    const C cm = mkc<double>(gm * cm0.x, gm * cm0.y), cp = mkc<double>(gp * cp0.x, gp * cp0.y);
    C za = mkc<double>(0.0, 0.0), zb = za;
    if (lo) {
      const C a0 = ld2<float>(w0 - sp + 2 * q), a1 = ld2<float>(w1 - sp + 2 * q);
      za = mkc<double>(ak * a0.x, ak * a0.y);
      zb = mkc<double>(ak * a1.x, ak * a1.y);
    }
    if (hi) {
      const C g0 = ld2<float>(w0 + sp + 2 * q), g1 = ld2<float>(w1 + sp + 2 * q);
      za = mkc<double>(za.x + gk * g0.x, za.y + gk * g0.y);
      zb = mkc<double>(zb.x + gk * g1.x, zb.y + gk * g1.y);
    }
    // slots 2q, 2q+1 (for q = 0: slot 0 the mean, slot 1 the Nyquist mode)
    const double s0 = sx[2 * q], s1 = sx[2 * q + 1];
    const double la0 = (cm.x - 2.0 * c0.x + c1.x) * idy2 + za.x - (dk + s0) * c0.x;
    const double la1 = (cm.y - 2.0 * c0.y + c1.y) * idy2 + za.y - (dk + s1) * c0.y;
    const double lb0 = (c0.x - 2.0 * c1.x + cp.x) * idy2 + zb.x - (dk + s0) * c1.x;
    const double lb1 = (c0.y - 2.0 * c1.y + cp.y) * idy2 + zb.y - (dk + s1) * c1.y;
    *reinterpret_cast<cplx<float> *>(oa + 2 * q) =
        mkc<float>((float)(A.x - inv_ny * la0), (float)(A.y - inv_ny * la1));
    *reinterpret_cast<cplx<float> *>(ob + 2 * q) =
        mkc<float>((float)(B.x - inv_ny * lb0), (float)(B.y - inv_ny * lb1));
    if (q == 0) {
      // the iterate's line sums (the cosine's slot 0 holds twice the sum)
      const double sc = XW == 1 ? 0.5 * inv_ny : inv_ny;
      sums_p[(size_t)k * ny + j] = c0.x * sc;
      sums_p[(size_t)k * ny + j + 1] = c1.x * sc;
    }
  }
}
template <int N, int TPL, int LPW, int XW, int RO = 0>
__global__ __launch_bounds__(TPL *LPW) void k_resid_spec(
    const double *__restrict__ f, const double *__restrict__ fbar, const float *__restrict__ W,
    float *__restrict__ out, const cplx<double> *__restrict__ tw, const cplx<double> *__restrict__ ctw,
    double *__restrict__ sums_p, const double *__restrict__ sx, const double *__restrict__ zal,
    const double *__restrict__ zga, const double *__restrict__ zex, int ny, int nz, double idy2,
    double inv_ny, int ywalls, size_t sp) {
  resid_spec_body<N, TPL, LPW, XW, RO>(f, fbar, W, out, tw, ctw, sums_p, sx, zal, zga, zex, ny, nz, idy2, inv_ny, ywalls, sp, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------- y forward

// YW = 1: zero-gradient walls at both y ends instead of periodicity. Every
// slot pair is then one complex line whose cosine transform
// X_q = 2 sum_y x_y cos(pi q (2y + 1) / 2N) is written in natural order (row
// q), for slots 0 and 1 as well: the transform has real coefficients, so it
// maps the real and imaginary parts separately. It is computed with one
// complex FFT of length N (Makhoul's reordering): v_n = x_{2n} and
// v_{N-1-n} = x_{2n+1}, V = FFT(v), X_q = c_q V_q + conj(c_q) V_{N-q} with
// c_q = exp(-i pi q / 2N) (ctw) and V_N = V_0.
// YW = 2: value-zero walls, the sine transform
// Y_q = 2 sum_y x_y sin(pi (q + 1) (2y + 1) / 2N), which is the cosine
// transform of (-1)^y x_y read backwards (Y_q = X'_{N-1-q}): the odd rows are
// negated as they are read and mode q is written to row N-1-q.
// XR (periodic y only): the x slots are real coefficients of x walls'
// cosine or sine transforms, so every slot pair is two real columns and takes
// the split into packed real y spectra that slots 0 and 1 take otherwise.
// A field on the y faces between value-zero walls (YW = 3): the type-I sine
// transform of each column's NR - 1 interior faces (rows 0..NR-2 hold the
// faces 1..NR-1, row NR-1 the top wall face), N = 2 NR. The column is
// extended oddly (e_m = x_m, e_{N-m} = -x_m, e_0 = e_NR = 0), transformed by
// one complex FFT of length N, and X_q = i E_q (q = 1..NR-1) goes to row
// q - 1, zero to the wall row. The transform has real coefficients, so the
// two columns of a slot pair transform together as the real and imaginary
// parts of one line, and it is its own inverse up to the factor 1 / N,
// which the x inverse's scale carries: the y forward and y inverse are this
// same function.
template <typename T, int N, int TPL, int LPW, int RO>
__device__ __forceinline__ void y_faces_body(T *base, const cplx<double> *__restrict__ tw, int nx,
                                             cplx<double> *lds, int tid) {
  using C = cplx<double>;
  constexpr int NR = N / 2, NT = TPL * LPW;
  static_assert(N % (2 * TPL) == 0, "every thread takes N / TPL positions");
  const int l = tid % LPW, t = tid / LPW;
  C *buf = lds + l * y_stride(N);
#pragma unroll
  for (int s = 0; s < N / (2 * TPL); ++s) {
    const int e = tid + s * NT;
    const int l2 = e % LPW, r = e / LPW;
    C *b2 = lds + l2 * y_stride(N);
    if (r < NR - 1) {
      const C v = ld2<T>(base + (size_t)r * nx + 2 * l2);
      b2[lds_idx(r + 1)] = v;
      b2[lds_idx(N - 1 - r)] = mkc<double>(-v.x, -v.y);
    } else {
      b2[lds_idx(0)] = mkc<double>(0.0, 0.0);
      b2[lds_idx(NR)] = mkc<double>(0.0, 0.0);
    }
  }
  __syncthreads();
  auto dst = [&](int q, const C &v) {
    if (q >= 1 && q < NR)
      st2<T>(base + (size_t)(q - 1) * nx + 2 * l, -v.y, v.x);
    else if (q == NR)
      st2<T>(base + (size_t)(NR - 1) * nx + 2 * l, 0.0, 0.0);
  };
  fft_line_io<double, N, TPL, false, false, true, RO>(buf, tw, t, [](int) { return C{}; }, dst);
}

// The y forward's store of the workgroup holding slots 0 and 1 (and, with x
// walls, of every workgroup), from the transformed lines in LDS: slots 0
// and 1 are two real columns (x modes 0 and nx/2), split into two packed
// real y spectra (rows 2q, 2q+1 hold the real and imaginary parts of mode
// q; rows 0 and 1 the modes 0 and ny/2) in float64 before rounding to the
// storage type; the other slot pairs are stored as they are.
template <typename T, int N, int TPL, int LPW, bool XR>
__device__ __forceinline__ void yfwd_split_store(const cplx<double> *lds, T *base, int nx, int tid) {
  using C = cplx<double>;
  constexpr int NT = TPL * LPW;
#pragma unroll
  for (int s = 0; s < N / TPL; ++s) {
    const int e = tid + s * NT;
    const int l2 = e % LPW, y = e / LPW;
    const C *b2 = lds + l2 * y_stride(N);
    if (l2 != 0 && !XR) {
      const C v = b2[lds_idx(y)];
      st2<T>(base + (size_t)y * nx + 2 * l2, v.x, v.y);
    } else if (y < N / 2) {
      const int q = y;
      C r0, r1;
      if (q == 0) {
        r0 = b2[lds_idx(0)];
        r1 = b2[lds_idx(N / 2)];
      } else {
        C A, B;
        split_pair<double>(b2[lds_idx(q)], b2[lds_idx(N - q)], A, B);
        r0 = mkc<double>(A.x, B.x);
        r1 = mkc<double>(A.y, B.y);
      }
      st2<T>(base + (size_t)(2 * q) * nx + 2 * l2, r0.x, r0.y);
      st2<T>(base + (size_t)(2 * q + 1) * nx + 2 * l2, r1.x, r1.y);
    }
  }
}

// Inverse of yfwd_split_store: the workgroup's lines into LDS, slots 0 and 1
// (every slot pair with x walls) joined from their two packed real spectra.
// The caller publishes the LDS lines with a barrier.
template <typename T, int N, int TPL, int LPW, bool XR>
__device__ __forceinline__ void yinv_join_load(cplx<double> *lds, const T *base, int nx, int tid) {
  using C = cplx<double>;
  constexpr int NT = TPL * LPW;
#pragma unroll
  for (int s = 0; s < N / TPL; ++s) {
    const int e = tid + s * NT;
    const int l2 = e % LPW, y = e / LPW;
    C *b2 = lds + l2 * y_stride(N);
    if (l2 != 0 && !XR) {
      b2[lds_idx(y)] = ld2<T>(base + (size_t)y * nx + 2 * l2);
    } else if (y < N / 2) {
      const int q = y;
      const C r0 = ld2<T>(base + (size_t)(2 * q) * nx + 2 * l2);
      const C r1 = ld2<T>(base + (size_t)(2 * q + 1) * nx + 2 * l2);
      if (q == 0) {
        b2[lds_idx(0)] = r0;
        b2[lds_idx(N / 2)] = r1;
      } else {
        C zq, zn;
        join_pair<double>(mkc<double>(r0.x, r1.x), mkc<double>(r0.y, r1.y), zq, zn);
        b2[lds_idx(q)] = zq;
        b2[lds_idx(N - q)] = zn;
      }
    }
  }
}

template <typename T, int N, int TPL, int LPW, int YW, bool XR = false, int RO = 0>
__device__ __forceinline__ void yfwd_body(T *__restrict__ data,
                                                   const cplx<double> *__restrict__ tw,
                                                   const cplx<double> *__restrict__ ctw, int nx,
                                                   int nib, size_t sp,
                                          unsigned bx_, unsigned gx_) {
  using C = cplx<double>;
  static_assert(N % (2 * TPL) == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * y_stride(N)];
  constexpr int NT = TPL * LPW;
  const int tid = threadIdx.x;
  const unsigned blk = xcd_block(bx_, gx_);
  const int ib = blk % nib;
  const long k = blk / nib;
  T *base = data + (size_t)k * sp + (size_t)ib * 2 * LPW;
  // lines run fastest across the lanes, so the first pass's reads (and the
  // last pass's writes) of row y cover the 2*LPW contiguous slots
  const int l = tid % LPW, t = tid / LPW;
  C *buf = lds + l * y_stride(N);
  auto src = [&](int y) { return ld2<T>(base + (size_t)y * nx + 2 * l); };
  if constexpr (YW == 3) {
    y_faces_body<T, N, TPL, LPW, RO>(base, tw, nx, lds, tid);
    return;
  } else if constexpr (YW != 0) {
    auto srcw = [&](int n) {
      const int y = n < N / 2 ? 2 * n : 2 * N - 1 - 2 * n;
      const C v = src(y);
      return (YW == 2 && (y & 1)) ? mkc<double>(-v.x, -v.y) : v;
    };
    fft_line_io<double, N, TPL, false, true, false, RO>(buf, tw, t, srcw, [](int, const C &) {});
#pragma unroll
    for (int s = 0; s < N / TPL; ++s) {
      const int e = tid + s * NT;
      const int l2 = e % LPW, q = e / LPW;
      const C *b2 = lds + l2 * y_stride(N);
      const C v1 = b2[lds_idx(q)], v2 = b2[lds_idx(q == 0 ? 0 : N - q)], c = ctw[q];
      const int row = YW == 2 ? N - 1 - q : q;
      st2<T>(base + (size_t)row * nx + 2 * l2, c.x * v1.x - c.y * v1.y + c.x * v2.x + c.y * v2.y,
             c.x * v1.y + c.y * v1.x + c.x * v2.y - c.y * v2.x);
    }
    return;
  }
  if (ib != 0 && !XR) {
    // slot pairs (2m, 2m+1), m >= 1, are the real and imaginary parts of x
    // mode m: their y transform is the complex spectrum itself, written in
    // natural order (row ky) by the last pass
    auto dst = [&](int y, const C &v) { st2<T>(base + (size_t)y * nx + 2 * l, v.x, v.y); };
    fft_line_io<double, N, TPL, false, true, true, RO>(buf, tw, t, src, dst);
    return;
  }
  // the workgroup of slots 0..2*LPW-1: slots 0 and 1 are two real columns
  // (x modes 0 and nx/2), split into two packed real y spectra (rows 2q,
  // 2q+1 hold the real and imaginary parts of mode q; rows 0 and 1 the
  // modes 0 and ny/2) in float64 before rounding to the storage type
  fft_line_io<double, N, TPL, false, true, false, RO>(buf, tw, t, src, [](int, const C &) {});
  yfwd_split_store<T, N, TPL, LPW, XR>(lds, base, nx, tid);
}
template <typename T, int N, int TPL, int LPW, int YW, bool XR = false, int RO = 0>
__global__ __launch_bounds__(TPL *LPW) void k_yfwd(T *__restrict__ data,
                                                   const cplx<double> *__restrict__ tw,
                                                   const cplx<double> *__restrict__ ctw, int nx,
                                                   int nib, size_t sp) {
  yfwd_body<T, N, TPL, LPW, YW, XR, RO>(data, tw, ctw, nx, nib, sp, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------- y inverse
// Inverse of k_yfwd's layout: complex spectra in natural order for slot
// pairs m >= 1, two packed real spectra for slots 0 and 1.
// YW != 0: inverse of k_yfwd's cosine (sine) transform: V_q = conj(c_q)
// (X_q - i X_{N-q}) / 2 (X_N = 0), the inverse FFT of V, and the rows 2n and
// 2n+1 from v_n and v_{N-1-n} (sine: X_q is read from row N-1-q and the odd
// rows negated); the 1/N is left to the x inverse's scale, as for the
// periodic transform.
template <typename T, int N, int TPL, int LPW, int YW, bool XR = false, int RO = 0>
__device__ __forceinline__ void yinv_body(T *__restrict__ data,
                                                   const cplx<double> *__restrict__ tw,
                                                   const cplx<double> *__restrict__ ctw, int nx,
                                                   int nib, size_t sp,
                                          unsigned bx_, unsigned gx_) {
  using C = cplx<double>;
  static_assert(N % (2 * TPL) == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * y_stride(N)];
  constexpr int NT = TPL * LPW;
  const int tid = threadIdx.x;
  const unsigned blk = xcd_block(bx_, gx_);
  const int ib = blk % nib;
  const long k = blk / nib;
  T *base = data + (size_t)k * sp + (size_t)ib * 2 * LPW;
  const int l = tid % LPW, t = tid / LPW;
  C *buf = lds + l * y_stride(N);
  auto dst = [&](int y, const C &v) { st2<T>(base + (size_t)y * nx + 2 * l, v.x, v.y); };
  if constexpr (YW == 3) {
    y_faces_body<T, N, TPL, LPW, RO>(base, tw, nx, lds, tid);
    return;
  } else if constexpr (YW != 0) {
#pragma unroll
    for (int s = 0; s < N / TPL; ++s) {
      const int e = tid + s * NT;
      const int l2 = e % LPW, q = e / LPW;
      const int row = YW == 2 ? N - 1 - q : q;
      lds[l2 * y_stride(N) + lds_idx(q)] = ld2<T>(base + (size_t)row * nx + 2 * l2);
    }
    __syncthreads();
    // one thread per mode pair (q, N - q), q = 0..N/2: it reads both
    // coefficients before it overwrites them
    for (int e = tid; e < LPW * (N / 2 + 1); e += NT) {
      const int l2 = e % LPW, q = e / LPW;
      C *b2 = lds + l2 * y_stride(N);
      const C xq = b2[lds_idx(q)];
      const C xn = q == 0 ? mkc<double>(0.0, 0.0) : b2[lds_idx(N - q)];
      const C cq = ctw[q];
      // conj(c) (a - i b) / 2
      const double ur = 0.5 * (xq.x + xn.y), ui = 0.5 * (xq.y - xn.x);
      b2[lds_idx(q)] = mkc<double>(cq.x * ur + cq.y * ui, cq.x * ui - cq.y * ur);
      if (q != 0 && 2 * q != N) {
        const C cn = ctw[N - q];
        const double wr = 0.5 * (xn.x + xq.y), wi = 0.5 * (xn.y - xq.x);
        b2[lds_idx(N - q)] = mkc<double>(cn.x * wr + cn.y * wi, cn.x * wi - cn.y * wr);
      }
    }
    __syncthreads();
    auto dstw = [&](int n, const C &v) {
      const int y = n < N / 2 ? 2 * n : 2 * N - 1 - 2 * n;
      dst(y, (YW == 2 && (y & 1)) ? mkc<double>(-v.x, -v.y) : v);
    };
    fft_line_io<double, N, TPL, true, false, true, RO>(buf, tw, t, [](int) { return C{}; }, dstw);
    return;
  }
  if (ib != 0 && !XR) {
    // the first pass reads the complex spectrum straight from row ky
    auto src = [&](int y) { return ld2<T>(base + (size_t)y * nx + 2 * l); };
    fft_line_io<double, N, TPL, true, true, true, RO>(buf, tw, t, src, dst);
    return;
  }
  yinv_join_load<T, N, TPL, LPW, XR>(lds, base, nx, tid);
  __syncthreads();
  fft_line_io<double, N, TPL, true, false, true, RO>(buf, tw, t, [](int) { return C{}; }, dst);
}
template <typename T, int N, int TPL, int LPW, int YW, bool XR = false, int RO = 0>
__global__ __launch_bounds__(TPL *LPW) void k_yinv(T *__restrict__ data,
                                                   const cplx<double> *__restrict__ tw,
                                                   const cplx<double> *__restrict__ ctw, int nx,
                                                   int nib, size_t sp) {
  yinv_body<T, N, TPL, LPW, YW, XR, RO>(data, tw, ctw, nx, nib, sp, blockIdx.x, gridDim.x);
}

// ------------------------------------------- persistent y transforms
// The periodic y transforms of k_yfwd / k_yinv for a grid of at most one
// round of resident workgroups: workgroup w takes the blocks i G + w' of
// rounds i = 0, 1, ... (G workgroups; w' the XCD-contiguous renumbering of
// w in full rounds), and loads the next block's rows into registers right
// after the current block's first pass, so that those loads travel while
// the current block's other passes and stores run. The y inverse of slots 0
// and 1 joins its two packed real spectra while loading, so it takes its
// rows itself (without the prefetch). Same arithmetic as k_yfwd / k_yinv.
__device__ __forceinline__ long pf_round_block(long i, long G, long nblk) {
  const long b0 = i * G;
  return b0 + G <= nblk ? b0 + xcd_block(blockIdx.x, (unsigned)G) : b0 + blockIdx.x;
}
template <typename T, int N, int TPL, int LPW, bool INV>
__global__ __launch_bounds__(TPL *LPW) void k_y_persist(T *__restrict__ data,
                                                        const cplx<double> *__restrict__ tw, int nx,
                                                        int nib, size_t sp, long nblk) {
  using C = cplx<double>;
  using F = FirstPass<N, TPL, 0>;
  static_assert(N % (2 * TPL) == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * y_stride(N)];
  const int tid = threadIdx.x;
  const int l = tid % LPW, t = tid / LPW;
  C *buf = lds + l * y_stride(N);
  const long G = gridDim.x;
  long blk = pf_round_block(0, G, nblk);
  if (blk >= nblk) return;  // uniform
  auto at = [&](long b) { return data + (size_t)(b / nib) * sp + (size_t)(b % nib) * 2 * LPW; };
  // a block whose first pass starts from registers
  auto from_regs = [&](long b) { return !INV || b % nib != 0; };
  cplx<T> pre[F::IT][F::R];
  auto load = [&](long b) {
    const T *bb = at(b);
    first_load<N, TPL, 0>(pre, t, [&](int y) { return *reinterpret_cast<const cplx<T> *>(bb + (size_t)y * nx + 2 * l); });
  };
  if (from_regs(blk)) load(blk);
  for (long i = 0;; ++i) {
    const int ib = (int)(blk % nib);
    T *base = at(blk);
    const long nb = pf_round_block(i + 1, G, nblk);
    const bool more = nb < nblk;  // uniform
    // the thread's positions as values the compiler cannot carry from one
    // block to the next: otherwise it keeps every address of the passes
    // live across the loop and runs out of registers
    int tl = t, ll = l, tidl = tid;
    asm volatile("" : "+v"(tl), "+v"(ll), "+v"(tidl));
    C *bufl = lds + ll * y_stride(N);
    // nothing reads the LDS lines of the previous block any more
    if (i > 0) __syncthreads();
    auto dst = [&](int y, const C &v) { st2<T>(base + (size_t)y * nx + 2 * ll, v.x, v.y); };
    const bool regs = from_regs(blk);  // uniform
    if (regs) {
      fft_from_regs<double, N, TPL, INV, 0>(bufl, pre, tl);
    } else {
      yinv_join_load<T, N, TPL, LPW, false>(lds, base, nx, tidl);
      __syncthreads();
    }
    if (more && from_regs(nb)) {
      const T *bb = at(nb);
      first_load<N, TPL, 0>(pre, tl, [&](int y) { return *reinterpret_cast<const cplx<T> *>(bb + (size_t)y * nx + 2 * ll); });
    }
    if (!regs) {
      // the joined lines are in LDS: every pass from there
      fft_line_io<double, N, TPL, true, false, true, 0>(bufl, tw, tl, [](int) { return C{}; }, dst);
    } else if (INV || ib != 0) {
      fft_rest<double, N, TPL, INV, true, 0>(bufl, tw, tl, dst);
    } else {
      fft_rest<double, N, TPL, INV, false, 0>(bufl, tw, tl, dst);
      yfwd_split_store<T, N, TPL, LPW, false>(lds, base, nx, tidl);
    }
    if (!more) break;
    blk = nb;
  }
}

// ------------------------------------------------------------- x inverse
// in and out may be the same array (each workgroup reads its line pair into
// LDS before writing it), so they are not marked restrict.
// SUM2: the transform of in + in2 (two spectra of the same layout, summed
// in float64 before the inverse).
// XW = 1 (2): inverse of k_xfwd's cosine (sine) transform, as along y for y
// walls: V_q = conj(c_q) (X_q - i X_{N-q}) / 2 (X_N = 0) from the two lines'
// coefficients X = a + ib, the inverse FFT, and the positions 2n and 2n+1
// from v_n and v_{N-1-n} (sine: mode q read from slot q as the cosine index
// N-1-q, odd positions negated); the 1/N is in `scale`.
template <typename TS, typename TO, int N, int TPL, int LPW, bool ADDZ, bool SUM2, int XW, int RO = 0>
__device__ __forceinline__ void xinv_body(const TS *in, TO *out,
                                                   const cplx<double> *__restrict__ tw,
                                                   const cplx<double> *__restrict__ ctw,
                                                   const double *__restrict__ zm,
                                                   const TS *__restrict__ in2, double scale,
                                                   int ny, long ncl, size_t sp,
                                                   unsigned long long *__restrict__ stat,
                                          unsigned bx_, unsigned gx_) {
  using C = cplx<double>;
  static_assert(N % TPL == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * lds_len(N)];
  const int tid = threadIdx.x, l = tid / TPL, t = tid % TPL;
  const long c = (long)bx_ * LPW + l;
  const bool ok = c < ncl;
  C *buf = lds + l * lds_len(N);
  constexpr int NL = XW == 3 ? N / 2 : N;  // line length
  double m0 = 0.0, m1 = 0.0;  // largest |iterate| and |correction| seen (SUM2)
  if (XW == 3 && ok) {
    // the pair's slots oddly extended: mode q (slot q - 1) at positions q and
    // N - q negated; positions 0 and NL zero (the wall slot is not read)
    const size_t o = (size_t)(2 * c / ny) * sp + (size_t)(2 * c % ny) * NL;
    const TS *a = in + o;
    const TS *b = a + NL;
#pragma unroll
    for (int s = t; s < NL; s += TPL) {
      if (s < NL - 1) {
        double xa = (double)a[s], xb = (double)b[s];
        if (SUM2) {
          const double ya = (double)in2[o + s], yb = (double)in2[o + NL + s];
          m0 = fmax(m0, fmax(fabs(xa), fabs(xb)));
          m1 = fmax(m1, fmax(fabs(ya), fabs(yb)));
          xa += ya;
          xb += yb;
        }
        buf[lds_idx(s + 1)] = mkc<double>(xa, xb);
        buf[lds_idx(N - 1 - s)] = mkc<double>(-xa, -xb);
      } else {
        buf[lds_idx(0)] = mkc<double>(0.0, 0.0);
        buf[lds_idx(NL)] = mkc<double>(0.0, 0.0);
      }
    }
  }
  if (XW != 0 && XW != 3 && ok) {
    const size_t o = (size_t)(2 * c / ny) * sp + (size_t)(2 * c % ny) * N;
    const TS *a = in + o;
    const TS *b = a + N;
#pragma unroll
    for (int s = t; s < N; s += TPL) {
      double xa = (double)a[s], xb = (double)b[s];
      if (SUM2) {
        const double ya = (double)in2[o + s], yb = (double)in2[o + N + s];
        m0 = fmax(m0, fmax(fabs(xa), fabs(xb)));
        m1 = fmax(m1, fmax(fabs(ya), fabs(yb)));
        xa += ya;
        xb += yb;
      }
      // cosine index of the stored coefficient
      buf[lds_idx(XW == 2 ? N - 1 - s : s)] = mkc<double>(xa, xb);
    }
  }
  if (XW != 0) {
    __syncthreads();
    // one thread per index pair (q, N - q), q = 0..N/2: both read before
    // either is overwritten
    if (XW != 3 && ok) {
      for (int q = t; q <= N / 2; q += TPL) {
        const C xq = buf[lds_idx(q)];
        const C xn = q == 0 ? mkc<double>(0.0, 0.0) : buf[lds_idx(N - q)];
        const C cq = ctw[q];
        const double ur = 0.5 * (xq.x + xn.y), ui = 0.5 * (xq.y - xn.x);
        buf[lds_idx(q)] = mkc<double>(cq.x * ur + cq.y * ui, cq.x * ui - cq.y * ur);
        if (q != 0 && 2 * q != N) {
          const C cn = ctw[N - q];
          const double wr = 0.5 * (xn.x + xq.y), wi = 0.5 * (xn.y - xq.x);
          buf[lds_idx(N - q)] = mkc<double>(cn.x * wr + cn.y * wi, cn.x * wi - cn.y * wr);
        }
      }
    }
  }
  if (XW == 0 && ok) {
    const size_t o = (size_t)(2 * c / ny) * sp + (size_t)(2 * c % ny) * N;
    const TS *a = in + o;
    const TS *b = a + N;
    const TS *a2 = SUM2 ? in2 + o : nullptr;
    const TS *b2 = SUM2 ? a2 + N : nullptr;
#pragma unroll
    for (int q = t; q < N / 2; q += TPL) {
      C A = ld2<TS>(a + 2 * q);
      C B = ld2<TS>(b + 2 * q);
      if (SUM2) {
        const C A2 = ld2<TS>(a2 + 2 * q), B2 = ld2<TS>(b2 + 2 * q);
        m0 = fmax(m0, fmax(fmax(fabs(A.x), fabs(A.y)), fmax(fabs(B.x), fabs(B.y))));
        m1 = fmax(m1, fmax(fmax(fabs(A2.x), fabs(A2.y)), fmax(fabs(B2.x), fabs(B2.y))));
        A = mkc<double>(A.x + A2.x, A.y + A2.y);
        B = mkc<double>(B.x + B2.x, B.y + B2.y);
      }
      if (q == 0) {
        buf[lds_idx(0)] = mkc<double>(A.x, B.x);
        buf[lds_idx(N / 2)] = mkc<double>(A.y, B.y);
      } else {
        C zq, zn;
        join_pair<double>(A, B, zq, zn);
        buf[lds_idx(q)] = zq;
        buf[lds_idx(N - q)] = zn;
      }
    }
  }
  if (SUM2 && stat) {  // uniform: the a-posteriori estimate of the refinement
    for (int o = 32; o > 0; o >>= 1) {
      m0 = fmax(m0, __shfl_xor(m0, o));
      m1 = fmax(m1, __shfl_xor(m1, o));
    }
    // non-negative doubles order like their bit patterns
    if ((threadIdx.x & 63) == 0) {
      atomicMax(stat, (unsigned long long)__double_as_longlong(m0));
      atomicMax(stat + 1, (unsigned long long)__double_as_longlong(m1));
    }
  }
  __syncthreads();
  // the last pass writes both real lines straight to global memory
  const double add = ADDZ && ok ? zm[(2 * c) / ny] : 0.0;
  TO *oa = out + (ok ? (size_t)(2 * c) * NL : 0);
  TO *ob = oa + NL;
  auto dst = [&](int pos, const C &z) {
    if (ok) {
      if constexpr (XW == 3) {
        // the inverse DFT of the odd extension is 2i sum_q X_q sin(pi q m / NL):
        // face m = pos (position m - 1) takes -i z, times 1 / (2 NL) in scale
        if (pos >= 1 && pos < NL) {
          oa[pos - 1] = (TO)(z.y * scale + add);
          ob[pos - 1] = (TO)(-z.x * scale + add);
        } else if (pos == NL) {
          oa[NL - 1] = (TO)add;
          ob[NL - 1] = (TO)add;
        }
      } else if constexpr (XW == 0) {
        oa[pos] = (TO)(z.x * scale + add);
        ob[pos] = (TO)(z.y * scale + add);
      } else {
        const int x = xw_src(pos, N);
        const double sg = (XW == 2 && (x & 1)) ? -scale : scale;
        oa[x] = (TO)(z.x * sg + add);
        ob[x] = (TO)(z.y * sg + add);
      }
    }
  };
  fft_line_io<double, N, TPL, true, false, true, RO>(buf, tw, t, [](int) { return C{}; }, dst);
}
template <typename TS, typename TO, int N, int TPL, int LPW, bool ADDZ, bool SUM2, int XW, int RO = 0>
__global__ __launch_bounds__(TPL *LPW) void k_xinv(const TS *in, TO *out,
                                                   const cplx<double> *__restrict__ tw,
                                                   const cplx<double> *__restrict__ ctw,
                                                   const double *__restrict__ zm,
                                                   const TS *__restrict__ in2, double scale,
                                                   int ny, long ncl, size_t sp,
                                                   unsigned long long *__restrict__ stat) {
  xinv_body<TS, TO, N, TPL, LPW, ADDZ, SUM2, XW, RO>(in, out, tw, ctw, zm, in2, scale, ny, ncl, sp, stat, blockIdx.x, gridDim.x);
}

}  // namespace pf
