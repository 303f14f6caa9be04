// Line transforms of the Poisson solve (paper Sec. 2.2.3 steps 2, 3, 7, 8;
// packed real layout of App. A).
//
// x direction: a workgroup takes LPW consecutive pairs of real x lines, so
// every global access is a run of contiguous values. y direction: a
// workgroup takes one z plane and 2*LPW adjacent x slots and transforms the
// LPW complex columns formed by pairing neighbouring slots; each row access
// is 2*LPW contiguous values (128 bytes by default). The x<->y permutation of
// the pencil method is therefore never materialised: the y kernel gathers
// its columns straight from the x-packed array and writes them back in place.
//
// Storage (HBM) is float64 or float32 (TS); the transforms themselves always
// run in float64 in LDS and registers. A float32 butterfly network leaves
// errors of about eps32 * max|X| in every mode, and the refinement residual is
// dominated by high wavenumbers, so its weakly damped low modes would lose
// all their digits; rounding only at the stores keeps the per-mode error
// relative to each stored value.
#include "pf_internal.hpp"

namespace pf {

bool fft_size_supported(int n) {
  switch (n) {
#define PF_CASE(N) case N:
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    return true;
    default:
      return false;
  }
}

// ----------------------------------------------------------- x forward
template <typename T, int N, int TPL, int LPW, bool SUMS>
__global__ __launch_bounds__(TPL *LPW) void k_xfwd(const double *__restrict__ in, T *__restrict__ out,
                                                   const cplx<double> *__restrict__ tw,
                                                   double *__restrict__ sums, long ncl, int ny,
                                                   size_t sp) {
  using C = cplx<double>;
  __shared__ C lds[LPW * lds_len(N)];
  static_assert(N % TPL == 0, "every thread takes N / TPL positions");
  const int tid = threadIdx.x, l = tid / TPL, t = tid % TPL;
  const long c = (long)blockIdx.x * LPW + l;
  const bool ok = c < ncl;
  C *buf = lds + l * lds_len(N);
  if (ok) {
    const double *a = in + (size_t)(2 * c) * N;
    const double *b = a + N;
#pragma unroll
    for (int s = 0; s < N / TPL; ++s) {
      const int pos = t + s * TPL;
      buf[lds_idx(pos)] = mkc<double>(a[pos], b[pos]);
    }
  }
  __syncthreads();
  fft_line<double, N, TPL, false>(buf, tw, t);
  if (!ok) return;
  T *oa = out + (size_t)(2 * c / ny) * sp + (size_t)(2 * c % ny) * N;
  T *ob = oa + N;
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

// -------------------------------------- x forward of the 7-point residual
// r = (f - fbar[k]) - L7 p0 in float64 from the float32 iterate p0 (Neumann
// z rows: alpha_0 = 0, gamma_{nz-1} = 0, no excess), then the float32
// transform of r. The iterate carries no plane means (its (0,0) slot was
// zeroed), so removing the plane means of f keeps the large constant-per-
// plane part out of the float32 spectrum, where its rounding would spread
// into the weakly damped (0,j) and (i,0) modes.
//
// A workgroup takes R = 2*LPW consecutive x lines j0..j0+R-1 of plane k, in
// the transform shape of k_xfwd (TPL threads per complex line). Every global
// load is issued up front as G-wide vectors: the p0 tile of rows j0-1..j0+R
// (periodic in y), and per thread the f values and the p0 values of planes
// k-1 and k+1 of its groups (two lines x G columns). The tile goes to LDS,
// aliased onto the transform buffer; the x and y differences read it there,
// and the residual is held in registers until the tile is dead.
template <typename T, int G>
struct alignas(sizeof(T) * G > 16 ? 16 : sizeof(T) * G) vec_t {
  T v[G];
};

template <int N, int TPL, int LPW>
__global__ __launch_bounds__(TPL *LPW) void k_xfwd_resid(
    const double *__restrict__ f, const double *__restrict__ fbar, const float *__restrict__ p0,
    float *__restrict__ out, const cplx<double> *__restrict__ tw, double *__restrict__ sums_p,
    const double *__restrict__ zal, const double *__restrict__ zga, int ny, int nz, double idx2,
    double idy2, size_t sp) {
  using C = cplx<double>;
  constexpr int NT = TPL * LPW;
  constexpr int R = 2 * LPW;
  constexpr int G = (N / TPL) % 4 == 0 ? 4 : ((N / TPL) % 2 == 0 ? 2 : 1);
  constexpr int NG = N / G;            // column groups per line
  static_assert((LPW * NG) % NT == 0, "whole groups per thread");
  constexpr int GS = LPW * NG / NT;    // groups (2 lines x G columns) per thread
  constexpr int TV = (R + 2) * NG;     // vectors in the p0 tile
  constexpr int TS = (TV + NT - 1) / NT;
  constexpr int TSUM = NT / R >= 64 ? 64 : (NT / R >= 32 ? 32 : (NT / R >= 16 ? 16 : 8));
  static_assert(NT / R >= 8 && N % TSUM == 0, "line-sum lanes");
  using VF = vec_t<float, G>;
  using VD = vec_t<double, G>;
  __shared__ C lds[LPW * lds_len(N)];
  static_assert((R + 2) * N * sizeof(float) <= sizeof(lds), "p0 tile fits the transform buffer");
  float *P = reinterpret_cast<float *>(lds);  // tile row u = line j0 - 1 + u
  const int tid = threadIdx.x;
  // planes fastest: the workgroups of planes k-1, k, k+1 of one y block run
  // next to each other on one XCD, so the plane-(k+-1) lines that this one
  // reads are the other two's own lines, still in L2
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int k = (int)(b % nz), j0 = (int)(b / nz) * R;
  const long line0 = (long)k * ny + j0;
  const size_t plane = (size_t)ny * N;
  const float *pk = p0 + (size_t)k * plane;
  const double *fk = f + (size_t)k * plane;
  const bool lo = k > 0, hi = k < nz - 1;

  VF tv[TS];
#pragma unroll
  for (int s = 0; s < TS; ++s) {
    const int e = tid + s * NT;
    if (TV % NT == 0 || e < TV) {
      const int u = e / NG, c = e % NG;
      int j = j0 - 1 + u;
      j = j < 0 ? j + ny : (j >= ny ? j - ny : j);
      tv[s] = *reinterpret_cast<const VF *>(pk + (size_t)j * N + c * G);
    }
  }
  VD fv[GS][2];
  VF zm[GS][2], zp[GS][2];
#pragma unroll
  for (int s = 0; s < GS; ++s) {
    const int g = tid + s * NT, m = g / NG, c = g % NG;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const size_t o = (size_t)(j0 + 2 * m + h) * N + c * G;
      fv[s][h] = *reinterpret_cast<const VD *>(fk + o);
      if (lo) zm[s][h] = *reinterpret_cast<const VF *>(pk - plane + o);
      if (hi) zp[s][h] = *reinterpret_cast<const VF *>(pk + plane + o);
    }
  }
#pragma unroll
  for (int s = 0; s < TS; ++s) {
    const int e = tid + s * NT;
    if (TV % NT == 0 || e < TV) *reinterpret_cast<VF *>(P + (e / NG) * N + (e % NG) * G) = tv[s];
  }
  __syncthreads();

  // float64 sums of the R lines of p0 (tile rows 1..R)
  if (tid < R * TSUM) {
    const int l = tid / TSUM, u = tid % TSUM;
    const float *row = P + (l + 1) * N;
    double sum = 0.0;
#pragma unroll 8
    for (int i = u; i < N; i += TSUM) sum += (double)row[i];
#pragma unroll
    for (int w = TSUM / 2; w > 0; w /= 2) sum += __shfl_xor(sum, w, TSUM);
    if (u == 0) sums_p[line0 + l] = sum;
  }

  const double ak = zal[k], gk = zga[k], dk = ak + gk, fb = fbar[k];
  double r[GS][2][G];
#pragma unroll
  for (int s = 0; s < GS; ++s) {
    const int g = tid + s * NT, m = g / NG, i0 = (g % NG) * G;
    const int il = i0 == 0 ? N - 1 : i0 - 1, ir = i0 + G == N ? 0 : i0 + G;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float *row = P + (2 * m + h + 1) * N;
      const VF cv = *reinterpret_cast<const VF *>(row + i0);
      const VF up = *reinterpret_cast<const VF *>(row + N + i0);
      const VF dn = *reinterpret_cast<const VF *>(row - N + i0);
      const double xl = (double)row[il], xr = (double)row[ir];
#pragma unroll
      for (int v = 0; v < G; ++v) {
        const double c0 = (double)cv.v[v];
        double z = 0.0;
        if (lo) z += ak * (double)zm[s][h].v[v];
        if (hi) z += gk * (double)zp[s][h].v[v];
        const double acc = (fv[s][h].v[v] - fb) - (z - dk * c0);
        const double xm = v == 0 ? xl : (double)cv.v[v - 1];
        const double xp = v == G - 1 ? xr : (double)cv.v[v + 1];
        const double lx = (xp - 2.0 * c0 + xm) * idx2;
        const double ly = ((double)up.v[v] - 2.0 * c0 + (double)dn.v[v]) * idy2;
        r[s][h][v] = acc - (lx + ly);
      }
    }
  }
  __syncthreads();  // the tile is dead: the transform buffer takes the residual
#pragma unroll
  for (int s = 0; s < GS; ++s) {
    const int g = tid + s * NT, m = g / NG, i0 = (g % NG) * G;
#pragma unroll
    for (int v = 0; v < G; ++v) lds[m * lds_len(N) + lds_idx(i0 + v)] = mkc<double>(r[s][0][v], r[s][1][v]);
  }
  __syncthreads();
  const int l = tid / TPL, t = tid % TPL;
  C *buf = lds + l * lds_len(N);
  fft_line<double, N, TPL, false>(buf, tw, t);
  float *oa = out + (size_t)k * sp + (size_t)(j0 + 2 * l) * N;
  float *ob = oa + N;
#pragma unroll
  for (int q = t; q < N / 2; q += TPL) {
    C A, B;
    if (q == 0) {
      const C z0 = buf[lds_idx(0)], zh = buf[lds_idx(N / 2)];
      A = mkc<double>(z0.x, zh.x);
      B = mkc<double>(z0.y, zh.y);
    } else {
      split_pair<double>(buf[lds_idx(q)], buf[lds_idx(N - q)], A, B);
    }
    *reinterpret_cast<cplx<float> *>(oa + 2 * q) = mkc<float>((float)A.x, (float)A.y);
    *reinterpret_cast<cplx<float> *>(ob + 2 * q) = mkc<float>((float)B.x, (float)B.y);
  }
}

// ------------------------------------------------------------- y forward
template <typename T>
__device__ __forceinline__ cplx<double> ld2(const T *p) {
  const cplx<T> v = *reinterpret_cast<const cplx<T> *>(p);
  return mkc<double>((double)v.x, (double)v.y);
}
template <typename T>
__device__ __forceinline__ void st2(T *p, double x, double y) {
  *reinterpret_cast<cplx<T> *>(p) = mkc<T>((T)x, (T)y);
}

template <typename T, int N, int TPL, int LPW>
__global__ __launch_bounds__(TPL *LPW) void k_yfwd(T *__restrict__ data,
                                                   const cplx<double> *__restrict__ tw, int nx,
                                                   int nib, size_t sp) {
  using C = cplx<double>;
  static_assert(N % (2 * TPL) == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * y_stride(N)];
  constexpr int NT = TPL * LPW;
  const int tid = threadIdx.x;
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int ib = blk % nib;
  const long k = blk / nib;
  T *base = data + (size_t)k * sp + (size_t)ib * 2 * LPW;
#pragma unroll
  for (int s = 0; s < N / TPL; ++s) {
    const int e = tid + s * NT;
    const int l = e % LPW, y = e / LPW;
    lds[l * y_stride(N) + lds_idx(y)] = ld2<T>(base + (size_t)y * nx + 2 * l);
  }
  __syncthreads();
  const int l = tid / TPL, t = tid % TPL;
  fft_line<double, N, TPL, false>(lds + l * y_stride(N), tw, t);
#pragma unroll
  for (int s = 0; s < N / (2 * TPL); ++s) {
    const int e = tid + s * NT;
    const int l2 = e % LPW, q = e / LPW;
    const C *buf = lds + l2 * y_stride(N);
    C r0, r1;
    if (q == 0) {
      r0 = buf[lds_idx(0)];
      r1 = buf[lds_idx(N / 2)];
    } else {
      C A, B;
      split_pair<double>(buf[lds_idx(q)], buf[lds_idx(N - q)], A, B);
      r0 = mkc<double>(A.x, B.x);
      r1 = mkc<double>(A.y, B.y);
    }
    st2<T>(base + (size_t)(2 * q) * nx + 2 * l2, r0.x, r0.y);
    st2<T>(base + (size_t)(2 * q + 1) * nx + 2 * l2, r1.x, r1.y);
  }
}

// ------------------------------------------------------------- y inverse
template <typename T, int N, int TPL, int LPW>
__global__ __launch_bounds__(TPL *LPW) void k_yinv(T *__restrict__ data,
                                                   const cplx<double> *__restrict__ tw, int nx,
                                                   int nib, size_t sp) {
  using C = cplx<double>;
  static_assert(N % (2 * TPL) == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * y_stride(N)];
  constexpr int NT = TPL * LPW;
  const int tid = threadIdx.x;
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int ib = blk % nib;
  const long k = blk / nib;
  T *base = data + (size_t)k * sp + (size_t)ib * 2 * LPW;
#pragma unroll
  for (int s = 0; s < N / (2 * TPL); ++s) {
    const int e = tid + s * NT;
    const int l2 = e % LPW, q = e / LPW;
    C *buf = lds + l2 * y_stride(N);
    const C r0 = ld2<T>(base + (size_t)(2 * q) * nx + 2 * l2);
    const C r1 = ld2<T>(base + (size_t)(2 * q + 1) * nx + 2 * l2);
    if (q == 0) {
      buf[lds_idx(0)] = r0;
      buf[lds_idx(N / 2)] = r1;
    } else {
      C zq, zn;
      join_pair<double>(mkc<double>(r0.x, r1.x), mkc<double>(r0.y, r1.y), zq, zn);
      buf[lds_idx(q)] = zq;
      buf[lds_idx(N - q)] = zn;
    }
  }
  __syncthreads();
  const int l = tid / TPL, t = tid % TPL;
  fft_line<double, N, TPL, true>(lds + l * y_stride(N), tw, t);
#pragma unroll
  for (int s = 0; s < N / TPL; ++s) {
    const int e = tid + s * NT;
    const int l2 = e % LPW, y = e / LPW;
    const C v = lds[l2 * y_stride(N) + lds_idx(y)];
    st2<T>(base + (size_t)y * nx + 2 * l2, v.x, v.y);
  }
}

// ------------------------------------------------------------- x inverse
// in and out may be the same array (each workgroup reads its line pair into
// LDS before writing it), so they are not marked restrict.
template <typename TS, typename TO, int N, int TPL, int LPW, bool ADDZ, bool ADDP0>
__global__ __launch_bounds__(TPL *LPW) void k_xinv(const TS *in, TO *out,
                                                   const cplx<double> *__restrict__ tw,
                                                   const double *__restrict__ zm,
                                                   const float *__restrict__ p0, double scale,
                                                   int ny, long ncl, size_t sp) {
  using C = cplx<double>;
  static_assert(N % TPL == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * lds_len(N)];
  const int tid = threadIdx.x, l = tid / TPL, t = tid % TPL;
  const long c = (long)blockIdx.x * LPW + l;
  const bool ok = c < ncl;
  C *buf = lds + l * lds_len(N);
  if (ok) {
    const TS *a = in + (size_t)(2 * c / ny) * sp + (size_t)(2 * c % ny) * N;
    const TS *b = a + N;
#pragma unroll
    for (int q = t; q < N / 2; q += TPL) {
      const C A = ld2<TS>(a + 2 * q);
      const C B = ld2<TS>(b + 2 * q);
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
  __syncthreads();
  fft_line<double, N, TPL, true>(buf, tw, t);
  if (!ok) return;
  double add = 0.0;
  if (ADDZ) add = zm[(2 * c) / ny];
  TO *oa = out + (size_t)(2 * c) * N;
  TO *ob = oa + N;
  const float *pa = ADDP0 ? p0 + (size_t)(2 * c) * N : nullptr;
  const float *pb = ADDP0 ? pa + N : nullptr;
#pragma unroll
  for (int s = 0; s < N / TPL; ++s) {
    const int pos = t + s * TPL;
    const C z = buf[lds_idx(pos)];
    double va = z.x * scale + add;
    double vb = z.y * scale + add;
    if (ADDP0) { va += (double)pa[pos]; vb += (double)pb[pos]; }
    oa[pos] = (TO)va;
    ob[pos] = (TO)vb;
  }
}

// ------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_xfwd(int nx, int ny, const double *in, T *out, size_t sp,
                       const cplx<double> *tw, double *sums, long lines, hipStream_t st) {
  const long ncl = lines / 2;
  switch (nx) {
#define PF_CASE(N)                                                                              \
  case N: {                                                                                     \
    constexpr int TPL = x_tpl(N), LPW = x_lpw(N);                                               \
    dim3 g((unsigned)((ncl + LPW - 1) / LPW));                                                  \
    if (sums)                                                                                   \
      hipLaunchKernelGGL((k_xfwd<T, N, TPL, LPW, true>), g, dim3(TPL * LPW), 0, st, in, out, tw, \
                         sums, ncl, ny, sp);                                                    \
    else                                                                                        \
      hipLaunchKernelGGL((k_xfwd<T, N, TPL, LPW, false>), g, dim3(TPL * LPW), 0, st, in, out,    \
                         tw, sums, ncl, ny, sp);                                                \
    return hipGetLastError();                                                                   \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_xfwd_resid(int nx, int ny, int nz, const double *f, const double *fbar,
                             const float *p0, float *out, size_t sp, const cplx<double> *tw,
                             double *sums_p0, const double *zal, const double *zga, double idx2,
                             double idy2, hipStream_t st) {
  switch (nx) {
#define PF_CASE(N)                                                                               \
  case N: {                                                                                      \
    constexpr int TPL = x_tpl(N), LPW = x_lpw(N);                                                \
    if (ny % (2 * LPW)) return hipErrorInvalidValue;                                             \
    const long nblk = (long)ny * nz / (2 * LPW);                                                 \
    hipLaunchKernelGGL((k_xfwd_resid<N, TPL, LPW>), dim3((unsigned)nblk), dim3(TPL * LPW), 0, st, \
                       f, fbar, p0, out, tw, sums_p0, zal, zga, ny, nz, idx2, idy2, sp);         \
    return hipGetLastError();                                                                    \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_yfwd(int nx, int ny, int nz, T *data, size_t sp, const cplx<double> *tw,
                       hipStream_t st) {
  switch (ny) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = y_tpl(N), LPW = y_lpw<T>(N);                                          \
    if (nx % (2 * LPW)) return hipErrorInvalidValue;                                          \
    const int nib = nx / (2 * LPW);                                                           \
    hipLaunchKernelGGL((k_yfwd<T, N, TPL, LPW>), dim3((unsigned)((long)nib * nz)),            \
                       dim3(TPL * LPW), 0, st, data, tw, nx, nib, sp);                        \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_yinv(int nx, int ny, int nz, T *data, size_t sp, const cplx<double> *tw,
                       hipStream_t st) {
  switch (ny) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = y_tpl(N), LPW = y_lpw<T>(N);                                          \
    if (nx % (2 * LPW)) return hipErrorInvalidValue;                                          \
    const int nib = nx / (2 * LPW);                                                           \
    hipLaunchKernelGGL((k_yinv<T, N, TPL, LPW>), dim3((unsigned)((long)nib * nz)),            \
                       dim3(TPL * LPW), 0, st, data, tw, nx, nib, sp);                        \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename TS, typename TO>
hipError_t launch_xinv(int nx, int ny, const TS *in, size_t sp, TO *out, const cplx<double> *tw,
                       const double *zm, const float *p0, double scale, long lines,
                       hipStream_t st) {
  const long ncl = lines / 2;
  switch (nx) {
#define PF_CASE(N)                                                                              \
  case N: {                                                                                     \
    constexpr int TPL = x_tpl(N), LPW = x_lpw(N);                                               \
    dim3 g((unsigned)((ncl + LPW - 1) / LPW)), b(TPL * LPW);                                    \
    if (zm && p0)                                                                               \
      hipLaunchKernelGGL((k_xinv<TS, TO, N, TPL, LPW, true, true>), g, b, 0, st, in, out, tw,  \
                         zm, p0, scale, ny, ncl, sp);                                               \
    else if (zm)                                                                                \
      hipLaunchKernelGGL((k_xinv<TS, TO, N, TPL, LPW, true, false>), g, b, 0, st, in, out, tw, \
                         zm, p0, scale, ny, ncl, sp);                                               \
    else                                                                                        \
      hipLaunchKernelGGL((k_xinv<TS, TO, N, TPL, LPW, false, false>), g, b, 0, st, in, out,    \
                         tw, zm, p0, scale, ny, ncl, sp);                                           \
    return hipGetLastError();                                                                   \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_xfwd<double>(int, int, const double *, double *, size_t,
                                        const cplx<double> *, double *, long, hipStream_t);
template hipError_t launch_xfwd<float>(int, int, const double *, float *, size_t,
                                       const cplx<double> *, double *, long, hipStream_t);
template hipError_t launch_yfwd<double>(int, int, int, double *, size_t, const cplx<double> *,
                                        hipStream_t);
template hipError_t launch_yfwd<float>(int, int, int, float *, size_t, const cplx<double> *,
                                       hipStream_t);
template hipError_t launch_yinv<double>(int, int, int, double *, size_t, const cplx<double> *,
                                        hipStream_t);
template hipError_t launch_yinv<float>(int, int, int, float *, size_t, const cplx<double> *,
                                       hipStream_t);
template hipError_t launch_xinv<double, double>(int, int, const double *, size_t, double *,
                                                const cplx<double> *, const double *,
                                                const float *, double, long, hipStream_t);
template hipError_t launch_xinv<float, float>(int, int, const float *, size_t, float *,
                                              const cplx<double> *, const double *, const float *,
                                              double, long, hipStream_t);
template hipError_t launch_xinv<float, double>(int, int, const float *, size_t, double *,
                                               const cplx<double> *, const double *, const float *,
                                               double, long, hipStream_t);

}  // namespace pf
