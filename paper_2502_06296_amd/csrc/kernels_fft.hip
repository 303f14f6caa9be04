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
                                                   double *__restrict__ sums, long ncl) {
  using C = cplx<double>;
  __shared__ C lds[LPW * lds_len(N)];
  static_assert(N % TPL == 0, "every thread takes N / TPL positions");
  __shared__ double red[SUMS ? 2 * LPW * TPL : 2];
  const int tid = threadIdx.x, l = tid / TPL, t = tid % TPL;
  const long c = (long)blockIdx.x * LPW + l;
  const bool ok = c < ncl;
  C *buf = lds + l * lds_len(N);
  double sa = 0.0, sb = 0.0;
  if (ok) {
    const double *a = in + (size_t)(2 * c) * N;
    const double *b = a + N;
#pragma unroll
    for (int s = 0; s < N / TPL; ++s) {
      const int pos = t + s * TPL;
      const double va = a[pos], vb = b[pos];
      if (SUMS) { sa += va; sb += vb; }
      buf[lds_idx(pos)] = mkc<double>(va, vb);
    }
  }
  if (SUMS) { red[2 * tid] = sa; red[2 * tid + 1] = sb; }
  __syncthreads();
  fft_line<double, N, TPL, false>(buf, tw, t);
  if (!ok) return;
  if (SUMS && t == 0) {
    double A = 0.0, B = 0.0;
    for (int u = 0; u < TPL; ++u) { A += red[2 * (l * TPL + u)]; B += red[2 * (l * TPL + u) + 1]; }
    sums[2 * c] = A;
    sums[2 * c + 1] = B;
  }
  T *oa = out + (size_t)(2 * c) * N;
  T *ob = oa + N;
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
// One workgroup per line pair (j, j+1) of plane k, TPL threads: every load
// (f, the pair and its y neighbours j-1, j+2 at plane k, the pair at k-1 and
// k+1) is issued up front; the plane-k lines go to LDS for the x and y
// differences. Each XCD walks a contiguous run of planes, so the neighbour
// lines read by other workgroups are still in its L2.
template <int N, int TPL>
__global__ __launch_bounds__(TPL) void k_xfwd_resid(
    const double *__restrict__ f, const double *__restrict__ fbar, const float *__restrict__ p0,
    float *__restrict__ out, const cplx<double> *__restrict__ tw, double *__restrict__ sums_p,
    const double *__restrict__ zal, const double *__restrict__ zga, int ny, int nz, double idx2,
    double idy2, long ncl) {
  using C = cplx<double>;
  static_assert(N % TPL == 0, "every thread takes N / TPL positions");
  constexpr int S = N / TPL;
  __shared__ C buf[lds_len(N)];
  __shared__ float P[4][N];          // lines j-1, j, j+1, j+2 of plane k
  __shared__ double red[2 * TPL];
  const int t = threadIdx.x;
  const long c = (long)xcd_block(blockIdx.x, gridDim.x);
  const long line0 = 2 * c;
  const int k = (int)(line0 / ny);
  const int j0 = (int)(line0 % ny);
  const double ak = zal[k], gk = zga[k], dk = ak + gk, fb = fbar[k];
  const size_t plane = (size_t)ny * N;
  const size_t row0 = ((size_t)k * ny + j0) * N;
  const size_t rym = ((size_t)k * ny + (j0 == 0 ? ny - 1 : j0 - 1)) * N;
  const size_t ryp = ((size_t)k * ny + (j0 + 2 == ny ? 0 : j0 + 2)) * N;
  double acc[2][S];
  float pc[2][S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = t + s * TPL;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const size_t o = row0 + (size_t)h * N + i;
      pc[h][s] = p0[o];
      double z = 0.0;
      if (k > 0) z += ak * (double)p0[o - plane];
      if (k < nz - 1) z += gk * (double)p0[o + plane];
      acc[h][s] = (f[o] - fb) - (z - dk * (double)pc[h][s]);
    }
    P[0][i] = p0[rym + i];
    P[3][i] = p0[ryp + i];
  }
  double sp0 = 0.0, sp1 = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = t + s * TPL;
    P[1][i] = pc[0][s];
    P[2][i] = pc[1][s];
    sp0 += (double)pc[0][s];
    sp1 += (double)pc[1][s];
  }
  red[2 * t] = sp0;
  red[2 * t + 1] = sp1;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = t + s * TPL;
    const int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
    double r[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double c0 = (double)P[h + 1][i];
      const double lx = ((double)P[h + 1][ip] - 2.0 * c0 + (double)P[h + 1][im]) * idx2;
      const double ly = ((double)P[h + 2][i] - 2.0 * c0 + (double)P[h][i]) * idy2;
      r[h] = acc[h][s] - (lx + ly);
    }
    buf[lds_idx(i)] = mkc<double>(r[0], r[1]);
  }
  __syncthreads();
  fft_line<double, N, TPL, false>(buf, tw, t);
  if (t == 0) {
    double b0 = 0, b1 = 0;
    for (int u = 0; u < TPL; ++u) { b0 += red[2 * u]; b1 += red[2 * u + 1]; }
    sums_p[2 * c] = b0;
    sums_p[2 * c + 1] = b1;
  }
  float *oa = out + row0;
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
                                                   int nib) {
  using C = cplx<double>;
  static_assert(N % (2 * TPL) == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * lds_len(N)];
  constexpr int NT = TPL * LPW;
  const int tid = threadIdx.x;
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int ib = blk % nib;
  const long k = blk / nib;
  T *base = data + (size_t)k * N * nx + (size_t)ib * 2 * LPW;
#pragma unroll
  for (int s = 0; s < N / TPL; ++s) {
    const int e = tid + s * NT;
    const int l = e % LPW, y = e / LPW;
    lds[l * lds_len(N) + lds_idx(y)] = ld2<T>(base + (size_t)y * nx + 2 * l);
  }
  __syncthreads();
  const int l = tid / TPL, t = tid % TPL;
  fft_line<double, N, TPL, false>(lds + l * lds_len(N), tw, t);
#pragma unroll
  for (int s = 0; s < N / (2 * TPL); ++s) {
    const int e = tid + s * NT;
    const int l2 = e % LPW, q = e / LPW;
    const C *buf = lds + l2 * lds_len(N);
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
                                                   int nib) {
  using C = cplx<double>;
  static_assert(N % (2 * TPL) == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * lds_len(N)];
  constexpr int NT = TPL * LPW;
  const int tid = threadIdx.x;
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int ib = blk % nib;
  const long k = blk / nib;
  T *base = data + (size_t)k * N * nx + (size_t)ib * 2 * LPW;
#pragma unroll
  for (int s = 0; s < N / (2 * TPL); ++s) {
    const int e = tid + s * NT;
    const int l2 = e % LPW, q = e / LPW;
    C *buf = lds + l2 * lds_len(N);
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
  fft_line<double, N, TPL, true>(lds + l * lds_len(N), tw, t);
#pragma unroll
  for (int s = 0; s < N / TPL; ++s) {
    const int e = tid + s * NT;
    const int l2 = e % LPW, y = e / LPW;
    const C v = lds[l2 * lds_len(N) + lds_idx(y)];
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
                                                   int ny, long ncl) {
  using C = cplx<double>;
  static_assert(N % TPL == 0, "every thread takes N / TPL positions");
  __shared__ C lds[LPW * lds_len(N)];
  const int tid = threadIdx.x, l = tid / TPL, t = tid % TPL;
  const long c = (long)blockIdx.x * LPW + l;
  const bool ok = c < ncl;
  C *buf = lds + l * lds_len(N);
  if (ok) {
    const TS *a = in + (size_t)(2 * c) * N;
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
hipError_t launch_xfwd(int nx, const double *in, T *out, const cplx<double> *tw, double *sums,
                       long lines, hipStream_t st) {
  const long ncl = lines / 2;
  switch (nx) {
#define PF_CASE(N)                                                                              \
  case N: {                                                                                     \
    constexpr int TPL = x_tpl(N), LPW = x_lpw(N);                                               \
    dim3 g((unsigned)((ncl + LPW - 1) / LPW));                                                  \
    if (sums)                                                                                   \
      hipLaunchKernelGGL((k_xfwd<T, N, TPL, LPW, true>), g, dim3(TPL * LPW), 0, st, in, out, tw, \
                         sums, ncl);                                                            \
    else                                                                                        \
      hipLaunchKernelGGL((k_xfwd<T, N, TPL, LPW, false>), g, dim3(TPL * LPW), 0, st, in, out,    \
                         tw, sums, ncl);                                                        \
    return hipGetLastError();                                                                   \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_xfwd_resid(int nx, int ny, int nz, const double *f, const double *fbar,
                             const float *p0, float *out, const cplx<double> *tw, double *sums_p0,
                             const double *zal, const double *zga, double idx2, double idy2,
                             hipStream_t st) {
  const long ncl = (long)ny * nz / 2;
  switch (nx) {
#define PF_CASE(N)                                                                               \
  case N: {                                                                                      \
    constexpr int TPL = N / 4 > 256 ? 256 : N / 4;                                               \
    hipLaunchKernelGGL((k_xfwd_resid<N, TPL>), dim3((unsigned)ncl), dim3(TPL), 0, st, f, fbar,   \
                       p0, out, tw, sums_p0, zal, zga, ny, nz, idx2, idy2, ncl);                 \
    return hipGetLastError();                                                                    \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_yfwd(int nx, int ny, int nz, T *data, const cplx<double> *tw, hipStream_t st) {
  switch (ny) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = y_tpl(N), LPW = y_lpw<T>(N);                                          \
    if (nx % (2 * LPW)) return hipErrorInvalidValue;                                          \
    const int nib = nx / (2 * LPW);                                                           \
    hipLaunchKernelGGL((k_yfwd<T, N, TPL, LPW>), dim3((unsigned)((long)nib * nz)),            \
                       dim3(TPL * LPW), 0, st, data, tw, nx, nib);                            \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_yinv(int nx, int ny, int nz, T *data, const cplx<double> *tw, hipStream_t st) {
  switch (ny) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = y_tpl(N), LPW = y_lpw<T>(N);                                          \
    if (nx % (2 * LPW)) return hipErrorInvalidValue;                                          \
    const int nib = nx / (2 * LPW);                                                           \
    hipLaunchKernelGGL((k_yinv<T, N, TPL, LPW>), dim3((unsigned)((long)nib * nz)),            \
                       dim3(TPL * LPW), 0, st, data, tw, nx, nib);                            \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename TS, typename TO>
hipError_t launch_xinv(int nx, int ny, const TS *in, TO *out, const cplx<double> *tw,
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
                         zm, p0, scale, ny, ncl);                                               \
    else if (zm)                                                                                \
      hipLaunchKernelGGL((k_xinv<TS, TO, N, TPL, LPW, true, false>), g, b, 0, st, in, out, tw, \
                         zm, p0, scale, ny, ncl);                                               \
    else                                                                                        \
      hipLaunchKernelGGL((k_xinv<TS, TO, N, TPL, LPW, false, false>), g, b, 0, st, in, out,    \
                         tw, zm, p0, scale, ny, ncl);                                           \
    return hipGetLastError();                                                                   \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_xfwd<double>(int, const double *, double *, const cplx<double> *,
                                        double *, long, hipStream_t);
template hipError_t launch_xfwd<float>(int, const double *, float *, const cplx<double> *,
                                       double *, long, hipStream_t);
template hipError_t launch_yfwd<double>(int, int, int, double *, const cplx<double> *, hipStream_t);
template hipError_t launch_yfwd<float>(int, int, int, float *, const cplx<double> *, hipStream_t);
template hipError_t launch_yinv<double>(int, int, int, double *, const cplx<double> *, hipStream_t);
template hipError_t launch_yinv<float>(int, int, int, float *, const cplx<double> *, hipStream_t);
template hipError_t launch_xinv<double, double>(int, int, const double *, double *,
                                                const cplx<double> *, const double *,
                                                const float *, double, long, hipStream_t);
template hipError_t launch_xinv<float, float>(int, int, const float *, float *,
                                              const cplx<double> *, const double *, const float *,
                                              double, long, hipStream_t);
template hipError_t launch_xinv<float, double>(int, int, const float *, double *,
                                               const cplx<double> *, const double *, const float *,
                                               double, long, hipStream_t);

}  // namespace pf
