// The alternative launch shapes of the periodic line transforms that the
// autotuner times (shapes 1-3 of pf_internal.hpp: threads per line, lines
// per workgroup, radix order), for the lengths 256, 512, 1024 and 2048. The
// kernels are the templates of fft_kernels.hpp; the default shapes are
// instantiated in kernels_fft.hip only.
#include "fft_kernels.hpp"
#include "pf_internal.hpp"

namespace pf {

namespace {
// one length and shape each; a shape that does not exist for the length is
// an invalid value (its kernel is never instantiated)
template <typename T, int N, int S>
hipError_t xfwd_one(int ny, const double *in, T *out, size_t sp, const cplx<double> *tw, double *sums,
                    long ncl, hipStream_t st) {
  constexpr TShape h = xfwd_shape(N, S);
  if constexpr (h.ok) {
    hipLaunchKernelGGL((k_xfwd<T, N, h.tpl, h.lpw, true, 0, h.ro>), dim3((unsigned)((ncl + h.lpw - 1) / h.lpw)),
                       dim3(h.tpl * h.lpw), 0, st, in, out, tw, nullptr, sums, ncl, ny, sp);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N, int S>
hipError_t resid_one(int ny, int nz, const double *f, const double *fbar, const float *W, float *out,
                     size_t sp, const cplx<double> *tw, double *sums_p, const double *sx,
                     const double *zal, const double *zga, const double *zex, double idy2, int ywalls,
                     hipStream_t st) {
  constexpr TShape h = resid_shape(N, S);
  if constexpr (h.ok) {
    if (ny % (2 * h.lpw)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_resid_spec<N, h.tpl, h.lpw, 0, h.ro>), dim3((unsigned)((long)ny * nz / (2 * h.lpw))),
                       dim3(h.tpl * h.lpw), 0, st, f, fbar, W, out, tw, nullptr, sums_p, sx, zal, zga, zex,
                       ny, nz, idy2, ywalls == 3 ? 0.5 / ny : 1.0 / ny, ywalls, sp);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T, int N, int S>
hipError_t y_one(bool inv, int nx, int nz, T *data, size_t sp, const cplx<double> *tw, hipStream_t st) {
  constexpr TShape h = y_shape<T>(N, S);
  if constexpr (h.ok) {
    if (nx % (2 * h.lpw)) return hipErrorInvalidValue;
    const int nib = nx / (2 * h.lpw);
    const dim3 g((unsigned)((long)nib * nz)), b(h.tpl * h.lpw);
    if (inv)
      hipLaunchKernelGGL((k_yinv<T, N, h.tpl, h.lpw, 0, false, h.ro>), g, b, 0, st, data, tw, nullptr, nx, nib,
                         sp);
    else
      hipLaunchKernelGGL((k_yfwd<T, N, h.tpl, h.lpw, 0, false, h.ro>), g, b, 0, st, data, tw, nullptr, nx, nib,
                         sp);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename TS, typename TO, int N, int S>
hipError_t xinv_one(int ny, const TS *in, size_t sp, TO *out, const cplx<double> *tw, const double *zm,
                    const TS *in2, double scale, long ncl, hipStream_t st, unsigned long long *stat) {
  constexpr TShape h = xinv_shape(N, S);
  if constexpr (h.ok) {
    const dim3 g((unsigned)((ncl + h.lpw - 1) / h.lpw)), b(h.tpl * h.lpw);
    if (in2)
      hipLaunchKernelGGL((k_xinv<TS, TO, N, h.tpl, h.lpw, true, true, 0, h.ro>), g, b, 0, st, in, out, tw,
                         nullptr, zm, in2, scale, ny, ncl, sp, stat);
    else
      hipLaunchKernelGGL((k_xinv<TS, TO, N, h.tpl, h.lpw, true, false, 0, h.ro>), g, b, 0, st, in, out, tw,
                         nullptr, zm, in2, scale, ny, ncl, sp, nullptr);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}
}  // namespace

#define PF_FOR_TUNED_SIZES(X) X(256) X(512) X(1024) X(2048)
// dispatch over the tuned lengths (n) and shapes 1..3 to F<..., N, S>(args)
#define PF_DISPATCH(n, F, ...)                                                                  \
  switch (n) {                                                                                  \
    PF_FOR_TUNED_SIZES(PF_DISPATCH_N)                                                           \
    default:                                                                                    \
      return hipErrorInvalidValue;                                                              \
  }

template <typename T>
hipError_t launch_xfwd_alt(int shape, int nx, int ny, const double *in, T *out, size_t sp,
                           const cplx<double> *tw, double *sums, long lines, hipStream_t st) {
  const long ncl = lines / 2;
#define PF_DISPATCH_N(N)                                                                        \
  case N:                                                                                       \
    if (shape == 1) return xfwd_one<T, N, 1>(ny, in, out, sp, tw, sums, ncl, st);              \
    if (shape == 2) return xfwd_one<T, N, 2>(ny, in, out, sp, tw, sums, ncl, st);              \
    if (shape == 3) return xfwd_one<T, N, 3>(ny, in, out, sp, tw, sums, ncl, st);              \
    return hipErrorInvalidValue;
  PF_DISPATCH(nx, )
#undef PF_DISPATCH_N
}

hipError_t launch_resid_alt(int shape, int nx, int ny, int nz, const double *f, const double *fbar,
                            const float *W, float *out, size_t sp, const cplx<double> *tw,
                            double *sums_p, const double *sx, const double *zal, const double *zga,
                            const double *zex, double idy2, int ywalls, hipStream_t st) {
#define PF_DISPATCH_N(N)                                                                                   \
  case N:                                                                                                  \
    if (shape == 1) return resid_one<N, 1>(ny, nz, f, fbar, W, out, sp, tw, sums_p, sx, zal, zga, zex, idy2, ywalls, st); \
    if (shape == 2) return resid_one<N, 2>(ny, nz, f, fbar, W, out, sp, tw, sums_p, sx, zal, zga, zex, idy2, ywalls, st); \
    if (shape == 3) return resid_one<N, 3>(ny, nz, f, fbar, W, out, sp, tw, sums_p, sx, zal, zga, zex, idy2, ywalls, st); \
    return hipErrorInvalidValue;
  PF_DISPATCH(nx, )
#undef PF_DISPATCH_N
}

template <typename T>
hipError_t launch_y_alt(bool inv, int shape, int nx, int ny, int nz, T *data, size_t sp,
                        const cplx<double> *tw, hipStream_t st) {
#define PF_DISPATCH_N(N)                                                                        \
  case N:                                                                                       \
    if (shape == 1) return y_one<T, N, 1>(inv, nx, nz, data, sp, tw, st);                      \
    if (shape == 2) return y_one<T, N, 2>(inv, nx, nz, data, sp, tw, st);                      \
    if (shape == 3) return y_one<T, N, 3>(inv, nx, nz, data, sp, tw, st);                      \
    return hipErrorInvalidValue;
  PF_DISPATCH(ny, )
#undef PF_DISPATCH_N
}

template <typename TS, typename TO>
hipError_t launch_xinv_alt(int shape, int nx, int ny, const TS *in, size_t sp, TO *out,
                           const cplx<double> *tw, const double *zm, const TS *in2, double scale,
                           long lines, hipStream_t st, unsigned long long *stat) {
  const long ncl = lines / 2;
  if (!zm) return hipErrorInvalidValue;
#define PF_DISPATCH_N(N)                                                                                   \
  case N:                                                                                                  \
    if (shape == 1) return xinv_one<TS, TO, N, 1>(ny, in, sp, out, tw, zm, in2, scale, ncl, st, stat);    \
    if (shape == 2) return xinv_one<TS, TO, N, 2>(ny, in, sp, out, tw, zm, in2, scale, ncl, st, stat);    \
    if (shape == 3) return xinv_one<TS, TO, N, 3>(ny, in, sp, out, tw, zm, in2, scale, ncl, st, stat);    \
    return hipErrorInvalidValue;
  PF_DISPATCH(nx, )
#undef PF_DISPATCH_N
}
#undef PF_DISPATCH

template hipError_t launch_xfwd_alt<double>(int, int, int, const double *, double *, size_t,
                                            const cplx<double> *, double *, long, hipStream_t);
template hipError_t launch_xfwd_alt<float>(int, int, int, const double *, float *, size_t,
                                           const cplx<double> *, double *, long, hipStream_t);
template hipError_t launch_y_alt<double>(bool, int, int, int, int, double *, size_t,
                                         const cplx<double> *, hipStream_t);
template hipError_t launch_y_alt<float>(bool, int, int, int, int, float *, size_t,
                                        const cplx<double> *, hipStream_t);
template hipError_t launch_xinv_alt<double, double>(int, int, int, const double *, size_t, double *,
                                                    const cplx<double> *, const double *,
                                                    const double *, double, long, hipStream_t,
                                                    unsigned long long *);
template hipError_t launch_xinv_alt<float, double>(int, int, int, const float *, size_t, double *,
                                                   const cplx<double> *, const double *,
                                                   const float *, double, long, hipStream_t,
                                                   unsigned long long *);

}  // namespace pf
