// Persistent launches of the periodic y transforms (k_y_persist of
// fft_kernels.hpp): one round of resident workgroups, each prefetching its
// next block's rows during the current block's passes. The autotuner's y
// transform shape kYPersistShape.
#include "fft_kernels.hpp"
#include "pf_internal.hpp"

namespace pf {

namespace {
// compute units of the current device
int device_cus() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) return 0;
    cached[dev] = n;
  }
  return cached[dev];
}

template <typename T, int N, bool INV>
hipError_t y_persist_one(int nx, int nz, T *data, size_t sp, const cplx<double> *tw, hipStream_t st) {
  constexpr int TPL = y_tpl(N), LPW = y_lpw<T>(N);
  if (nx % (2 * LPW)) return hipErrorInvalidValue;
  const int nib = nx / (2 * LPW);
  const long nblk = (long)nib * nz;
  if (nblk <= 0) return hipSuccess;
  int occ = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_y_persist<T, N, TPL, LPW, INV>,
                                                                   TPL * LPW, 0);
  if (e != hipSuccess) return e;
  const int cus = device_cus();
  if (occ < 1 || cus < 1) return hipErrorInvalidValue;
  const long G = nblk < (long)cus * occ ? nblk : (long)cus * occ;
  hipLaunchKernelGGL((k_y_persist<T, N, TPL, LPW, INV>), dim3((unsigned)G), dim3(TPL * LPW), 0, st, data, tw, nx,
                     nib, sp, nblk);
  return hipGetLastError();
}
}  // namespace

template <typename T>
hipError_t launch_y_persist(bool inv, int nx, int ny, int nz, T *data, size_t sp, const cplx<double> *tw,
                            hipStream_t st) {
  switch (ny) {
#define PF_CASE(N)                                                                               \
  case N:                                                                                        \
    return inv ? y_persist_one<T, N, true>(nx, nz, data, sp, tw, st)                             \
               : y_persist_one<T, N, false>(nx, nz, data, sp, tw, st);
    PF_FOR_FFT_SIZES_Y(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_y_persist<double>(bool, int, int, int, double *, size_t, const cplx<double> *,
                                             hipStream_t);
template hipError_t launch_y_persist<float>(bool, int, int, int, float *, size_t, const cplx<double> *,
                                            hipStream_t);

}  // namespace pf
