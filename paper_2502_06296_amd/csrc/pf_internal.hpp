// Internal declarations shared by the HIP translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fft_lds.hpp"

namespace pf {

// Workgroup b is dispatched to XCD b % 8, and each XCD has its own L2. This
// renumbers blocks so that every XCD walks one contiguous range of the
// logical block order: neighbouring blocks that read the two halves of the
// same 128-byte lines then share an L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  constexpr unsigned kXcd = 8;
  if (nb % kXcd) return b;
  return (b % kXcd) * (nb / kXcd) + b / kXcd;
}

// Transform lengths instantiated for the x and y directions: even 2^a 3^b
// up to 2048, the lengths of the paper's per-GPU weak-scaling share,
// 3456 x 3072, and of its strong-scaling grid, 3200 x 3456 (3200 = 2^7 5^2).
#define PF_FOR_FFT_SIZES_COMMON(X)                                                              \
  X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(3200) \
  X(3456)
#define PF_FOR_FFT_SIZES(X) PF_FOR_FFT_SIZES_COMMON(X)
#define PF_FOR_FFT_SIZES_Y(X) PF_FOR_FFT_SIZES_COMMON(X)

bool fft_size_supported(int n);    // x direction
bool fft_size_supported_y(int n);  // y direction

// Padding (elements) between the z planes of a float32 spectrum work array.
constexpr size_t kPlanePad = 64;

// Kernel shapes of the line transforms: TPL threads per complex line, LPW
// complex lines per workgroup. The LDS holds float64 complex lines whatever
// the storage type. x lines are contiguous; y lines are columns gathered as
// LPW pairs of adjacent x slots, 2*LPW contiguous values per row (128 bytes
// when the LDS budget allows). LPW is a power of two, so 2*LPW (at most 32)
// divides every supported nx.
// The lines longer than 2048 points keep 52-118 KB of LDS per workgroup, one
// to three workgroups per CU: the y transforms, the x inverse and the
// residual take more threads per line, the largest multiple of 32 up to 384
// that divides n / div (div = 2 where every thread takes pairs of
// positions), so that a CU still holds several waves per SIMD. The x
// forward transforms stop at 192 (384 made them slower, 1.23 -> 1.38 ms at
// 3456 points; 160-192 against 128 gains 1-2 %).
constexpr int long_tpl(int n, int div, int cap = 384) {
  for (int c = cap; c >= 64; c -= 32)
    if (n % (div * c) == 0) return c;
  return 0;
}
constexpr int xfwd_tpl(int n) {
  return n > 2048 && long_tpl(n, 1, 192) ? long_tpl(n, 1, 192) : (n / 16 < 16 ? 16 : (n / 16 > 128 ? 128 : n / 16));
}
constexpr int x_tpl(int n) { return n > 2048 && long_tpl(n, 1) ? long_tpl(n, 1) : xfwd_tpl(n); }
constexpr int x_lpw(int n) {
  const int by_threads = 256 / x_tpl(n);
  const int by_lds = 32768 / (n * 16);
  int v = 1;
  while (v * 2 <= by_threads && v * 2 <= by_lds) v *= 2;
  return v;
}
// the residual: twice the threads per line of the x transforms (its stencil
// loads after the transform need the extra waves to hide their latency)
constexpr int resid_tpl(int n) { return 2 * x_tpl(n) <= 256 && n % (2 * x_tpl(n)) == 0 ? 2 * x_tpl(n) : x_tpl(n); }
// planes per chunk of the residual's block order
constexpr int kResidPlanes = 8;
constexpr int resid_lpw(int n) {
  const int by_threads = 256 / resid_tpl(n) < 1 ? 1 : 256 / resid_tpl(n);
  const int by_lds = 32768 / (n * 16);
  int v = 1;
  while (v * 2 <= by_threads && v * 2 <= by_lds) v *= 2;
  return v;
}
constexpr int y_tpl(int n) {
  if (n > 2048 && long_tpl(n, 2)) return long_tpl(n, 2);
  int t = n / 8 < 8 ? 8 : (n / 8 > 256 ? 256 : n / 8);
  while (t > 8 && n % (2 * t)) t /= 2;  // every thread takes pairs of positions
  return t;
}
// LDS stride (complex elements) between the lines of a y workgroup: 2 mod 16,
// so that the load and store phases, whose lanes run over the lines first,
// put the 16 lanes of one 128-bit LDS access in different banks.
constexpr int y_stride(int n) {
  int s = lds_len(n);
  while (s % 16 != 2) ++s;
  return s;
}
template <typename T>
constexpr int y_lpw(int n) {
  const int want = sizeof(T) == 8 ? 8 : 16;
  const int by_lds = 65536 / (n * 16);
  int v = 2;
  while (v * 2 <= want && v * 2 <= by_lds) v *= 2;
  return v;
}

// Launch shapes of the periodic transforms the autotuner chooses from, per
// family: 0 the default above; 1 half the threads per line (twice the
// values per thread); 2 twice the threads per line (x transforms and the
// residual) or twice the lines per workgroup (y transforms); 3 the default
// threads and lines with the radix capped at 8. Shapes 1-3 exist for the
// lengths 256, 512, 1024 and 2048 where the length, the 1024-thread and the
// LDS limits allow them; shapes 0-2 compute the same butterflies (up to the
// compiler's fusion of multiply-adds), shape 3 in a different order of
// passes.
// Shape 4 (y transforms only, every length): the default threads and lines
// in a persistent launch that prefetches each workgroup's next block
// (k_y_persist).
constexpr int kTransformShapes = 5;
constexpr int kYPersistShape = 4;
constexpr bool tuned_len(int n) { return n == 256 || n == 512 || n == 1024 || n == 2048; }
struct TShape {
  int tpl, lpw, ro;
  bool ok;
};
constexpr TShape alt_shape(int n, int s, int t, int l, bool y, int lds_line_bytes, int tmin) {
  if (s == 0) return {t, l, 0, true};
  if (!tuned_len(n)) return {t, l, 0, false};
  if (s == 1) return {t / 2, l, 0, t / 2 >= tmin && n % (y ? t : t / 2) == 0};
  if (s == 2 && !y) return {2 * t, l, 0, 2 * t <= 256 && n % (2 * t) == 0 && 2 * t * l <= 1024};
  if (s == 2 && y)
    return {t, 2 * l, 0, 2 * l <= 16 && (long)2 * l * lds_line_bytes <= 160 * 1024 && t * 2 * l <= 1024};
  if (s == 3) return {t, l, 1, true};
  return {t, l, 0, false};
}
constexpr TShape xfwd_shape(int n, int s) { return alt_shape(n, s, xfwd_tpl(n), x_lpw(n), false, 0, 16); }
constexpr TShape xinv_shape(int n, int s) { return alt_shape(n, s, x_tpl(n), x_lpw(n), false, 0, 16); }
constexpr TShape resid_shape(int n, int s) { return alt_shape(n, s, resid_tpl(n), resid_lpw(n), false, 0, 16); }
template <typename T>
constexpr TShape y_shape(int n, int s) {
  return alt_shape(n, s, y_tpl(n), y_lpw<T>(n), true, y_stride(n) * 16, 8);
}

// --------------------------------------------------------------- launchers
// All return hipSuccess or the launch error. Lengths are runtime checked by
// the caller against fft_size_supported.

// Every transform runs in float64; T, TS and TO are storage types. A
// packed spectrum array holds its z planes sp >= nx*ny elements apart (the
// float32 work arrays are padded so that the z columns do not all fall on
// the same memory channels); real-space arrays are dense.
// x forward: rhs (float64 lines of nx) -> packed spectrum (T). Optional
// float64 sums of every input line (sums may be null). xw = 1 (2): walls at
// both x ends, the cosine (sine) transform, one real coefficient per slot in
// natural order; needs sums and ctwx = exp(-i pi q / 2 nx), q = 0..nx-1.
template <typename T>
hipError_t launch_xfwd(int nx, int ny, const double *in, T *out, size_t sp,
                       const cplx<double> *tw, double *sums, long lines, hipStream_t st,
                       int xw = 0, const cplx<double> *ctwx = nullptr, int shape = 0);
// x spectrum of the float64 7-point residual of the plane-mean-free
// problem, R = X(f - fbar[k]) - L7 of the iterate whose x spectrum (times ny)
// is W (float32, after the y inverse); the x operator is -sx per packed
// slot, the z rows (zal, zga, zex). Also the float64 line sums of the
// iterate. R is float32. ywalls: the y second difference wraps (0), or takes
// the end rows mirrored (1, zero-gradient walls) or negated (2, value-zero
// walls) as the ghost values beyond the walls, or (3, a field on the y
// faces) zero beyond row 0 and in the wall row ny - 1; W then holds the
// iterate's x spectrum times 2 ny.
hipError_t launch_resid_spec(int nx, int ny, int nz, const double *f, const double *fbar,
                             const float *W, float *out, size_t sp, const cplx<double> *tw,
                             double *sums_p, const double *sx, const double *zal,
                             const double *zga, const double *zex, double idy2, int ywalls,
                             hipStream_t st, int xw = 0, const cplx<double> *ctwx = nullptr,
                             int shape = 0);
// y forward / inverse, in place on the packed (T) data. yw = 1 (2) selects
// the cosine (sine) transform of zero-gradient (value-zero) y walls, in
// natural order for every slot pair; it needs ctw = exp(-i pi q / 2 ny),
// q = 0..ny-1. yw = 3: a field on the y faces between value-zero walls (row
// j the face j + 1, row ny - 1 the top wall face): the type-I sine
// transform, one FFT of length 2 ny per column (tw of that length), the
// same function forward and inverse (the inverse leaves the factor 2 ny).
// xr (periodic y): the x slots are real coefficients of x walls' transforms,
// so every slot pair is split into two packed real y spectra.
template <typename T>
hipError_t launch_yfwd(int nx, int ny, int nz, T *data, size_t sp, const cplx<double> *tw,
                       const cplx<double> *ctw, int yw, hipStream_t st, bool xr = false, int shape = 0);
template <typename T>
hipError_t launch_yinv(int nx, int ny, int nz, T *data, size_t sp, const cplx<double> *tw,
                       const cplx<double> *ctw, int yw, hipStream_t st, bool xr = false, int shape = 0);
// x inverse: packed (TS) -> real lines (TO), scaled by `scale`; optional
// per-plane float64 profile zm[k]; with in2 (requires zm) the inverse of
// in + in2, summed in float64.
// With in2, a non-null stat (4 unsigned 64-bit words) receives the largest
// |in| and |in2| values by atomic max (see launch_status_final).
// xw = 1 (2): the inverse cosine (sine) transform (requires zm and ctwx).
template <typename TS, typename TO>
hipError_t launch_xinv(int nx, int ny, const TS *in, size_t sp, TO *out, const cplx<double> *tw,
                       const double *zm, const TS *in2, double scale, long lines,
                       hipStream_t st, unsigned long long *stat = nullptr, int xw = 0,
                       const cplx<double> *ctwx = nullptr, int shape = 0);
// shapes 1..3 of the periodic transforms (kernels_fft_alt.hip); the
// arguments as above, validated by the callers
template <typename T>
hipError_t launch_xfwd_alt(int shape, int nx, int ny, const double *in, T *out, size_t sp,
                           const cplx<double> *tw, double *sums, long lines, hipStream_t st);
hipError_t launch_resid_alt(int shape, int nx, int ny, int nz, const double *f, const double *fbar,
                            const float *W, float *out, size_t sp, const cplx<double> *tw,
                            double *sums_p, const double *sx, const double *zal, const double *zga,
                            const double *zex, double idy2, int ywalls, hipStream_t st);
template <typename T>
hipError_t launch_y_alt(bool inv, int shape, int nx, int ny, int nz, T *data, size_t sp,
                        const cplx<double> *tw, hipStream_t st);
// the persistent y transforms (shape kYPersistShape, periodic x and y)
template <typename T>
hipError_t launch_y_persist(bool inv, int nx, int ny, int nz, T *data, size_t sp, const cplx<double> *tw,
                            hipStream_t st);
template <typename TS, typename TO>
hipError_t launch_xinv_alt(int shape, int nx, int ny, const TS *in, size_t sp, TO *out,
                           const cplx<double> *tw, const double *zm, const TS *in2, double scale,
                           long lines, hipStream_t st, unsigned long long *stat);
// a-posteriori status of a solve: zero the 4 words; then the estimate
// (max|in2| / max|in|)^2 into word 2 (-1 unless refined) and flag word 3
// when it exceeds tol
hipError_t launch_status_reset(unsigned long long *stat, hipStream_t st);
hipError_t launch_status_final(unsigned long long *stat, double tol, bool refined, hipStream_t st);

// Pressure projection (eqs. proj1_Lphi, proj1_ukp1, proj1_Pkp1, proj2_Pkp1).
// x forward of f = D u* / gdt built from the face velocities u, v (nz, ny,
// nx) and w (nz-1, ny, nx); rdzf[k] = 1/dzf[k], idx = nx/lx, idy = ny/ly,
// igdt = 1/gdt. A non-null stash receives f (real space, float64). Line sums
// always (sums must not be null).
struct DivArgs {
  const double *u, *v, *w, *rdzf;
  double idx, idy, igdt;
  double *stash;
  int ywalls;  // 1: zero-gradient y walls, v[ny-1] is the top wall face (no flux)
  int xwalls;  // 1: zero-gradient x walls, u[nx-1] is the east wall face (no flux);
               // the cosine transform along x with ctwx = exp(-i pi q / 2 nx)
  const cplx<double> *ctwx;
};
template <typename T>
hipError_t launch_xfwd_div(int nx, int ny, int nz, const DivArgs &d, T *out, size_t sp,
                           const cplx<double> *tw, double *sums, hipStream_t st);
// u -= gx (phi[i+1] - phi[i]), v -= gy (phi[j+1] - phi[j]), w -= gdt rdzc[k]
// (phi[k+1] - phi[k]) (gx = gdt/dx, gy = gdt/dy), p += phi - c L_z phi with
// the Neumann rows zal, zga. ywalls: no v correction on the top wall face
// j = ny-1; xwalls: no u correction on the east wall face i = nx-1.
hipError_t launch_project(int nx, int ny, int nz, const double *phi, double *u, double *v,
                          double *w, double *p, const double *zal, const double *zga,
                          const double *rdzc, double gx, double gy, double gdt, double c,
                          bool ywalls, bool xwalls, hipStream_t st);

// Poisson z solve on the doubly packed spectrum (in place), float64
// elimination in registers; the (0,0) slot column is set to zero. `variant`
// indexes a table of launch shapes (rows per thread, columns per workgroup,
// occupancy bound, reciprocal flavour); the z tables must be padded to a
// multiple of 16 rows. xr: x walls, every x slot its own real mode (the
// paired shapes then solve the two columns of a pair one after the other).
template <typename TS>
hipError_t launch_zsolve(int nx, int ny, int nz, TS *data, size_t sp, const double *zal,
                         const double *zga, const double *zex, const double *sx, const double *sy,
                         int variant, hipStream_t st, bool xr = false);
int zsolve_variant_count();
bool zsolve_variant_fits(int variant, int nx, int nz, int esize);  // esize: bytes per stored value
int zsolve_default_variant(int nx, int nz, bool fp64);

// ----------------------------------------------------- grouped launches
// One launch runs one stage of several independent problems that share the
// kernel instance (transform length; z-solve shape and chunk count):
// blockIdx.y selects the job, blockIdx.x runs over the widest job's blocks,
// and a job's blocks past its own count exit at once. Float32 storage with
// one float64-residual correction, periodic x and y. The fields a stage
// reads and writes:
//   x forward:  in = f (float64), out = W (float32), sums = line sums
//   y forward / inverse, z solve: out = W in place
//   residual:   in = f, in2 = W (iterate), out = correction's right-hand
//               side (float32), zm = fbar, sums = the iterate's line sums
//   x inverse:  in = W, in2 = correction, out = p (float64), zm = zero-mode
//               profile, scale, stat (nullable)
// nblk is set by the launcher.
constexpr int kMaxGroupJobs = 16;
struct GJob {
  const void *in;
  void *out;
  const void *in2;
  const cplx<double> *tw;
  double *sums;
  const double *zm;
  const double *zal, *zga, *zex, *sx, *sy;
  unsigned long long *stat;
  const double *aux;  // zero mode: dzf
  double scale, idy2;
  size_t sp;
  int nx, ny, nz, P;
  unsigned nblk;
};
struct GJobs {
  GJob j[kMaxGroupJobs];
  int count;
};
hipError_t launch_xfwd_grp(int nx, GJobs &g, hipStream_t st);
hipError_t launch_yfwd_grp(int ny, GJobs &g, hipStream_t st);
hipError_t launch_yinv_grp(int ny, GJobs &g, hipStream_t st);
hipError_t launch_resid_grp(int nx, GJobs &g, hipStream_t st);
hipError_t launch_xinv_grp(int nx, GJobs &g, hipStream_t st);
// the zero mode of every job: plane means fbar (out) of its line sums
// (sums), then the pinned solve for the profile m (in2 -> written) from
// fbar, dzf (aux), zal, zga; zero shift: plane means p0m (out) of the
// iterate's sums, then zm (zm, written) = m (in2) - p0m
hipError_t launch_zero_mode_grp(GJobs &g, hipStream_t st);
hipError_t launch_zero_shift_grp(GJobs &g, hipStream_t st);
// every job of the group runs z-solve `variant` (a separator-form shape)
// with the same chunk count
hipError_t launch_zsolve_grp(int variant, GJobs &g, hipStream_t st);
bool zsolve_variant_groups(int variant);
int zsolve_chunks(int variant, int nz);  // P of a variant for nz rows
// Singular (0,0) mode: plane means fbar[nz] of the right-hand side from its
// line sums, projection, pinned Neumann solve for the plane-mean profile
// m[nz] of p.
hipError_t launch_zero_mode(int nx, int ny, int nz, const double *sums, const double *dzf,
                            const double *zal, const double *zga, double *fbar, double *m,
                            hipStream_t st);
// zm = m - plane means of an iterate (from its float64 line sums; p0mean is
// nz doubles of scratch).
hipError_t launch_zero_shift(int nx, int ny, int nz, const double *sums_p0, const double *m,
                             double *p0mean, double *zm, hipStream_t st);

// Helmholtz apply (Algorithm 2, Steps 2-4).
struct HelmCoef {
  // per row r (n): forward multiplier alpha_r/b_{r-1}, backward multiplier
  // gamma_r/b_{r+1}, 1/b_r, |a_r|, |c_r|; M-matrix rows for the residual
  const void *fa, *bg, *ib, *ra, *rc;  // float or double per plan precision
  const double *al, *ga, *dg;          // float64 rows: s alpha, s gamma, diagonal
  const void *k1, *k2, *invd;          // reduced-system PCR multipliers [steps][2P], [2P]
  const void *tf, *tb, *ti;            // reduced-system twisted elimination [2P] each
  int n, P, steps;
};
struct HelmJob {
  void *field;
  int nx, ny;
  HelmCoef c;
};
constexpr int kMaxHelmJobs = 16;  // fields of one grouped Helmholtz launch
// precision: 0 float64, 1 float32 storage, 2 float64 I/O with a float32
// solve and one float64-residual correction.
// cw: columns per chunk, 16, 32 or 64, with P*cw <= 1024 (<= 512 staged).
// staged: persistent workgroups with the Step 1 tables in LDS.
hipError_t launch_helm(int precision, int chunk_rows, int cw, bool staged, int count,
                       const HelmJob *jobs, hipStream_t st);
int helm_default_cw(int P);

// Algorithm 2, Step 1 on the device: from the rows (alpha, gamma, excess)
// of -L_z (padded to P*M rows with zeros) and s, the 11 float64 tables of a
// Helmholtz plan in HelmCoef order (fa, bg, ib, ra, rc: P*M each; k1, k2:
// steps*2P; invd, tf, tb, ti: 2P), their float32 copies, and the M-matrix
// rows s alpha, s gamma, 1 + s excess and their sum. One workgroup; P <= 32,
// P*M <= 1024, M >= 3.
struct PcrPrep {
  const double *al, *ga, *ex;
  double *d[11];
  float *f[11];
  double *mA, *mG, *mE, *mD;
  int n, P, M, steps;
};
hipError_t launch_pcr_prepare(const PcrPrep &p, double s, hipStream_t st);
// dst[i] = src[i] + kappa for i < n
hipError_t launch_shift_add(const double *src, double *dst, int n, double kappa, hipStream_t st);

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st);

}  // namespace pf
