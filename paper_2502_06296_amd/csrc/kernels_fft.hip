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
#include "fft_kernels.hpp"
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

bool fft_size_supported_y(int n) {
  switch (n) {
#define PF_CASE(N) case N:
    PF_FOR_FFT_SIZES_Y(PF_CASE)
#undef PF_CASE
    return true;
    default:
      return false;
  }
}

// ------------------------------------------- x forward of the divergence
// Right-hand side of a projection (eq. proj1_Lphi), f = D u* / gdt, formed
// while the first pass reads its positions: u on the x faces i+1/2 (the west
// face of cell i is the east face of cell i-1, periodic), v on the y faces
// j+1/2, w on the interior z faces (w[k] is the top face of cell k, 0 on
// both walls). The two lines of a pair are rows j, j+1 of one plane (ny is
// even), so they share the v row j. With STASH, f itself is also written
// (float64, real space) for the residual of a refinement; the first pass
// reads every position exactly once. Otherwise as k_xfwd with line sums.
// XW = 1: zero-gradient walls at both x ends: u[nx-1] is the east wall face
// and the west face of cell 0 a wall face, both without flux; the line then
// goes through the cosine transform along x (as k_xfwd with XW = 1).
template <typename T, int N, int TPL, int LPW, bool STASH, int XW = 0>
__global__ __launch_bounds__(TPL *LPW) void k_xfwd_div(DivArgs d, T *__restrict__ out,
                                                       const cplx<double> *__restrict__ tw,
                                                       double *__restrict__ sums, long ncl, int ny,
                                                       int nz, size_t sp) {
  static_assert(XW == 0 || XW == 1, "periodic x or zero-gradient x walls");
  using C = cplx<double>;
  __shared__ C lds[LPW * lds_len(N)];
  static_assert(N % TPL == 0, "every thread takes N / TPL positions");
  const int tid = threadIdx.x, l = tid / TPL, t = tid % TPL;
  const long c = (long)blockIdx.x * LPW + l;
  const bool ok = c < ncl;
  C *buf = lds + l * lds_len(N);
  const long L = ok ? 2 * c : 0;  // line of row j; L + 1 is row j + 1
  const int k = (int)(L / ny), j = (int)(L % ny);
  const size_t o = (size_t)L * N;
  const double *ua = d.u + o, *ub = ua + N;
  const double *va = d.v + o, *vb = va + N;
  const double *vm = d.v + ((size_t)k * ny + (j == 0 ? ny - 1 : j - 1)) * N;
  const bool top = k < nz - 1, bot = k > 0;
  const double *wta = top ? d.w + o : d.w;                   // top faces of rows j, j+1
  const double *wba = bot ? d.w + (o - (size_t)ny * N) : d.w;  // bottom faces
  const double rz = d.rdzf[k];
  auto src = [&](int n) {
    if (!ok) return mkc<double>(0.0, 0.0);
    // the position the transform takes at n: natural order, or Makhoul's
    // order for the cosine transform
    const int i = XW ? xw_src(n, N) : n;
    const int im = i == 0 ? N - 1 : i - 1;
    const double v0 = va[i];
    // with y walls the bottom wall face (below row 0) and the top one (row
    // ny-1, the north face of line b of the last pair) carry no flux; with
    // x walls the east face of the last cell and the west face of the first
    const double vs = (d.ywalls && j == 0) ? 0.0 : vm[i];
    const double vn = (d.ywalls && j + 2 == ny) ? 0.0 : vb[i];
    const double uea = XW && i == N - 1 ? 0.0 : ua[i], ueb = XW && i == N - 1 ? 0.0 : ub[i];
    const double uwa = XW && i == 0 ? 0.0 : ua[im], uwb = XW && i == 0 ? 0.0 : ub[im];
    double fa = (uea - uwa) * d.idx + (v0 - vs) * d.idy;
    double fb = (ueb - uwb) * d.idx + (vn - v0) * d.idy;
    if (top) {
      fa += wta[i] * rz;
      fb += wta[N + i] * rz;
    }
    if (bot) {
      fa -= wba[i] * rz;
      fb -= wba[N + i] * rz;
    }
    fa *= d.igdt;
    fb *= d.igdt;
    if (STASH) {
      d.stash[o + i] = fa;
      d.stash[o + N + i] = fb;
    }
    return mkc<double>(fa, fb);
  };
  fft_line_io<double, N, TPL, false, true, false>(buf, tw, t, src, [](int, const C &) {});
  if (!ok) return;
  T *oa = out + (size_t)k * sp + (size_t)j * N;
  T *ob = oa + N;
  if constexpr (XW == 1) {
    // one real cosine coefficient per slot: X_q = c_q Z_q + conj(c_q) Z_{N-q}
#pragma unroll
    for (int q = t; q < N; q += TPL) {
      const C v1 = buf[lds_idx(q)], v2 = buf[lds_idx(q == 0 ? 0 : N - q)], cq = d.ctwx[q];
      oa[q] = (T)(cq.x * v1.x - cq.y * v1.y + cq.x * v2.x + cq.y * v2.y);
      ob[q] = (T)(cq.x * v1.y + cq.y * v1.x + cq.x * v2.y - cq.y * v2.x);
      if (q == 0) {
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
      sums[2 * c] = z0.x;
      sums[2 * c + 1] = z0.y;
    } else {
      split_pair<double>(buf[lds_idx(q)], buf[lds_idx(N - q)], A, B);
    }
    *reinterpret_cast<cplx<T> *>(oa + 2 * q) = mkc<T>((T)A.x, (T)A.y);
    *reinterpret_cast<cplx<T> *>(ob + 2 * q) = mkc<T>((T)B.x, (T)B.y);
  }
}

// ------------------------------------------------ projection correction
// u -= gdt G phi on the faces and p += phi - c L_z phi (eqs. proj1_ukp1,
// proj1_Pkp1; proj2_Pkp1 with L_z for implicit wall-normal diffusion). A
// thread owns one (i, j) column and marches up the planes with phi[k-1],
// phi[k], phi[k+1] in registers; a wave covers 64 consecutive i, so every
// access is a 512-byte row segment and the x and y neighbours of phi come
// from lines the neighbouring lanes and rows read. The Neumann rows have
// alpha_0 = 0 and gamma_{nz-1} = 0, so the zeros past the walls drop out.
template <bool LZ>
__global__ __launch_bounds__(256) void k_project(const double *__restrict__ phi,
                                                 double *__restrict__ u, double *__restrict__ v,
                                                 double *__restrict__ w, double *__restrict__ p,
                                                 const double *__restrict__ zal,
                                                 const double *__restrict__ zga,
                                                 const double *__restrict__ rdzc, int nx, int ny,
                                                 int nz, double gx, double gy, double gdt, double c,
                                                 int ywalls, int xwalls) {
  const int i = blockIdx.x * 64 + (int)(threadIdx.x % 64);
  const int j = blockIdx.y * 4 + (int)(threadIdx.x / 64);
  if (i >= nx || j >= ny) return;  // no barrier follows
  // y (x) walls: no gradient across the top (east) wall face, v (u) there
  // stays as it is
  const double gyj = (ywalls && j + 1 == ny) ? 0.0 : gy;
  const double gxi = (xwalls && i + 1 == nx) ? 0.0 : gx;
  const size_t plane = (size_t)nx * ny;
  const size_t o = (size_t)j * nx + i;
  const size_t ox = (size_t)j * nx + (i + 1 == nx ? 0 : i + 1);
  const size_t oy = (size_t)(j + 1 == ny ? 0 : j + 1) * nx + i;
  double fm = 0.0, f0 = phi[o];
#pragma unroll 2
  for (int k = 0; k < nz; ++k) {
    const size_t b = (size_t)k * plane;
    const bool up = k + 1 < nz;
    const double fp = up ? phi[b + plane + o] : 0.0;
    const double fx = phi[b + ox], fy = phi[b + oy];
    u[b + o] -= gxi * (fx - f0);
    v[b + o] -= gyj * (fy - f0);
    if (up) w[b + o] -= gdt * rdzc[k] * (fp - f0);  // w is (nz-1, ny, nx)
    double dp = f0;
    if (LZ) {
      const double a = zal[k], g = zga[k];
      dp -= c * (a * fm + g * fp - (a + g) * f0);
    }
    p[b + o] += dp;
    fm = f0;
    f0 = fp;
  }
}

// ------------------------------------------------ a-posteriori status
// stat[0], stat[1]: largest |iterate| and |correction| spectra (bit
// patterns, atomic max); stat[2]: the estimate (max|corr| / max|iter|)^2 of
// the relative error one correction leaves, -1 without a correction;
// stat[3]: flags (1: the estimate exceeds tol).
__global__ void k_status_reset(unsigned long long *stat) {
  if (threadIdx.x < 4) stat[threadIdx.x] = 0ull;
}
__global__ void k_status_final(unsigned long long *stat, double tol, int refined) {
  if (threadIdx.x != 0) return;
  double est = -1.0;
  if (refined) {
    const double m0 = __longlong_as_double((long long)stat[0]);
    const double m1 = __longlong_as_double((long long)stat[1]);
    est = m0 > 0.0 ? (m1 / m0) * (m1 / m0) : (m1 > 0.0 ? 1.0 : 0.0);
  }
  stat[2] = (unsigned long long)__double_as_longlong(est);
  stat[3] = refined && !(est <= tol) ? 1ull : 0ull;
}
hipError_t launch_status_reset(unsigned long long *stat, hipStream_t st) {
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, st, stat);
  return hipGetLastError();
}
hipError_t launch_status_final(unsigned long long *stat, double tol, bool refined, hipStream_t st) {
  hipLaunchKernelGGL(k_status_final, dim3(1), dim3(64), 0, st, stat, tol, refined ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xfwd_div(int nx, int ny, int nz, const DivArgs &d, T *out, size_t sp,
                           const cplx<double> *tw, double *sums, hipStream_t st) {
  const long ncl = (long)ny * nz / 2;
  if (d.xwalls && !d.ctwx) return hipErrorInvalidValue;
  switch (nx) {
#define PF_CASE(N)                                                                               \
  case N: {                                                                                      \
    constexpr int TPL = xfwd_tpl(N), LPW = x_lpw(N);                                             \
    dim3 g((unsigned)((ncl + LPW - 1) / LPW));                                                   \
    if (d.xwalls && d.stash)                                                                     \
      hipLaunchKernelGGL((k_xfwd_div<T, N, TPL, LPW, true, 1>), g, dim3(TPL * LPW), 0, st, d,    \
                         out, tw, sums, ncl, ny, nz, sp);                                        \
    else if (d.xwalls)                                                                           \
      hipLaunchKernelGGL((k_xfwd_div<T, N, TPL, LPW, false, 1>), g, dim3(TPL * LPW), 0, st, d,   \
                         out, tw, sums, ncl, ny, nz, sp);                                        \
    else if (d.stash)                                                                            \
      hipLaunchKernelGGL((k_xfwd_div<T, N, TPL, LPW, true>), g, dim3(TPL * LPW), 0, st, d, out,  \
                         tw, sums, ncl, ny, nz, sp);                                             \
    else                                                                                         \
      hipLaunchKernelGGL((k_xfwd_div<T, N, TPL, LPW, false>), g, dim3(TPL * LPW), 0, st, d, out, \
                         tw, sums, ncl, ny, nz, sp);                                             \
    return hipGetLastError();                                                                    \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}
template hipError_t launch_xfwd_div<double>(int, int, int, const DivArgs &, double *, size_t,
                                            const cplx<double> *, double *, hipStream_t);
template hipError_t launch_xfwd_div<float>(int, int, int, const DivArgs &, float *, size_t,
                                           const cplx<double> *, double *, hipStream_t);

hipError_t launch_project(int nx, int ny, int nz, const double *phi, double *u, double *v,
                          double *w, double *p, const double *zal, const double *zga,
                          const double *rdzc, double gx, double gy, double gdt, double c,
                          bool ywalls, bool xwalls, hipStream_t st) {
  dim3 g((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4));
  const int yw = ywalls ? 1 : 0, xw = xwalls ? 1 : 0;
  if (c != 0.0)
    hipLaunchKernelGGL((k_project<true>), g, dim3(256), 0, st, phi, u, v, w, p, zal, zga, rdzc, nx,
                       ny, nz, gx, gy, gdt, c, yw, xw);
  else
    hipLaunchKernelGGL((k_project<false>), g, dim3(256), 0, st, phi, u, v, w, p, zal, zga, rdzc,
                       nx, ny, nz, gx, gy, gdt, c, yw, xw);
  return hipGetLastError();
}

// ------------------------------------------------------ grouped kernels
// One stage of several problems of one transform length per launch (float32
// storage with one float64-residual correction, periodic x and y); the job
// table is a kernel argument, read with scalar loads.
template <int N, int TPL, int LPW>
__global__ __launch_bounds__(TPL *LPW) void k_xfwd_grp(const GJobs g) {
  const GJob &J = g.j[blockIdx.y];
  if (blockIdx.x >= J.nblk) return;  // uniform per block
  xfwd_body<float, N, TPL, LPW, true, 0>(static_cast<const double *>(J.in), static_cast<float *>(J.out),
                                         J.tw, nullptr, J.sums, (long)J.ny * J.nz / 2, J.ny, J.sp,
                                         blockIdx.x, J.nblk);
}
template <int N, int TPL, int LPW>
__global__ __launch_bounds__(TPL *LPW) void k_yfwd_grp(const GJobs g) {
  const GJob &J = g.j[blockIdx.y];
  if (blockIdx.x >= J.nblk) return;
  yfwd_body<float, N, TPL, LPW, 0, false>(static_cast<float *>(J.out), J.tw, nullptr, J.nx,
                                          J.nx / (2 * LPW), J.sp, blockIdx.x, J.nblk);
}
template <int N, int TPL, int LPW>
__global__ __launch_bounds__(TPL *LPW) void k_yinv_grp(const GJobs g) {
  const GJob &J = g.j[blockIdx.y];
  if (blockIdx.x >= J.nblk) return;
  yinv_body<float, N, TPL, LPW, 0, false>(static_cast<float *>(J.out), J.tw, nullptr, J.nx,
                                          J.nx / (2 * LPW), J.sp, blockIdx.x, J.nblk);
}
template <int N, int TPL, int LPW>
__global__ __launch_bounds__(TPL *LPW) void k_resid_grp(const GJobs g) {
  const GJob &J = g.j[blockIdx.y];
  if (blockIdx.x >= J.nblk) return;
  resid_spec_body<N, TPL, LPW, 0>(static_cast<const double *>(J.in), J.zm, static_cast<const float *>(J.in2),
                                  static_cast<float *>(J.out), J.tw, nullptr, J.sums, J.sx, J.zal, J.zga,
                                  J.zex, J.ny, J.nz, J.idy2, 1.0 / J.ny, 0, J.sp, blockIdx.x, J.nblk);
}
template <int N, int TPL, int LPW>
__global__ __launch_bounds__(TPL *LPW) void k_xinv_grp(const GJobs g) {
  const GJob &J = g.j[blockIdx.y];
  if (blockIdx.x >= J.nblk) return;
  xinv_body<float, double, N, TPL, LPW, true, true, 0>(
      static_cast<const float *>(J.in), static_cast<double *>(J.out), J.tw, nullptr, J.zm,
      static_cast<const float *>(J.in2), J.scale, J.ny, (long)J.ny * J.nz / 2, J.sp, J.stat, blockIdx.x,
      J.nblk);
}

// ------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_xfwd(int nx, int ny, const double *in, T *out, size_t sp,
                       const cplx<double> *tw, double *sums, long lines, hipStream_t st, int xw,
                       const cplx<double> *ctwx, int shape) {
  const long ncl = lines / 2;
  if (xw != 0 && (!sums || !ctwx)) return hipErrorInvalidValue;
  if (xw == 3) {
    // a field on the x faces: one transform of twice the line length
    if (shape != 0) return hipErrorInvalidValue;
    switch (2 * nx) {
#define PF_CASE(N)                                                                              \
  case N: {                                                                                     \
    constexpr int TPL = xfwd_tpl(N), LPW = x_lpw(N);                                            \
    dim3 g((unsigned)((ncl + LPW - 1) / LPW));                                                  \
    hipLaunchKernelGGL((k_xfwd<T, N, TPL, LPW, true, 3>), g, dim3(TPL * LPW), 0, st, in, out,    \
                       tw, ctwx, sums, ncl, ny, sp);                                            \
    return hipGetLastError();                                                                   \
  }
      PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  if (shape != 0) {
    if (xw != 0 || !sums) return hipErrorInvalidValue;
    return launch_xfwd_alt<T>(shape, nx, ny, in, out, sp, tw, sums, lines, st);
  }
  switch (nx) {
#define PF_CASE(N)                                                                              \
  case N: {                                                                                     \
    constexpr int TPL = xfwd_tpl(N), LPW = x_lpw(N);                                            \
    dim3 g((unsigned)((ncl + LPW - 1) / LPW));                                                  \
    if (xw == 1)                                                                                \
      hipLaunchKernelGGL((k_xfwd<T, N, TPL, LPW, true, 1>), g, dim3(TPL * LPW), 0, st, in, out,  \
                         tw, ctwx, sums, ncl, ny, sp);                                          \
    else if (xw == 2)                                                                           \
      hipLaunchKernelGGL((k_xfwd<T, N, TPL, LPW, true, 2>), g, dim3(TPL * LPW), 0, st, in, out,  \
                         tw, ctwx, sums, ncl, ny, sp);                                          \
    else if (sums)                                                                              \
      hipLaunchKernelGGL((k_xfwd<T, N, TPL, LPW, true, 0>), g, dim3(TPL * LPW), 0, st, in, out,  \
                         tw, ctwx, sums, ncl, ny, sp);                                          \
    else                                                                                        \
      hipLaunchKernelGGL((k_xfwd<T, N, TPL, LPW, false, 0>), g, dim3(TPL * LPW), 0, st, in, out, \
                         tw, ctwx, sums, ncl, ny, sp);                                          \
    return hipGetLastError();                                                                   \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_resid_spec(int nx, int ny, int nz, const double *f, const double *fbar,
                             const float *W, float *out, size_t sp, const cplx<double> *tw,
                             double *sums_p, const double *sx, const double *zal,
                             const double *zga, const double *zex, double idy2, int ywalls,
                             hipStream_t st, int xw, const cplx<double> *ctwx, int shape) {
  if (xw != 0 && !ctwx) return hipErrorInvalidValue;
  if (shape != 0) {
    if (xw != 0) return hipErrorInvalidValue;
    return launch_resid_alt(shape, nx, ny, nz, f, fbar, W, out, sp, tw, sums_p, sx, zal, zga, zex, idy2,
                            ywalls, st);
  }
#define PF_RESID(N, XW)                                                                          \
  hipLaunchKernelGGL((k_resid_spec<N, TPL, LPW, XW>), dim3((unsigned)nblk), dim3(TPL * LPW), 0,  \
                     st, f, fbar, W, out, tw, ctwx, sums_p, sx, zal, zga, zex, ny, nz, idy2,      \
                     ywalls == 3 ? 0.5 / ny : 1.0 / ny, ywalls, sp)
  if (xw == 3) {
    // a field on the x faces: one transform of twice the line length
    switch (2 * nx) {
#define PF_CASE(N)                                                                               \
  case N: {                                                                                      \
    constexpr int TPL = resid_tpl(N), LPW = resid_lpw(N);                                        \
    if (ny % (2 * LPW)) return hipErrorInvalidValue;                                             \
    const long nblk = (long)ny * nz / (2 * LPW);                                                 \
    PF_RESID(N, 3);                                                                              \
    return hipGetLastError();                                                                    \
  }
      PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  switch (nx) {
#define PF_CASE(N)                                                                               \
  case N: {                                                                                      \
    constexpr int TPL = resid_tpl(N), LPW = resid_lpw(N);                                        \
    if (ny % (2 * LPW)) return hipErrorInvalidValue;                                             \
    const long nblk = (long)ny * nz / (2 * LPW);                                                 \
    if (xw == 1)                                                                                 \
      PF_RESID(N, 1);                                                                            \
    else if (xw == 2)                                                                            \
      PF_RESID(N, 2);                                                                            \
    else                                                                                         \
      PF_RESID(N, 0);                                                                            \
    return hipGetLastError();                                                                    \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
#undef PF_RESID
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_yfwd(int nx, int ny, int nz, T *data, size_t sp, const cplx<double> *tw,
                       const cplx<double> *ctw, int yw, hipStream_t st, bool xr, int shape) {
  if (yw == 3) {
    // a field on the y faces: one FFT of twice the rows per column
    if (shape != 0) return hipErrorInvalidValue;
    switch (2 * ny) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = y_tpl(N), LPW = y_lpw<T>(N);                                          \
    if (nx % (2 * LPW)) return hipErrorInvalidValue;                                          \
    const int nib = nx / (2 * LPW);                                                           \
    hipLaunchKernelGGL((k_yfwd<T, N, TPL, LPW, 3>), dim3((unsigned)((long)nib * nz)),          \
                       dim3(TPL * LPW), 0, st, data, tw, ctw, nx, nib, sp);                   \
    return hipGetLastError();                                                                 \
  }
      PF_FOR_FFT_SIZES_Y(PF_CASE)
#undef PF_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  if (shape != 0) {
    if (yw != 0 || xr) return hipErrorInvalidValue;
    if (shape == kYPersistShape) return launch_y_persist<T>(false, nx, ny, nz, data, sp, tw, st);
    return launch_y_alt<T>(false, shape, nx, ny, nz, data, sp, tw, st);
  }
  switch (ny) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = y_tpl(N), LPW = y_lpw<T>(N);                                          \
    if (nx % (2 * LPW)) return hipErrorInvalidValue;                                          \
    const int nib = nx / (2 * LPW);                                                           \
    const dim3 g((unsigned)((long)nib * nz)), b(TPL * LPW);                                   \
    if (yw != 0 && !ctw) return hipErrorInvalidValue;                                         \
    if (yw == 1)                                                                              \
      hipLaunchKernelGGL((k_yfwd<T, N, TPL, LPW, 1>), g, b, 0, st, data, tw, ctw, nx, nib,    \
                         sp);                                                                 \
    else if (yw == 2)                                                                         \
      hipLaunchKernelGGL((k_yfwd<T, N, TPL, LPW, 2>), g, b, 0, st, data, tw, ctw, nx, nib,    \
                         sp);                                                                 \
    else if (xr)                                                                              \
      hipLaunchKernelGGL((k_yfwd<T, N, TPL, LPW, 0, true>), g, b, 0, st, data, tw, ctw, nx,   \
                         nib, sp);                                                            \
    else                                                                                      \
      hipLaunchKernelGGL((k_yfwd<T, N, TPL, LPW, 0>), g, b, 0, st, data, tw, ctw, nx, nib,    \
                         sp);                                                                 \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES_Y(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_yinv(int nx, int ny, int nz, T *data, size_t sp, const cplx<double> *tw,
                       const cplx<double> *ctw, int yw, hipStream_t st, bool xr, int shape) {
  if (yw == 3) {
    // a field on the y faces: one FFT of twice the rows per column
    if (shape != 0) return hipErrorInvalidValue;
    switch (2 * ny) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = y_tpl(N), LPW = y_lpw<T>(N);                                          \
    if (nx % (2 * LPW)) return hipErrorInvalidValue;                                          \
    const int nib = nx / (2 * LPW);                                                           \
    hipLaunchKernelGGL((k_yinv<T, N, TPL, LPW, 3>), dim3((unsigned)((long)nib * nz)),          \
                       dim3(TPL * LPW), 0, st, data, tw, ctw, nx, nib, sp);                   \
    return hipGetLastError();                                                                 \
  }
      PF_FOR_FFT_SIZES_Y(PF_CASE)
#undef PF_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  if (shape != 0) {
    if (yw != 0 || xr) return hipErrorInvalidValue;
    if (shape == kYPersistShape) return launch_y_persist<T>(true, nx, ny, nz, data, sp, tw, st);
    return launch_y_alt<T>(true, shape, nx, ny, nz, data, sp, tw, st);
  }
  switch (ny) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = y_tpl(N), LPW = y_lpw<T>(N);                                          \
    if (nx % (2 * LPW)) return hipErrorInvalidValue;                                          \
    const int nib = nx / (2 * LPW);                                                           \
    const dim3 g((unsigned)((long)nib * nz)), b(TPL * LPW);                                   \
    if (yw != 0 && !ctw) return hipErrorInvalidValue;                                         \
    if (yw == 1)                                                                              \
      hipLaunchKernelGGL((k_yinv<T, N, TPL, LPW, 1>), g, b, 0, st, data, tw, ctw, nx, nib,    \
                         sp);                                                                 \
    else if (yw == 2)                                                                         \
      hipLaunchKernelGGL((k_yinv<T, N, TPL, LPW, 2>), g, b, 0, st, data, tw, ctw, nx, nib,    \
                         sp);                                                                 \
    else if (xr)                                                                              \
      hipLaunchKernelGGL((k_yinv<T, N, TPL, LPW, 0, true>), g, b, 0, st, data, tw, ctw, nx,   \
                         nib, sp);                                                            \
    else                                                                                      \
      hipLaunchKernelGGL((k_yinv<T, N, TPL, LPW, 0>), g, b, 0, st, data, tw, ctw, nx, nib,    \
                         sp);                                                                 \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES_Y(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename TS, typename TO>
hipError_t launch_xinv(int nx, int ny, const TS *in, size_t sp, TO *out, const cplx<double> *tw,
                       const double *zm, const TS *in2, double scale, long lines,
                       hipStream_t st, unsigned long long *stat, int xw,
                       const cplx<double> *ctwx, int shape) {
  const long ncl = lines / 2;
  // the walls' inverses are built for the solves' uses (with the zero-mode
  // profile, with or without a second spectrum)
  if (xw != 0 && (!zm || !ctwx)) return hipErrorInvalidValue;
  if (shape != 0) {
    if (xw != 0 || !zm) return hipErrorInvalidValue;
    return launch_xinv_alt<TS, TO>(shape, nx, ny, in, sp, out, tw, zm, in2, scale, lines, st, stat);
  }
#define PF_XINV(N, ADDZ, SUM2, XW, STAT)                                                         \
  hipLaunchKernelGGL((k_xinv<TS, TO, N, TPL, LPW, ADDZ, SUM2, XW>), g, b, 0, st, in, out, tw,    \
                     ctwx, zm, in2, scale, ny, ncl, sp, STAT)
  if (xw == 3) {
    // a field on the x faces: one transform of twice the line length
    switch (2 * nx) {
#define PF_CASE(N)                                                                              \
  case N: {                                                                                     \
    constexpr int TPL = x_tpl(N), LPW = x_lpw(N);                                               \
    dim3 g((unsigned)((ncl + LPW - 1) / LPW)), b(TPL * LPW);                                    \
    if (in2)                                                                                    \
      PF_XINV(N, true, true, 3, stat);                                                          \
    else                                                                                        \
      PF_XINV(N, true, false, 3, nullptr);                                                      \
    return hipGetLastError();                                                                   \
  }
      PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  switch (nx) {
#define PF_CASE(N)                                                                              \
  case N: {                                                                                     \
    constexpr int TPL = x_tpl(N), LPW = x_lpw(N);                                               \
    dim3 g((unsigned)((ncl + LPW - 1) / LPW)), b(TPL * LPW);                                    \
    if (xw == 1 && in2)                                                                         \
      PF_XINV(N, true, true, 1, stat);                                                             \
    else if (xw == 1)                                                                           \
      PF_XINV(N, true, false, 1, nullptr);                                                         \
    else if (xw == 2 && in2)                                                                    \
      PF_XINV(N, true, true, 2, stat);                                                             \
    else if (xw == 2)                                                                           \
      PF_XINV(N, true, false, 2, nullptr);                                                         \
    else if (zm && in2)                                                                         \
      PF_XINV(N, true, true, 0, stat);                                                             \
    else if (zm)                                                                                \
      PF_XINV(N, true, false, 0, nullptr);                                                         \
    else                                                                                        \
      PF_XINV(N, false, false, 0, nullptr);                                                        \
    return hipGetLastError();                                                                   \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
#undef PF_XINV
    default:
      return hipErrorInvalidValue;
  }
}

// grouped launchers: the grid spans the widest job; every job of a group
// has the length of the switch
static dim3 grp_grid(const GJobs &g) {
  unsigned m = 1;
  for (int k = 0; k < g.count; ++k) m = g.j[k].nblk > m ? g.j[k].nblk : m;
  return dim3(m, (unsigned)g.count);
}
static bool grp_ok(const GJobs &g) { return g.count >= 1 && g.count <= kMaxGroupJobs; }

hipError_t launch_xfwd_grp(int nx, GJobs &g, hipStream_t st) {
  if (!grp_ok(g)) return hipErrorInvalidValue;
  switch (nx) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = xfwd_tpl(N), LPW = x_lpw(N);                                          \
    for (int k = 0; k < g.count; ++k) {                                                       \
      if (g.j[k].nx != N || g.j[k].ny % 2) return hipErrorInvalidValue;                       \
      g.j[k].nblk = (unsigned)(((long)g.j[k].ny * g.j[k].nz / 2 + LPW - 1) / LPW);            \
    }                                                                                         \
    hipLaunchKernelGGL((k_xfwd_grp<N, TPL, LPW>), grp_grid(g), dim3(TPL * LPW), 0, st, g);    \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <bool INV>
static hipError_t launch_y_grp(int ny, GJobs &g, hipStream_t st) {
  if (!grp_ok(g)) return hipErrorInvalidValue;
  switch (ny) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = y_tpl(N), LPW = y_lpw<float>(N);                                      \
    for (int k = 0; k < g.count; ++k) {                                                       \
      if (g.j[k].ny != N || g.j[k].nx % (2 * LPW)) return hipErrorInvalidValue;               \
      g.j[k].nblk = (unsigned)(g.j[k].nx / (2 * LPW) * g.j[k].nz);                            \
    }                                                                                         \
    if (INV)                                                                                  \
      hipLaunchKernelGGL((k_yinv_grp<N, TPL, LPW>), grp_grid(g), dim3(TPL * LPW), 0, st, g);  \
    else                                                                                      \
      hipLaunchKernelGGL((k_yfwd_grp<N, TPL, LPW>), grp_grid(g), dim3(TPL * LPW), 0, st, g);  \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES_Y(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_yfwd_grp(int ny, GJobs &g, hipStream_t st) { return launch_y_grp<false>(ny, g, st); }
hipError_t launch_yinv_grp(int ny, GJobs &g, hipStream_t st) { return launch_y_grp<true>(ny, g, st); }

hipError_t launch_resid_grp(int nx, GJobs &g, hipStream_t st) {
  if (!grp_ok(g)) return hipErrorInvalidValue;
  switch (nx) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = resid_tpl(N), LPW = resid_lpw(N);                                     \
    for (int k = 0; k < g.count; ++k) {                                                       \
      if (g.j[k].nx != N || g.j[k].ny % (2 * LPW)) return hipErrorInvalidValue;               \
      g.j[k].nblk = (unsigned)((long)g.j[k].ny * g.j[k].nz / (2 * LPW));                      \
    }                                                                                         \
    hipLaunchKernelGGL((k_resid_grp<N, TPL, LPW>), grp_grid(g), dim3(TPL * LPW), 0, st, g);   \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_xinv_grp(int nx, GJobs &g, hipStream_t st) {
  if (!grp_ok(g)) return hipErrorInvalidValue;
  switch (nx) {
#define PF_CASE(N)                                                                            \
  case N: {                                                                                   \
    constexpr int TPL = x_tpl(N), LPW = x_lpw(N);                                             \
    for (int k = 0; k < g.count; ++k) {                                                       \
      if (g.j[k].nx != N || g.j[k].ny % 2 || !g.j[k].zm) return hipErrorInvalidValue;         \
      g.j[k].nblk = (unsigned)(((long)g.j[k].ny * g.j[k].nz / 2 + LPW - 1) / LPW);            \
    }                                                                                         \
    hipLaunchKernelGGL((k_xinv_grp<N, TPL, LPW>), grp_grid(g), dim3(TPL * LPW), 0, st, g);    \
    return hipGetLastError();                                                                 \
  }
    PF_FOR_FFT_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_xfwd<double>(int, int, const double *, double *, size_t,
                                        const cplx<double> *, double *, long, hipStream_t, int,
                                        const cplx<double> *, int);
template hipError_t launch_xfwd<float>(int, int, const double *, float *, size_t,
                                       const cplx<double> *, double *, long, hipStream_t, int,
                                       const cplx<double> *, int);
template hipError_t launch_yfwd<double>(int, int, int, double *, size_t, const cplx<double> *,
                                        const cplx<double> *, int, hipStream_t, bool, int);
template hipError_t launch_yfwd<float>(int, int, int, float *, size_t, const cplx<double> *,
                                       const cplx<double> *, int, hipStream_t, bool, int);
template hipError_t launch_yinv<double>(int, int, int, double *, size_t, const cplx<double> *,
                                        const cplx<double> *, int, hipStream_t, bool, int);
template hipError_t launch_yinv<float>(int, int, int, float *, size_t, const cplx<double> *,
                                       const cplx<double> *, int, hipStream_t, bool, int);
template hipError_t launch_xinv<double, double>(int, int, const double *, size_t, double *,
                                                const cplx<double> *, const double *,
                                                const double *, double, long, hipStream_t,
                                                unsigned long long *, int, const cplx<double> *, int);
template hipError_t launch_xinv<float, double>(int, int, const float *, size_t, double *,
                                               const cplx<double> *, const double *, const float *,
                                               double, long, hipStream_t, unsigned long long *,
                                               int, const cplx<double> *, int);

}  // namespace pf
