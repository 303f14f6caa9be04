// Host side of the C ABI: plans, grid and coefficient tables, validation,
// launch sequences, stage timing and graph capture.
//
// Every table is built here in float64 from the grid definition (paper Sec.
// 2.1: staggered grid, uniform in x and y, stretched in z) and uploaded once
// per plan; the solves only enqueue kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pf_channel.h"
#include "pf_internal.hpp"

namespace {

thread_local std::string g_err;

pf_status fail(pf_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define PF_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(PF_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

// ------------------------------------------------------------------ grid
pf_status check_grid(const pf_grid *g, bool need_fft) {
  if (!g) return fail(PF_ERR_ARG, "grid is NULL");
  if (g->nz < 4) return fail(PF_ERR_ARG, "nz must be >= 4 (got %d)", g->nz);
  if (!(g->lz > 0.0) && !g->zf) return fail(PF_ERR_ARG, "lz must be > 0");
  if (!(g->beta >= 0.0) || !std::isfinite(g->beta)) return fail(PF_ERR_ARG, "beta must be finite and >= 0");
  if (g->ybc != PF_Y_PERIODIC && g->ybc != PF_Y_WALLS && g->ybc != PF_Y_DIRICHLET && g->ybc != PF_Y_FACES)
    return fail(PF_ERR_ARG, "ybc must be PF_Y_PERIODIC, PF_Y_WALLS, PF_Y_DIRICHLET or PF_Y_FACES (got %d)",
                g->ybc);
  if (g->xbc != PF_X_PERIODIC && g->xbc != PF_X_WALLS && g->xbc != PF_X_DIRICHLET && g->xbc != PF_X_FACES)
    return fail(PF_ERR_ARG, "xbc must be PF_X_PERIODIC, PF_X_WALLS, PF_X_DIRICHLET or PF_X_FACES (got %d)",
                g->xbc);
  if (need_fft) {
    if (!(g->lx > 0.0) || !(g->ly > 0.0)) return fail(PF_ERR_ARG, "lx, ly must be > 0");
#define PF_LEN_STR(N) " " #N
    // a field on the x (y) faces takes one transform of twice its length
    if (g->xbc == PF_X_FACES ? !pf::fft_size_supported(2 * g->nx) : !pf::fft_size_supported(g->nx))
      return fail(PF_ERR_UNSUPPORTED, "x length %d%s not built (built:" PF_FOR_FFT_SIZES(PF_LEN_STR) ")",
                  g->nx, g->xbc == PF_X_FACES ? " (faces: twice the length)" : "");
    if (g->ybc == PF_Y_FACES ? !pf::fft_size_supported_y(2 * g->ny) : !pf::fft_size_supported_y(g->ny))
      return fail(PF_ERR_UNSUPPORTED,
                  "y length %d%s not built (built:" PF_FOR_FFT_SIZES_Y(PF_LEN_STR) ")", g->ny,
                  g->ybc == PF_Y_FACES ? " (faces: twice the rows)" : "");
#undef PF_LEN_STR
  }
  if (g->zf) {
    for (int k = 0; k < g->nz; ++k)
      if (!(g->zf[k + 1] > g->zf[k]) || !std::isfinite(g->zf[k + 1]))
        return fail(PF_ERR_ARG, "zf must be finite and strictly increasing (k=%d)", k);
  }
  return PF_OK;
}

// faces: user array, or the tanh wall clustering
std::vector<double> faces_of(const pf_grid *g) {
  std::vector<double> zf(g->nz + 1);
  if (g->zf) {
    for (int k = 0; k <= g->nz; ++k) zf[k] = g->zf[k];
  } else {
    for (int k = 0; k <= g->nz; ++k) {
      if (g->beta == 0.0) {
        zf[k] = g->lz * (double)k / g->nz;
      } else {
        const long double t = std::tanh((long double)g->beta * (2.0L * k / g->nz - 1.0L)) /
                              std::tanh((long double)g->beta);
        zf[k] = (double)(0.5L * g->lz * (1.0L + t));
      }
    }
  }
  return zf;
}

// sign-normalised rows of -L_z: flux difference over the control volume
void zrows(const std::vector<double> &zf, int bc, std::vector<double> &al, std::vector<double> &ga,
           std::vector<double> &ex) {
  const int nz = (int)zf.size() - 1;
  std::vector<double> zc(nz), w(nz);
  for (int k = 0; k < nz; ++k) {
    zc[k] = 0.5 * (zf[k] + zf[k + 1]);
    w[k] = zf[k + 1] - zf[k];
  }
  if (bc == PF_BC_NEUMANN || bc == PF_BC_DIRICHLET_CENTRE) {
    al.assign(nz, 0.0); ga.assign(nz, 0.0); ex.assign(nz, 0.0);
    for (int k = 0; k < nz; ++k) {
      if (k > 0) al[k] = 1.0 / (w[k] * (zc[k] - zc[k - 1]));
      if (k < nz - 1) ga[k] = 1.0 / (w[k] * (zc[k + 1] - zc[k]));
    }
    if (bc == PF_BC_DIRICHLET_CENTRE) {
      // the wall value is reached over half a cell from the first centre
      ex[0] = 1.0 / (w[0] * (zc[0] - zf[0]));
      ex[nz - 1] = 1.0 / (w[nz - 1] * (zf[nz] - zc[nz - 1]));
    }
  } else {
    const int n = nz - 1;
    al.assign(n, 0.0); ga.assign(n, 0.0); ex.assign(n, 0.0);
    for (int u = 0; u < n; ++u) {
      const int k = u + 1;
      const double cv = zc[k] - zc[k - 1];
      const double dn = 1.0 / (cv * w[k - 1]), up = 1.0 / (cv * w[k]);
      if (u > 0) al[u] = dn; else ex[u] += dn;
      if (u < n - 1) ga[u] = up; else ex[u] += up;
    }
  }
}

// modified wavenumbers 4 sin^2(pi q / n) / dx^2 in packed slot order
std::vector<double> sigma_slots(int n, double len) {
  std::vector<double> s(n);
  const double dx = len / n;
  for (int sl = 0; sl < n; ++sl) {
    const int q = sl == 0 ? 0 : (sl == 1 ? n / 2 : sl / 2);
    const long double v = std::sin((long double)M_PI * q / n);
    s[sl] = (double)(4.0L * v * v / ((long double)dx * dx));
  }
  return s;
}

// exp(-2 pi i t / n), t = 0..n-1
template <typename T>
std::vector<T> twiddles(int n) {
  std::vector<T> tw(n);
  for (int t = 0; t < n; ++t) {
    const long double a = 2.0L * (long double)M_PI * t / n;
    tw[t].x = (decltype(tw[t].x))std::cos(a);
    tw[t].y = (decltype(tw[t].y))(-std::sin(a));
  }
  return tw;
}

// one device block holding all small tables of a plan
struct DevArena {
  char *base = nullptr;
  size_t used = 0, cap = 0;
  std::vector<char> host;
  template <typename T>
  size_t add(const T *src, size_t n) {
    const size_t off = (used + 255) & ~size_t(255);
    used = off + n * sizeof(T);
    if (host.size() < used) host.resize(used);
    if (src) std::memcpy(host.data() + off, src, n * sizeof(T));
    return off;
  }
  template <typename T>
  T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
};

struct Timing {
  bool on = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  double ms[PF_STAGE_COUNT] = {};
  int n[PF_STAGE_COUNT] = {};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void destroy() {
    for (auto &p : pending) { hipEventDestroy(p.second.first); hipEventDestroy(p.second.second); }
    for (auto e : pool) hipEventDestroy(e);
    pending.clear(); pool.clear();
  }
};

// launches a stage, bracketed by events when timing is on
template <typename F>
pf_status run_stage(Timing &tm, hipStream_t st, int stage, F &&f) {
  hipEvent_t a = nullptr, b = nullptr;
  if (tm.on) {
    a = tm.get(); b = tm.get();
    if (!a || !b) return fail(PF_ERR_DEVICE, "hipEventCreate failed");
    PF_HIP(hipEventRecord(a, st));
  }
  hipError_t e = f();
  if (e != hipSuccess) return fail(PF_ERR_DEVICE, "stage %d launch failed: %s", stage, hipGetErrorString(e));
  if (tm.on) {
    PF_HIP(hipEventRecord(b, st));
    tm.pending.push_back({stage, {a, b}});
  }
  return PF_OK;
}

pf_status timing_read(Timing &tm, hipStream_t st, double *ms, int32_t *count) {
  if (!ms || !count) return fail(PF_ERR_ARG, "NULL output array");
  PF_HIP(hipStreamSynchronize(st));
  for (auto &p : tm.pending) {
    float v = 0.f;
    PF_HIP(hipEventElapsedTime(&v, p.second.first, p.second.second));
    tm.ms[p.first] += v;
    tm.n[p.first] += 1;
    tm.pool.push_back(p.second.first);
    tm.pool.push_back(p.second.second);
  }
  tm.pending.clear();
  for (int s = 0; s < PF_STAGE_COUNT; ++s) {
    ms[s] = tm.ms[s];
    count[s] = tm.n[s];
    tm.ms[s] = 0.0;
    tm.n[s] = 0;
  }
  return PF_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + nb && y < x + na;
}

}  // namespace

// ====================================================================== plans
struct pf_poisson_plan {
  int nx, ny, nz;  // nz: planes of the field (nz - 1 for a face-centred Helmholtz)
  double lx, ly;
  int bc = PF_BC_NEUMANN;  // NEUMANN: pressure Poisson; DIRICHLET_*: 3-D Helmholtz
  double kappa = 0.0;      // 1/s of the 3-D Helmholtz, folded into the sx table
  int prec, nref;
  hipStream_t st;
  int zchunk;
  int xshape = 0, yshape = 0;  // launch shapes of the periodic x and y transforms
  DevArena ar;
  size_t o_zal, o_zga, o_zex, o_dzf, o_sx, o_sxb, o_sy, o_twx_d, o_twy_d, o_sums, o_sump,
      o_fbar, o_m, o_zm, o_p0m, o_rdzf, o_rdzc, o_ctw, o_ctwx;
  int ybc = PF_Y_PERIODIC, xbc = PF_X_PERIODIC;
  void *ws = nullptr;
  size_t ws_bytes = 0, ws_need = 0;
  unsigned long long *stat = nullptr;  // caller's pf_solve_status (device) or null
  double stat_tol = 1e-10;
  Timing tm;
  size_t npts() const { return (size_t)nx * ny * nz; }
  // plane stride of the float32 spectrum work array
  size_t sp32() const { return (size_t)nx * ny + pf::kPlanePad; }
};

struct pf_pcr_plan {
  int n, prec, M, P, steps, cw;
  bool staged;
  double s;
  hipStream_t st;
  std::vector<double> al, ga, ex;
  DevArena ar;
  size_t o_raw[3], o_d[11], o_f[11], o_m[4];  // rows of -L_z, double and float tables, M-matrix rows
  Timing tm;
};

struct pf_graph {
  hipGraph_t g;
  hipGraphExec_t ex;
};

namespace {

constexpr int kPcrTables = 11;

// lengths of the Step 1 tables (order of pf::HelmCoef): fa, bg, ib, ra, rc
// (P*M each); the cyclic-reduction multipliers k1, k2 (steps*2P); invd and
// the twisted elimination's tf, tb, ti (2P each)
size_t pcr_table_len(const pf_pcr_plan &pl, int t) {
  const size_t np = (size_t)pl.P * pl.M, nr = 2 * (size_t)pl.P;
  return t < 5 ? np : (t < 7 ? (size_t)pl.steps * nr : nr);
}

// Lays out and allocates the plan's device tables: the rows of -L_z
// (padded with zero rows, which become identity rows of I - s L_z), the
// float64 and float32 Step 1 tables and the M-matrix rows; uploads the rows.
pf_status pcr_alloc(pf_pcr_plan *pl) {
  const size_t np = (size_t)pl->P * pl->M;
  std::vector<double> al(np, 0.0), ga(np, 0.0), ex(np, 0.0);
  std::copy(pl->al.begin(), pl->al.end(), al.begin());
  std::copy(pl->ga.begin(), pl->ga.end(), ga.begin());
  std::copy(pl->ex.begin(), pl->ex.end(), ex.begin());
  pl->ar = DevArena();
  pl->o_raw[0] = pl->ar.add(al.data(), np);
  pl->o_raw[1] = pl->ar.add(ga.data(), np);
  pl->o_raw[2] = pl->ar.add(ex.data(), np);
  for (int t = 0; t < kPcrTables; ++t) pl->o_d[t] = pl->ar.add<double>(nullptr, pcr_table_len(*pl, t));
  for (int t = 0; t < kPcrTables; ++t) pl->o_f[t] = pl->ar.add<float>(nullptr, pcr_table_len(*pl, t));
  for (int t = 0; t < 4; ++t) pl->o_m[t] = pl->ar.add<double>(nullptr, np);
  pl->ar.cap = pl->ar.used;
  PF_HIP(hipMalloc((void **)&pl->ar.base, pl->ar.cap));
  PF_HIP(hipMemcpy(pl->ar.base, pl->ar.host.data(), pl->ar.used, hipMemcpyHostToDevice));
  return PF_OK;
}

// Algorithm 2, Step 1 for the plan's s, enqueued on stream st (a kernel:
// no host work, no copy, capturable).
pf_status pcr_recompute(pf_pcr_plan *pl, double s, hipStream_t st) {
  pf::PcrPrep p;
  p.al = pl->ar.at<double>(pl->o_raw[0]);
  p.ga = pl->ar.at<double>(pl->o_raw[1]);
  p.ex = pl->ar.at<double>(pl->o_raw[2]);
  for (int t = 0; t < kPcrTables; ++t) {
    p.d[t] = pl->ar.at<double>(pl->o_d[t]);
    p.f[t] = pl->ar.at<float>(pl->o_f[t]);
  }
  p.mA = pl->ar.at<double>(pl->o_m[0]);
  p.mG = pl->ar.at<double>(pl->o_m[1]);
  p.mE = pl->ar.at<double>(pl->o_m[2]);
  p.mD = pl->ar.at<double>(pl->o_m[3]);
  p.n = pl->n;
  p.P = pl->P;
  p.M = pl->M;
  p.steps = pl->steps;
  hipError_t e = pf::launch_pcr_prepare(p, s, st);
  if (e != hipSuccess) return fail(PF_ERR_DEVICE, "Step 1 kernel: %s", hipGetErrorString(e));
  return PF_OK;
}

pf::HelmCoef helm_coef(const pf_pcr_plan *pl) {
  pf::HelmCoef c;
  const size_t *o = pl->prec == PF_FP64 ? pl->o_d : pl->o_f;
  c.fa = pl->ar.base + o[0];
  c.bg = pl->ar.base + o[1];
  c.ib = pl->ar.base + o[2];
  c.ra = pl->ar.base + o[3];
  c.rc = pl->ar.base + o[4];
  c.k1 = pl->ar.base + o[5];
  c.k2 = pl->ar.base + o[6];
  c.invd = pl->ar.base + o[7];
  c.tf = pl->ar.base + o[8];
  c.tb = pl->ar.base + o[9];
  c.ti = pl->ar.base + o[10];
  c.al = pl->ar.at<double>(pl->o_m[0]);
  c.ga = pl->ar.at<double>(pl->o_m[1]);
  c.dg = pl->ar.at<double>(pl->o_m[3]);
  c.n = pl->n;
  c.P = pl->P;
  c.steps = pl->steps;
  return c;
}

// rows per thread of the Poisson z solve; a column of up to 64 chunks of
// 16 rows fits a 512-thread workgroup of 8 columns
constexpr int kZChunk = 16;
int zpad(int nz) { return (nz + kZChunk - 1) / kZChunk * kZChunk; }

}  // namespace

// ====================================================================== ABI
extern "C" {

const char *pf_last_error(void) { return g_err.c_str(); }
int32_t pf_abi_version(void) { return 3; }

pf_status pf_grid_faces(const pf_grid *g, double *zf_out) {
  pf_status s = check_grid(g, false);
  if (s) return s;
  if (!zf_out) return fail(PF_ERR_ARG, "zf_out is NULL");
  std::vector<double> zf = faces_of(g);
  std::memcpy(zf_out, zf.data(), zf.size() * sizeof(double));
  return PF_OK;
}

pf_status pf_zop_rows(const pf_grid *g, int32_t bc, double *alpha, double *gamma, double *excess) {
  pf_status s = check_grid(g, false);
  if (s) return s;
  if (bc < 0 || bc > 2) return fail(PF_ERR_ARG, "unknown boundary family %d", bc);
  if (!alpha || !gamma || !excess) return fail(PF_ERR_ARG, "NULL output array");
  std::vector<double> al, ga, ex;
  zrows(faces_of(g), bc, al, ga, ex);
  std::memcpy(alpha, al.data(), al.size() * 8);
  std::memcpy(gamma, ga.data(), ga.size() * 8);
  std::memcpy(excess, ex.data(), ex.size() * 8);
  return PF_OK;
}

// The pressure Poisson plan (bc NEUMANN, s = 0) and the 3-D Helmholtz plan
// (bc DIRICHLET_CENTRE or _FACE, s > 0) share the machinery: the Helmholtz
// per mode is the same z system with its Dirichlet rows and 1/s added to
// the shift, and has no singular column.
static pf_status channel_plan(pf_poisson_plan **out, const pf_grid *g, int32_t precision,
                              int32_t n_refine, void *stream, size_t *workspace_bytes, int bc,
                              double hs) {
  if (!out) return fail(PF_ERR_ARG, "out is NULL");
  *out = nullptr;
  pf_status s = check_grid(g, true);
  if (s) return s;
  if (precision < PF_FP64 || precision > PF_FP32_REFINE) return fail(PF_ERR_ARG, "unknown precision %d", precision);
  if (precision == PF_FP32_REFINE && (n_refine < 0 || n_refine > 1))
    return fail(PF_ERR_UNSUPPORTED, "n_refine must be 0 or 1 (got %d)", n_refine);
  if (g->nz > 1024) return fail(PF_ERR_UNSUPPORTED, "nz=%d too large for the z solve (max 1024)", g->nz);
  if ((g->ybc == PF_Y_FACES || g->xbc == PF_X_FACES) && bc == PF_BC_NEUMANN)
    return fail(PF_ERR_UNSUPPORTED, "PF_Y_FACES / PF_X_FACES place a velocity component on the faces: "
                                    "helmholtz3d_plan only");
  {
    // a y workgroup takes 2*LPW adjacent x slots of every row
    const int nyt = g->ybc == PF_Y_FACES ? 2 * g->ny : g->ny;
    const int lpw = precision == PF_FP64 ? pf::y_lpw<double>(nyt) : pf::y_lpw<float>(nyt);
    if (g->nx % (2 * lpw))
      return fail(PF_ERR_UNSUPPORTED, "nx=%d must be a multiple of %d for the y transforms of this grid "
                                      "and precision", g->nx, 2 * lpw);
  }
  const int nzu = bc == PF_BC_DIRICHLET_FACE ? g->nz - 1 : g->nz;  // planes of the field
  int zc = pf::zsolve_default_variant(g->nx, nzu, precision == PF_FP64);
  if (const char *ev = std::getenv("PF_ZSOLVE_VARIANT")) {
    const int v = std::atoi(ev);
    if (pf::zsolve_variant_fits(v, g->nx, nzu, precision == PF_FP64 ? 8 : 4)) zc = v;
  }
  if (zc < 0) return fail(PF_ERR_UNSUPPORTED, "no z-solve shape fits nx=%d nz=%d", g->nx, nzu);
  auto *pl = new pf_poisson_plan();
  pl->nx = g->nx; pl->ny = g->ny; pl->nz = nzu;
  pl->lx = g->lx; pl->ly = g->ly;
  pl->bc = bc;
  pl->ybc = g->ybc;
  pl->xbc = g->xbc;
  pl->kappa = bc == PF_BC_NEUMANN ? 0.0 : 1.0 / hs;
  pl->prec = precision;
  pl->nref = precision == PF_FP32_REFINE ? n_refine : 0;
  if (precision == PF_FP32_REFINE && n_refine == 0) pl->prec = PF_FP32;
  pl->st = (hipStream_t)stream;
  pl->zchunk = zc;
  std::vector<double> zf = faces_of(g), al, ga, ex;
  zrows(zf, bc, al, ga, ex);
  // identity rows pad the z tables to whole chunks
  al.resize(zpad(nzu), 0.0);
  ga.resize(zpad(nzu), 0.0);
  ex.resize(zpad(nzu), 1.0);
  std::vector<double> dzf(g->nz), rdzf(g->nz), rdzc(g->nz - 1);
  for (int k = 0; k < g->nz; ++k) dzf[k] = zf[k + 1] - zf[k];
  // the projection's metrics: 1/dzf per cell, 1/dzc per interior face
  for (int k = 0; k < g->nz; ++k) rdzf[k] = 1.0 / dzf[k];
  for (int k = 0; k + 1 < g->nz; ++k) rdzc[k] = 2.0 / (zf[k + 2] - zf[k]);
  // y: the packed slots of x slots 0 and 1, then the complex modes 0..ny-1
  // of every other slot pair. With y walls every slot pair holds the cosine
  // modes q = 0..ny-1 in natural order, wavenumber 4 sin^2(pi q / 2 ny) / dy^2
  // (zero-gradient walls), or the sine modes, 4 sin^2(pi (q + 1) / 2 ny) / dy^2
  // (value-zero walls); ctw[q] = exp(-i pi q / 2 ny) serves both transforms.
  auto sx = sigma_slots(g->nx, g->lx), sy = sigma_slots(g->ny, g->ly);
  // x walls: one real cosine (sine) mode per slot in natural order, the
  // wavenumbers 4 sin^2(pi (q + q0) / 2 nx) / dx^2; ctwx[q] = exp(-i pi q / 2 nx)
  std::vector<double2> ctwx;
  if (g->xbc != PF_X_PERIODIC) {
    const double dx = g->lx / g->nx;
    // x faces: the type-I sine modes q = 1..nx-1 in slots 0..nx-2, the value-
    // zero walls' formula (the last slot, the wall face, holds no mode)
    const int q0 = g->xbc == PF_X_DIRICHLET || g->xbc == PF_X_FACES ? 1 : 0;
    for (int q = 0; q < g->nx; ++q) {
      const long double v = std::sin((long double)M_PI * (q + q0) / (2.0L * g->nx));
      sx[q] = (double)(4.0L * v * v / ((long double)dx * dx));
      const long double a = (long double)M_PI * q / (2.0L * g->nx);
      ctwx.push_back(double2{(double)std::cos(a), (double)(-std::sin(a))});
    }
  }
  const std::vector<double> sxb = sx;  // without the Helmholtz shift kappa
  for (double &v : sx) v += pl->kappa;
  std::vector<double2> ctw;
  {
    const double dy = g->ly / g->ny;
    const bool walls = g->ybc != PF_Y_PERIODIC;
    // y faces: the type-I sine modes q = 1..ny-1 in rows 0..ny-2, the same
    // formula as the value-zero walls' sine modes (row ny - 1, the wall face,
    // holds no mode)
    const int q0 = g->ybc == PF_Y_DIRICHLET || g->ybc == PF_Y_FACES ? 1 : 0;
    if (walls) sy.clear();
    for (int h = 0; h < (walls ? 2 : 1); ++h)
      for (int m = 0; m < g->ny; ++m) {
        const long double v = std::sin((long double)M_PI * (m + q0) / ((walls ? 2 : 1) * g->ny));
        sy.push_back((double)(4.0L * v * v / ((long double)dy * dy)));
      }
    if (walls)
      for (int q = 0; q < g->ny; ++q) {
        const long double a = (long double)M_PI * q / (2.0L * g->ny);
        ctw.push_back(double2{(double)std::cos(a), (double)(-std::sin(a))});
      }
    // x walls with periodic y: every x slot is a real column whose y
    // spectrum is packed, so the z solve's second table (complex modes of
    // the other slot pairs) holds the packed wavenumbers as well
    if (!walls && g->xbc != PF_X_PERIODIC)
      for (int m = 0; m < g->ny; ++m) sy[g->ny + m] = sy[m];
  }
  auto twxd = twiddles<double2>(g->xbc == PF_X_FACES ? 2 * g->nx : g->nx),
       twyd = twiddles<double2>(g->ybc == PF_Y_FACES ? 2 * g->ny : g->ny);
  DevArena &A = pl->ar;
  pl->o_zal = A.add(al.data(), al.size());
  pl->o_zga = A.add(ga.data(), ga.size());
  pl->o_zex = A.add(ex.data(), ex.size());
  pl->o_dzf = A.add(dzf.data(), dzf.size());
  pl->o_sx = A.add(sx.data(), sx.size());
  pl->o_sxb = A.add(sxb.data(), sxb.size());
  pl->o_sy = A.add(sy.data(), sy.size());
  pl->o_twx_d = A.add(twxd.data(), twxd.size());
  pl->o_twy_d = A.add(twyd.data(), twyd.size());
  pl->o_ctw = ctw.empty() ? 0 : A.add(ctw.data(), ctw.size());
  pl->o_ctwx = ctwx.empty() ? 0 : A.add(ctwx.data(), ctwx.size());
  // per-plane buffers; fbar and zm stay zero for the Helmholtz (no zero mode)
  pl->o_sums = A.add<double>(nullptr, (size_t)g->ny * nzu);
  pl->o_sump = A.add<double>(nullptr, (size_t)g->ny * nzu);
  pl->o_fbar = A.add<double>(nullptr, (size_t)nzu);
  pl->o_m = A.add<double>(nullptr, (size_t)nzu);
  pl->o_zm = A.add<double>(nullptr, (size_t)nzu);
  pl->o_p0m = A.add<double>(nullptr, (size_t)nzu);
  pl->o_rdzf = A.add(rdzf.data(), rdzf.size());
  pl->o_rdzc = A.add(rdzc.data(), rdzc.size());
  A.cap = A.used;
  hipError_t e = hipMalloc((void **)&A.base, A.cap);
  if (e == hipSuccess) e = hipMemcpy(A.base, A.host.data(), A.used, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (A.base) (void)hipFree(A.base);
    delete pl;
    return fail(PF_ERR_DEVICE, "plan tables: %s", hipGetErrorString(e));
  }
  const size_t N = pl->npts();
  // float32: the padded spectrum; float32 + refinement: the iterate's and
  // the correction's padded spectra
  const size_t S = pl->sp32() * (size_t)pl->nz;
  pl->ws_need = pl->prec == PF_FP64 ? 0 : (pl->prec == PF_FP32 ? 4 * S : 8 * S);
  if (workspace_bytes) *workspace_bytes = pl->ws_need;
  *out = pl;
  return PF_OK;
}

pf_status poisson_plan(pf_poisson_plan **out, const pf_grid *g, int32_t precision, int32_t n_refine,
                       void *stream, size_t *workspace_bytes) {
  return channel_plan(out, g, precision, n_refine, stream, workspace_bytes, PF_BC_NEUMANN, 0.0);
}

pf_status helmholtz3d_plan(pf_poisson_plan **out, const pf_grid *g, int32_t bc, double s, int32_t precision,
                           int32_t n_refine, void *stream, size_t *workspace_bytes) {
  if (out) *out = nullptr;
  if (bc != PF_BC_DIRICHLET_CENTRE && bc != PF_BC_DIRICHLET_FACE)
    return fail(PF_ERR_ARG, "bc must be PF_BC_DIRICHLET_CENTRE or PF_BC_DIRICHLET_FACE (got %d)", bc);
  if (!(s > 0.0) || !std::isfinite(s)) return fail(PF_ERR_ARG, "s must be finite and > 0");
  return channel_plan(out, g, precision, n_refine, stream, workspace_bytes, bc, s);
}

pf_status helmholtz3d_update(pf_poisson_plan *pl, double s) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  if (pl->bc == PF_BC_NEUMANN) return fail(PF_ERR_ARG, "not a Helmholtz plan");
  if (!(s > 0.0) || !std::isfinite(s)) return fail(PF_ERR_ARG, "s must be finite and > 0");
  // the shifted x-slot table is rebuilt by a kernel on the plan's stream
  // from the unshifted one (no host staging: capturable, and several
  // updates may be queued); later solves take kappa as a launch argument
  const double kappa = 1.0 / s;
  hipError_t e = pf::launch_shift_add(pl->ar.at<double>(pl->o_sxb), pl->ar.at<double>(pl->o_sx), pl->nx,
                                      kappa, pl->st);
  if (e != hipSuccess) return fail(PF_ERR_DEVICE, "helmholtz3d_update: %s", hipGetErrorString(e));
  pl->kappa = kappa;
  return PF_OK;
}

pf_status poisson_set_workspace(pf_poisson_plan *pl, void *ws, size_t bytes) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  if (bytes < pl->ws_need) return fail(PF_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, pl->ws_need);
  if (pl->ws_need && !ws) return fail(PF_ERR_WORKSPACE, "workspace is NULL");
  if (ws && ((uintptr_t)ws & 255)) return fail(PF_ERR_ARG, "workspace must be 256-byte aligned");
  pl->ws = ws;
  pl->ws_bytes = bytes;
  return PF_OK;
}

pf_status poisson_set_stream(pf_poisson_plan *pl, void *stream) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  pl->st = (hipStream_t)stream;
  return PF_OK;
}

static pf_status poisson_check_solve(pf_poisson_plan *pl, const double *rhs, double *p) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  if (!rhs || !p) return fail(PF_ERR_ARG, "rhs and p must be device pointers");
  const size_t nb = pl->npts() * sizeof(double);
  if (overlaps(rhs, nb, p, nb)) return fail(PF_ERR_ARG, "p must not overlap rhs");
  if (pl->ws_need) {
    if (!pl->ws || pl->ws_bytes < pl->ws_need)
      return fail(PF_ERR_WORKSPACE, "workspace of %zu bytes required (poisson_set_workspace)", pl->ws_need);
    if (overlaps(pl->ws, pl->ws_need, p, nb) || overlaps(pl->ws, pl->ws_need, rhs, nb))
      return fail(PF_ERR_ARG, "workspace overlaps rhs or p");
  }
  if (((uintptr_t)rhs & 15) || ((uintptr_t)p & 15)) return fail(PF_ERR_ARG, "rhs and p must be 16-byte aligned");
  return PF_OK;
}

// With div, the right-hand side is D u* / gdt formed in the first x pass
// (rhs unused); for the float32 refinement f is stashed in p, which the
// residual reads before the last pass overwrites it.
static pf_status poisson_enqueue_plain(pf_poisson_plan *pl, const double *rhs, double *p, hipStream_t st,
                                       const pf::DivArgs *div, bool helm, double oscale, void *ws);
static pf_status poisson_enqueue_refined(pf_poisson_plan *pl, const double *rhs, double *p, hipStream_t st,
                                         const pf::DivArgs *div, bool helm, double oscale, void *ws);

#define STAGE(id, expr)                                      \
  if ((s = run_stage(tm, st, id, [&]() { return (expr); }))) \
    return s;

// ws: the float32 work arrays (the plan's workspace, or the static scratch
// of poisson_solve_noalloc)
static pf_status poisson_enqueue(pf_poisson_plan *pl, const double *rhs, double *p, hipStream_t st,
                                 const pf::DivArgs *div = nullptr, void *ws = nullptr) {
  if (!ws) ws = pl->ws;
  // the 3-D Helmholtz: no singular mode (zm stays zero, added as a no-op),
  // and the chain solves (L - kappa) u' = r, so u = -kappa u'. Value-zero y
  // walls: no singular mode either (nothing projected, no pin)
  // the y and x inverses leave the factors ny and nx (2 ny, 2 nx for the
  // type-I sine transform of a field on the y, x faces)
  const double scale = 1.0 / ((double)pl->nx * pl->ny * (pl->ybc == PF_Y_FACES ? 2 : 1) *
                              (pl->xbc == PF_X_FACES ? 2 : 1));
  const bool helm = pl->bc != PF_BC_NEUMANN;
  const double oscale = helm ? -pl->kappa * scale : scale;
  const bool nozero = helm || pl->ybc == PF_Y_DIRICHLET || pl->xbc == PF_X_DIRICHLET;
  if (pl->stat) PF_HIP(pf::launch_status_reset(pl->stat, st));
  if (pl->prec != PF_FP32_REFINE) {
    pf_status s = poisson_enqueue_plain(pl, rhs, p, st, div, nozero, oscale, ws);
    if (!s && pl->stat) PF_HIP(pf::launch_status_final(pl->stat, pl->stat_tol, false, st));
    return s;
  }
  return poisson_enqueue_refined(pl, rhs, p, st, div, nozero, oscale, ws);
}

// float64, or float32 without a correction
static pf_status poisson_enqueue_plain(pf_poisson_plan *pl, const double *rhs, double *p, hipStream_t st,
                                       const pf::DivArgs *div, bool helm, double oscale, void *ws) {
  const int nx = pl->nx, ny = pl->ny, nz = pl->nz;
  const long lines = (long)ny * nz;
  const DevArena &A = pl->ar;
  const double *zal = A.at<double>(pl->o_zal), *zga = A.at<double>(pl->o_zga), *zex = A.at<double>(pl->o_zex);
  const double *dzf = A.at<double>(pl->o_dzf), *sx = A.at<double>(pl->o_sx), *sy = A.at<double>(pl->o_sy);
  double *sums = A.at<double>(pl->o_sums);
  double *fbar = A.at<double>(pl->o_fbar), *mm = A.at<double>(pl->o_m), *zm = A.at<double>(pl->o_zm);
  Timing &tm = pl->tm;
  pf_status s;
  if (pl->prec == PF_FP64) {
    const double2 *twx = A.at<double2>(pl->o_twx_d), *twy = A.at<double2>(pl->o_twy_d);
    const double2 *ctw = pl->ybc != PF_Y_PERIODIC ? A.at<double2>(pl->o_ctw) : nullptr;
    const double2 *ctwx = pl->xbc != PF_X_PERIODIC ? A.at<double2>(pl->o_ctwx) : nullptr;
    const int yw = pl->ybc, xw = pl->xbc;
    const bool xr = xw != PF_X_PERIODIC;
    const int xs = xw == PF_X_PERIODIC ? pl->xshape : 0, ys = yw == PF_Y_PERIODIC && !xr ? pl->yshape : 0;
    // the spectrum lives in p itself, dense
    const size_t sd = (size_t)nx * ny;
    STAGE(PF_STAGE_XFWD, div ? pf::launch_xfwd_div<double>(nx, ny, nz, *div, p, sd, twx, sums, st)
                             : pf::launch_xfwd<double>(nx, ny, rhs, p, sd, twx, sums, lines, st, xw, ctwx, xs));
    if (!helm) STAGE(PF_STAGE_ZERO_MODE, pf::launch_zero_mode(nx, ny, nz, sums, dzf, zal, zga, fbar, mm, st));
    STAGE(PF_STAGE_YFWD, pf::launch_yfwd<double>(nx, ny, nz, p, sd, twy, ctw, yw, st, xr, ys));
    STAGE(PF_STAGE_ZSOLVE, pf::launch_zsolve<double>(nx, ny, nz, p, sd, zal, zga, zex, sx, sy, pl->zchunk, st, xr));
    STAGE(PF_STAGE_YINV, pf::launch_yinv<double>(nx, ny, nz, p, sd, twy, ctw, yw, st, xr, ys));
    STAGE(PF_STAGE_XINV, (pf::launch_xinv<double, double>(nx, ny, p, sd, p, twx, helm ? zm : mm, nullptr, oscale,
                                                          lines, st, nullptr, xw, ctwx, xs)));
    return PF_OK;
  }
  const double2 *twx = A.at<double2>(pl->o_twx_d), *twy = A.at<double2>(pl->o_twy_d);
  const double2 *ctw = pl->ybc != PF_Y_PERIODIC ? A.at<double2>(pl->o_ctw) : nullptr;
  const double2 *ctwx = pl->xbc != PF_X_PERIODIC ? A.at<double2>(pl->o_ctwx) : nullptr;
  const int yw = pl->ybc, xw = pl->xbc;
  const bool xr = xw != PF_X_PERIODIC;
  const int xs = xw == PF_X_PERIODIC ? pl->xshape : 0, ys = yw == PF_Y_PERIODIC && !xr ? pl->yshape : 0;
  float *W0 = (float *)ws;
  const size_t sp = pl->sp32();
  if (pl->prec == PF_FP32) {
    STAGE(PF_STAGE_XFWD, div ? pf::launch_xfwd_div<float>(nx, ny, nz, *div, W0, sp, twx, sums, st)
                             : pf::launch_xfwd<float>(nx, ny, rhs, W0, sp, twx, sums, lines, st, xw, ctwx, xs));
    if (!helm) STAGE(PF_STAGE_ZERO_MODE, pf::launch_zero_mode(nx, ny, nz, sums, dzf, zal, zga, fbar, mm, st));
    STAGE(PF_STAGE_YFWD, pf::launch_yfwd<float>(nx, ny, nz, W0, sp, twy, ctw, yw, st, xr, ys));
    STAGE(PF_STAGE_ZSOLVE, pf::launch_zsolve<float>(nx, ny, nz, W0, sp, zal, zga, zex, sx, sy, pl->zchunk, st, xr));
    STAGE(PF_STAGE_YINV, pf::launch_yinv<float>(nx, ny, nz, W0, sp, twy, ctw, yw, st, xr, ys));
    STAGE(PF_STAGE_XINV_FINAL, (pf::launch_xinv<float, double>(nx, ny, W0, sp, p, twx, helm ? zm : mm, nullptr,
                                                               oscale, lines, st, nullptr, xw, ctwx, xs)));
    return PF_OK;
  }
  return fail(PF_ERR_ARG, "unexpected precision");
}

// float32 with one float64-residual correction
static pf_status poisson_enqueue_refined(pf_poisson_plan *pl, const double *rhs, double *p, hipStream_t st,
                                         const pf::DivArgs *div, bool helm, double oscale, void *ws) {
  const int nx = pl->nx, ny = pl->ny, nz = pl->nz;
  const long lines = (long)ny * nz;
  const DevArena &A = pl->ar;
  const double *zal = A.at<double>(pl->o_zal), *zga = A.at<double>(pl->o_zga), *zex = A.at<double>(pl->o_zex);
  const double *dzf = A.at<double>(pl->o_dzf), *sx = A.at<double>(pl->o_sx), *sy = A.at<double>(pl->o_sy);
  double *sums = A.at<double>(pl->o_sums), *sump = A.at<double>(pl->o_sump);
  double *fbar = A.at<double>(pl->o_fbar), *mm = A.at<double>(pl->o_m), *zm = A.at<double>(pl->o_zm);
  Timing &tm = pl->tm;
  pf_status s;
  const double2 *twx = A.at<double2>(pl->o_twx_d), *twy = A.at<double2>(pl->o_twy_d);
  const double2 *ctw = pl->ybc != PF_Y_PERIODIC ? A.at<double2>(pl->o_ctw) : nullptr;
  const double2 *ctwx = pl->xbc != PF_X_PERIODIC ? A.at<double2>(pl->o_ctwx) : nullptr;
  const int yw = pl->ybc, xw = pl->xbc;
  const bool xr = xw != PF_X_PERIODIC;
  const int xs = xw == PF_X_PERIODIC ? pl->xshape : 0, ys = yw == PF_Y_PERIODIC && !xr ? pl->yshape : 0;
  float *W0 = (float *)ws;
  const size_t sp = pl->sp32();
  // float32 solve without the zero mode, kept as its x spectrum W0 after the
  // y inverse; the float64 residual of the plane-mean-free problem formed in
  // x-spectral space into W1; the correction; one x inverse of W0 + W1 with
  // the zero mode, which is solved once, in float64, from the plane means of
  // f and shifted by the iterate's plane means
  float *W1 = W0 + sp * (size_t)nz;
  if (div) {
    pf::DivArgs d = *div;
    d.stash = p;
    STAGE(PF_STAGE_XFWD, pf::launch_xfwd_div<float>(nx, ny, nz, d, W0, sp, twx, sums, st));
    rhs = p;
  } else {
    STAGE(PF_STAGE_XFWD, pf::launch_xfwd<float>(nx, ny, rhs, W0, sp, twx, sums, lines, st, xw, ctwx, xs));
  }
  if (!helm) STAGE(PF_STAGE_ZERO_MODE, pf::launch_zero_mode(nx, ny, nz, sums, dzf, zal, zga, fbar, mm, st));
  STAGE(PF_STAGE_YFWD, pf::launch_yfwd<float>(nx, ny, nz, W0, sp, twy, ctw, yw, st, xr, ys));
  STAGE(PF_STAGE_ZSOLVE, pf::launch_zsolve<float>(nx, ny, nz, W0, sp, zal, zga, zex, sx, sy, pl->zchunk, st, xr));
  STAGE(PF_STAGE_YINV, pf::launch_yinv<float>(nx, ny, nz, W0, sp, twy, ctw, yw, st, xr, ys));
  const double idy2 = (double)ny * ny / (pl->ly * pl->ly);
  STAGE(PF_STAGE_XFWD_RESID,
        pf::launch_resid_spec(nx, ny, nz, rhs, fbar, W0, W1, sp, twx, sump, sx, zal, zga, zex, idy2,
                             pl->ybc, st, xw, ctwx, xs));
  if (!helm) STAGE(PF_STAGE_ZERO_MODE, pf::launch_zero_shift(nx, ny, nz, sump, mm, A.at<double>(pl->o_p0m), zm, st));
  STAGE(PF_STAGE_YFWD, pf::launch_yfwd<float>(nx, ny, nz, W1, sp, twy, ctw, yw, st, xr, ys));
  STAGE(PF_STAGE_ZSOLVE, pf::launch_zsolve<float>(nx, ny, nz, W1, sp, zal, zga, zex, sx, sy, pl->zchunk, st, xr));
  STAGE(PF_STAGE_YINV, pf::launch_yinv<float>(nx, ny, nz, W1, sp, twy, ctw, yw, st, xr, ys));
  STAGE(PF_STAGE_XINV_FINAL,
        (pf::launch_xinv<float, double>(nx, ny, W0, sp, p, twx, zm, W1, oscale, lines, st, pl->stat, xw,
                                        ctwx, xs)));
  if (pl->stat) PF_HIP(pf::launch_status_final(pl->stat, pl->stat_tol, true, st));
#undef STAGE
  return PF_OK;
}

pf_status poisson_set_status(pf_poisson_plan *pl, void *dev_status, double tol) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  if (!(tol >= 0.0) || std::isnan(tol)) return fail(PF_ERR_ARG, "tol must be >= 0");
  if ((uintptr_t)dev_status & 7) return fail(PF_ERR_ARG, "dev_status must be 8-byte aligned");
  pl->stat = reinterpret_cast<unsigned long long *>(dev_status);
  pl->stat_tol = tol;
  return PF_OK;
}

pf_status poisson_solve(pf_poisson_plan *pl, const double *rhs, double *p) {
  pf_status s = poisson_check_solve(pl, rhs, p);
  if (s) return s;
  if (pl->bc != PF_BC_NEUMANN) return fail(PF_ERR_ARG, "a 3-D Helmholtz plan: use helmholtz3d_solve");
  return poisson_enqueue(pl, rhs, p, pl->st);
}

// ------------------------------------------------- allocation-free solve
// Device scratch for callers that cannot allocate: one static array per GPU,
// reached through its device address (hipGetSymbolAddress, taken once per
// device on the first call there with that device current; the array's name
// in host code is only a host-side stand-in). It serves as the float32 work
// arrays of the solve; every call on a device shares it.
constexpr size_t kNoAllocScratch = size_t(320) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};
}  // namespace

static pf_status scratch_of_device(void **out) {
  int dev = 0;
  PF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(PF_ERR_UNSUPPORTED, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PF_ERR_DEVICE, "device scratch address: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PF_OK;
}

pf_status poisson_solve_noalloc(pf_poisson_plan *pl, const double *rhs, double *p) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  if (pl->bc != PF_BC_NEUMANN) return fail(PF_ERR_ARG, "a 3-D Helmholtz plan: use helmholtz3d_solve");
  if (!rhs || !p) return fail(PF_ERR_ARG, "rhs and p must be device pointers");
  const size_t nb = pl->npts() * sizeof(double);
  if (overlaps(rhs, nb, p, nb)) return fail(PF_ERR_ARG, "p must not overlap rhs");
  if (((uintptr_t)rhs & 15) || ((uintptr_t)p & 15)) return fail(PF_ERR_ARG, "rhs and p must be 16-byte aligned");
  if (pl->ws_need > kNoAllocScratch)
    return fail(PF_ERR_UNSUPPORTED, "the solve needs %zu bytes of scratch; the static scratch holds %zu",
                pl->ws_need, kNoAllocScratch);
  void *ws = nullptr;
  if (pl->ws_need) {
    pf_status s = scratch_of_device(&ws);
    if (s) return s;
    if (overlaps(ws, pl->ws_need, p, nb) || overlaps(ws, pl->ws_need, rhs, nb))
      return fail(PF_ERR_ARG, "rhs or p overlaps the static scratch");
  }
  return poisson_enqueue(pl, rhs, p, pl->st, nullptr, ws);
}

pf_status helmholtz3d_solve(pf_poisson_plan *pl, const double *r, double *u) {
  pf_status s = poisson_check_solve(pl, r, u);
  if (s) return s;
  if (pl->bc == PF_BC_NEUMANN) return fail(PF_ERR_ARG, "a Poisson plan: use poisson_solve");
  return poisson_enqueue(pl, r, u, pl->st);
}

pf_status poisson_project(pf_poisson_plan *pl, double *u, double *v, double *w, double *p, double *phi,
                          double gdt, double c) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  if (pl->bc != PF_BC_NEUMANN) return fail(PF_ERR_ARG, "poisson_project needs a Poisson plan");
  if (pl->ybc == PF_Y_DIRICHLET)
    return fail(PF_ERR_UNSUPPORTED, "poisson_project: the pressure takes periodic or zero-gradient y ends");
  if (pl->xbc == PF_X_DIRICHLET)
    return fail(PF_ERR_UNSUPPORTED, "poisson_project: the pressure takes periodic or zero-gradient x ends");
  if (!u || !v || !w || !p || !phi) return fail(PF_ERR_ARG, "u, v, w, p and phi must be device pointers");
  if (!(gdt > 0.0) || !std::isfinite(gdt)) return fail(PF_ERR_ARG, "gdt must be finite and > 0");
  if (!(c >= 0.0) || !std::isfinite(c)) return fail(PF_ERR_ARG, "c must be finite and >= 0");
  const size_t nb = pl->npts() * sizeof(double);
  const size_t nbw = (size_t)pl->nx * pl->ny * (pl->nz - 1) * sizeof(double);
  const void *ptr[5] = {u, v, w, p, phi};
  const size_t len[5] = {nb, nb, nbw, nb, nb};
  for (int a = 0; a < 5; ++a) {
    if ((uintptr_t)ptr[a] & 15) return fail(PF_ERR_ARG, "fields must be 16-byte aligned");
    for (int b = a + 1; b < 5; ++b)
      if (overlaps(ptr[a], len[a], ptr[b], len[b])) return fail(PF_ERR_ARG, "u, v, w, p, phi must not overlap");
    if (pl->ws_need && overlaps(pl->ws, pl->ws_need, ptr[a], len[a]))
      return fail(PF_ERR_ARG, "workspace overlaps a field");
  }
  if (pl->ws_need && (!pl->ws || pl->ws_bytes < pl->ws_need))
    return fail(PF_ERR_WORKSPACE, "workspace of %zu bytes required (poisson_set_workspace)", pl->ws_need);
  const DevArena &A = pl->ar;
  pf::DivArgs d;
  d.u = u;
  d.v = v;
  d.w = w;
  d.rdzf = A.at<double>(pl->o_rdzf);
  d.idx = pl->nx / pl->lx;
  d.idy = pl->ny / pl->ly;
  d.igdt = 1.0 / gdt;
  d.stash = nullptr;
  d.ywalls = pl->ybc == PF_Y_WALLS ? 1 : 0;
  d.xwalls = pl->xbc == PF_X_WALLS ? 1 : 0;
  d.ctwx = d.xwalls ? A.at<double2>(pl->o_ctwx) : nullptr;
  pf_status s = poisson_enqueue(pl, nullptr, phi, pl->st, &d);
  if (s) return s;
  return run_stage(pl->tm, pl->st, PF_STAGE_PROJECT, [&]() {
    return pf::launch_project(pl->nx, pl->ny, pl->nz, phi, u, v, w, p, A.at<double>(pl->o_zal),
                              A.at<double>(pl->o_zga), A.at<double>(pl->o_rdzc), gdt * d.idx,
                              gdt * d.idy, gdt, c, d.ywalls != 0, d.xwalls != 0, pl->st);
  });
}

}  // extern "C"

// Grouped batch: the plans that can share launches (float32 with one
// float64-residual correction, periodic x and y, a separator-form z solve)
// run stage by stage; each stage of all plans with the same kernel instance
// (transform length; z-solve shape and chunk count) is one launch of up to
// kMaxGroupJobs jobs. The per-plan zero-mode and status kernels run between.
namespace {
struct GroupKey {
  int a, b;
  bool operator==(const GroupKey &o) const { return a == o.a && b == o.b; }
};
// launches fn(key, jobs) for every group of the plans' jobs, in first-seen
// key order, splitting groups larger than kMaxGroupJobs
template <typename KeyFn, typename JobFn, typename LaunchFn>
hipError_t run_groups(const std::vector<int> &ids, KeyFn key, JobFn job, LaunchFn launch) {
  std::vector<GroupKey> keys;
  for (int t : ids) {
    const GroupKey k = key(t);
    bool seen = false;
    for (const GroupKey &q : keys) seen = seen || q == k;
    if (!seen) keys.push_back(k);
  }
  for (const GroupKey &k : keys) {
    pf::GJobs g{};
    for (int t : ids) {
      if (!(key(t) == k)) continue;
      g.j[g.count++] = job(t);
      if (g.count == pf::kMaxGroupJobs) {
        const hipError_t e = launch(k, g);
        if (e != hipSuccess) return e;
        g = pf::GJobs{};
      }
    }
    if (g.count) {
      const hipError_t e = launch(k, g);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}
}  // namespace

static bool poisson_groupable(const pf_poisson_plan *pl) {
  return pl->prec == PF_FP32_REFINE && pl->ybc == PF_Y_PERIODIC && pl->xbc == PF_X_PERIODIC &&
         pf::zsolve_variant_groups(pl->zchunk) && pl->xshape == 0 && pl->yshape == 0;
}

#define STAGE(id, expr)                                      \
  if ((s = run_stage(tm, st, id, [&]() { return (expr); }))) \
    return s;
static pf_status poisson_enqueue_grouped(pf_poisson_plan *const *plans, const double *const *rhs,
                                         double *const *p, const std::vector<int> &ids, hipStream_t st) {
  Timing &tm = plans[ids[0]]->tm;
  pf_status s;
  auto helm = [&](int t) { return plans[t]->bc != PF_BC_NEUMANN; };
  // the fields of job t: its tables and its two float32 work arrays
  auto base = [&](int t) {
    const pf_poisson_plan *pl = plans[t];
    const DevArena &A = pl->ar;
    pf::GJob J{};
    J.tw = A.at<double2>(pl->o_twx_d);
    J.zal = A.at<double>(pl->o_zal);
    J.zga = A.at<double>(pl->o_zga);
    J.zex = A.at<double>(pl->o_zex);
    J.sx = A.at<double>(pl->o_sx);
    J.sy = A.at<double>(pl->o_sy);
    J.sp = pl->sp32();
    J.nx = pl->nx;
    J.ny = pl->ny;
    J.nz = pl->nz;
    return J;
  };
  auto W0 = [&](int t) { return (float *)plans[t]->ws; };
  auto W1 = [&](int t) { return (float *)plans[t]->ws + plans[t]->sp32() * (size_t)plans[t]->nz; };
  auto kx = [&](int t) { return GroupKey{plans[t]->nx, 0}; };
  auto ky = [&](int t) { return GroupKey{plans[t]->ny, 0}; };
  auto kz = [&](int t) {
    const pf_poisson_plan *pl = plans[t];
    return GroupKey{pl->zchunk, pl->nz};
  };
  for (int t : ids)
    if (plans[t]->stat) PF_HIP(pf::launch_status_reset(plans[t]->stat, st));
  // x forward of f into W0, with the float64 line sums
  STAGE(PF_STAGE_XFWD, run_groups(ids, kx, [&](int t) {
          pf::GJob J = base(t);
          J.in = rhs[t];
          J.out = W0(t);
          J.sums = plans[t]->ar.at<double>(plans[t]->o_sums);
          return J;
        }, [&](GroupKey k, pf::GJobs &g) { return pf::launch_xfwd_grp(k.a, g, st); }));
  // the zero modes of the Poisson plans (the 3-D Helmholtz has none)
  std::vector<int> pois;
  for (int t : ids)
    if (!helm(t)) pois.push_back(t);
  auto kone = [&](int) { return GroupKey{0, 0}; };
  if (!pois.empty())
    STAGE(PF_STAGE_ZERO_MODE, run_groups(pois, kone, [&](int t) {
            pf::GJob J = base(t);
            const pf_poisson_plan *pl = plans[t];
            J.sums = pl->ar.at<double>(pl->o_sums);
            J.out = pl->ar.at<double>(pl->o_fbar);
            J.in2 = pl->ar.at<double>(pl->o_m);
            J.aux = pl->ar.at<double>(pl->o_dzf);
            return J;
          }, [&](GroupKey, pf::GJobs &g) { return pf::launch_zero_mode_grp(g, st); }));
  // y forward, z solve, y inverse of one work array
  auto yzy = [&](bool second) -> pf_status {
    auto wj = [&](int t) {
      pf::GJob J = base(t);
      J.tw = plans[t]->ar.at<double2>(plans[t]->o_twy_d);
      J.out = second ? W1(t) : W0(t);
      return J;
    };
    auto zj = [&](int t) {
      pf::GJob J = base(t);
      J.out = second ? W1(t) : W0(t);
      J.P = pf::zsolve_chunks(plans[t]->zchunk, plans[t]->nz);
      return J;
    };
    pf_status s2;
    if ((s2 = run_stage(tm, st, PF_STAGE_YFWD, [&]() {
           return run_groups(ids, ky, wj, [&](GroupKey k, pf::GJobs &g) { return pf::launch_yfwd_grp(k.a, g, st); });
         })))
      return s2;
    if ((s2 = run_stage(tm, st, PF_STAGE_ZSOLVE, [&]() {
           return run_groups(ids, kz, zj, [&](GroupKey k, pf::GJobs &g) { return pf::launch_zsolve_grp(k.a, g, st); });
         })))
      return s2;
    return run_stage(tm, st, PF_STAGE_YINV, [&]() {
      return run_groups(ids, ky, wj, [&](GroupKey k, pf::GJobs &g) { return pf::launch_yinv_grp(k.a, g, st); });
    });
  };
  if ((s = yzy(false))) return s;
  // the float64 residual of the iterate W0 into W1
  STAGE(PF_STAGE_XFWD_RESID, run_groups(ids, kx, [&](int t) {
          pf::GJob J = base(t);
          const pf_poisson_plan *pl = plans[t];
          J.in = rhs[t];
          J.in2 = W0(t);
          J.out = W1(t);
          J.zm = pl->ar.at<double>(pl->o_fbar);
          J.sums = pl->ar.at<double>(pl->o_sump);
          J.idy2 = (double)pl->ny * pl->ny / (pl->ly * pl->ly);
          return J;
        }, [&](GroupKey k, pf::GJobs &g) { return pf::launch_resid_grp(k.a, g, st); }));
  if (!pois.empty())
    STAGE(PF_STAGE_ZERO_MODE, run_groups(pois, kone, [&](int t) {
            pf::GJob J = base(t);
            const pf_poisson_plan *pl = plans[t];
            J.sums = pl->ar.at<double>(pl->o_sump);
            J.out = pl->ar.at<double>(pl->o_p0m);
            J.in2 = pl->ar.at<double>(pl->o_m);
            J.zm = pl->ar.at<double>(pl->o_zm);
            return J;
          }, [&](GroupKey, pf::GJobs &g) { return pf::launch_zero_shift_grp(g, st); }));
  if ((s = yzy(true))) return s;
  // one x inverse of W0 + W1 with the zero-mode profile
  STAGE(PF_STAGE_XINV_FINAL, run_groups(ids, kx, [&](int t) {
          pf::GJob J = base(t);
          const pf_poisson_plan *pl = plans[t];
          const double scale = 1.0 / ((double)pl->nx * pl->ny);  // periodic y only
          J.in = W0(t);
          J.in2 = W1(t);
          J.out = p[t];
          J.zm = pl->ar.at<double>(pl->o_zm);
          J.scale = helm(t) ? -pl->kappa * scale : scale;
          J.stat = pl->stat;
          return J;
        }, [&](GroupKey k, pf::GJobs &g) { return pf::launch_xinv_grp(k.a, g, st); }));
  for (int t : ids)
    if (plans[t]->stat) PF_HIP(pf::launch_status_final(plans[t]->stat, plans[t]->stat_tol, true, st));
  return PF_OK;
}

#undef STAGE

extern "C" {

pf_status poisson_solve_batched(int32_t count, pf_poisson_plan *const *plans, const double *const *rhs,
                                double *const *p) {
  if (count < 0 || (count > 0 && (!plans || !rhs || !p))) return fail(PF_ERR_ARG, "bad batch arguments");
  for (int t = 0; t < count; ++t) {
    pf_status s = poisson_check_solve(plans[t], rhs[t], p[t]);
    if (s) return s;
    for (int u = 0; u < t; ++u)
      if (plans[u] == plans[t]) return fail(PF_ERR_ARG, "entries %d and %d share a plan", u, t);
  }
  if (count == 0) return PF_OK;
  // the batch runs in one stream: a problem's output may not feed another
  for (int a = 0; a < count; ++a)
    for (int b = 0; b < count; ++b) {
      const size_t na = plans[a]->npts() * sizeof(double), nb = plans[b]->npts() * sizeof(double);
      if (a != b && overlaps(p[a], na, p[b], nb)) return fail(PF_ERR_ARG, "outputs %d and %d overlap", a, b);
      if (a != b && overlaps(p[a], na, rhs[b], nb)) return fail(PF_ERR_ARG, "output %d overlaps input %d", a, b);
      if (a != b && plans[a]->ws_need && plans[b]->ws_need &&
          overlaps(plans[a]->ws, plans[a]->ws_need, plans[b]->ws, plans[b]->ws_need))
        return fail(PF_ERR_ARG, "workspaces %d and %d overlap", a, b);
      if (a != b && plans[a]->ws_need &&
          (overlaps(plans[a]->ws, plans[a]->ws_need, rhs[b], nb) || overlaps(plans[a]->ws, plans[a]->ws_need, p[b], nb)))
        return fail(PF_ERR_ARG, "workspace %d overlaps the fields of entry %d", a, b);
    }
  const hipStream_t st = plans[0]->st;
  std::vector<int> grouped;
  for (int t = 0; t < count; ++t)
    if (poisson_groupable(plans[t])) grouped.push_back(t);
  if (!grouped.empty()) {
    pf_status s = poisson_enqueue_grouped(plans, rhs, p, grouped, st);
    if (s) return s;
  }
  for (int t = 0; t < count; ++t) {
    if (poisson_groupable(plans[t])) continue;
    pf_status s = poisson_enqueue(plans[t], rhs[t], p[t], st);
    if (s) return s;
  }
  return PF_OK;
}

pf_status poisson_destroy(pf_poisson_plan *pl) {
  if (!pl) return PF_OK;
  pl->tm.destroy();
  if (pl->ar.base) (void)hipFree(pl->ar.base);
  delete pl;
  return PF_OK;
}

// the transform shapes a plan can take: periodic directions only; the x
// shape covers the x forward, the x inverse and the residual, the y shape
// both y transforms
static bool transform_shape_fits(const pf_poisson_plan *pl, int stage, int v) {
  if (v < 0 || v >= pf::kTransformShapes) return false;
  if (v == 0) return true;
  if (stage == PF_STAGE_XFWD)
    return pl->xbc == PF_X_PERIODIC && pf::xfwd_shape(pl->nx, v).ok && pf::xinv_shape(pl->nx, v).ok &&
           pf::resid_shape(pl->nx, v).ok && pl->ny % (2 * pf::resid_shape(pl->nx, v).lpw) == 0;
  const pf::TShape h = pl->prec == PF_FP64 ? pf::y_shape<double>(pl->ny, v == pf::kYPersistShape ? 0 : v)
                                            : pf::y_shape<float>(pl->ny, v == pf::kYPersistShape ? 0 : v);
  return pl->xbc == PF_X_PERIODIC && pl->ybc == PF_Y_PERIODIC && h.ok && pl->nx % (2 * h.lpw) == 0;
}

pf_status poisson_variant_count(pf_poisson_plan *pl, int32_t stage, int32_t *count) {
  if (!pl || !count) return fail(PF_ERR_ARG, "NULL argument");
  if (stage == PF_STAGE_XFWD || stage == PF_STAGE_YFWD) {
    *count = pf::kTransformShapes;
    return PF_OK;
  }
  if (stage != PF_STAGE_ZSOLVE) return fail(PF_ERR_UNSUPPORTED, "stage %d has no variants", stage);
  *count = pf::zsolve_variant_count();
  return PF_OK;
}

pf_status poisson_set_variant(pf_poisson_plan *pl, int32_t stage, int32_t variant) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  if (stage == PF_STAGE_XFWD || stage == PF_STAGE_YFWD) {
    if (!transform_shape_fits(pl, stage, variant))
      return fail(PF_ERR_UNSUPPORTED, "transform shape %d does not fit stage %d of this plan", variant, stage);
    (stage == PF_STAGE_XFWD ? pl->xshape : pl->yshape) = variant;
    return PF_OK;
  }
  if (stage != PF_STAGE_ZSOLVE) return fail(PF_ERR_UNSUPPORTED, "stage %d has no variants", stage);
  if (!pf::zsolve_variant_fits(variant, pl->nx, pl->nz, pl->prec == PF_FP64 ? 8 : 4))
    return fail(PF_ERR_UNSUPPORTED, "z-solve variant %d does not fit nx=%d nz=%d", variant, pl->nx, pl->nz);
  pl->zchunk = variant;
  return PF_OK;
}

pf_status poisson_get_variant(pf_poisson_plan *pl, int32_t stage, int32_t *variant) {
  if (!pl || !variant) return fail(PF_ERR_ARG, "NULL argument");
  if (stage == PF_STAGE_XFWD || stage == PF_STAGE_YFWD) {
    *variant = stage == PF_STAGE_XFWD ? pl->xshape : pl->yshape;
    return PF_OK;
  }
  if (stage != PF_STAGE_ZSOLVE) return fail(PF_ERR_UNSUPPORTED, "stage %d has no variants", stage);
  *variant = pl->zchunk;
  return PF_OK;
}

pf_status poisson_timing(pf_poisson_plan *pl, int32_t enable) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  pl->tm.on = enable != 0;
  return PF_OK;
}

pf_status poisson_timing_read(pf_poisson_plan *pl, double *ms, int32_t *count) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  return timing_read(pl->tm, pl->st, ms, count);
}

// ------------------------------------------------------------ Helmholtz
pf_status pcr_prepare(pf_pcr_plan **out, int32_t n, const double *alpha, const double *gamma,
                      const double *excess, double s, int32_t precision, int32_t chunk_rows, void *stream) {
  if (!out) return fail(PF_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n < 4) return fail(PF_ERR_ARG, "n must be >= 4 (got %d)", n);
  if (!alpha || !gamma || !excess) return fail(PF_ERR_ARG, "coefficient arrays must be host pointers");
  if (!(s >= 0.0) || !std::isfinite(s)) return fail(PF_ERR_ARG, "s must be finite and >= 0");
  if (precision < PF_FP64 || precision > PF_FP32_REFINE) return fail(PF_ERR_ARG, "unknown precision %d", precision);
  if (alpha[0] != 0.0 || gamma[n - 1] != 0.0) return fail(PF_ERR_ARG, "alpha[0] and gamma[n-1] must be 0");
  for (int r = 0; r < n; ++r)
    if (!(alpha[r] >= 0.0) || !(gamma[r] >= 0.0) || !(excess[r] >= 0.0) || !std::isfinite(alpha[r] + gamma[r] + excess[r]))
      return fail(PF_ERR_ARG, "row %d: alpha, gamma, excess must be finite and >= 0", r);
  int M = chunk_rows;
  if (M == 0) {
    M = 32;
    for (int c : {8, 16, 32})
      if ((n + c - 1) / c <= 16) { M = c; break; }
  }
  if (M != 8 && M != 16 && M != 32) return fail(PF_ERR_UNSUPPORTED, "chunk_rows must be 8, 16 or 32");
  const int P = (n + M - 1) / M;  // rows past n are identity padding
  if (P > 32) return fail(PF_ERR_UNSUPPORTED, "n=%d needs %d chunks of %d rows (max 32)", n, P, M);
  auto *pl = new pf_pcr_plan();
  pl->n = n; pl->prec = precision; pl->M = M; pl->P = P; pl->s = s;
  pl->steps = 0;
  while ((1 << pl->steps) < 2 * P) ++pl->steps;
  pl->cw = pf::helm_default_cw(P);
  pl->staged = false;
  if (const char *ev = std::getenv("PF_PCR_CW")) {
    const int c = std::atoi(ev);
    if ((c == 16 || c == 32 || c == 64) && c * P <= 1024) pl->cw = c;
  }
  if (const char *ev = std::getenv("PF_PCR_STAGED")) pl->staged = std::atoi(ev) != 0 && pl->cw * P <= 512;
  pl->st = (hipStream_t)stream;
  pl->al.assign(alpha, alpha + n);
  pl->ga.assign(gamma, gamma + n);
  pl->ex.assign(excess, excess + n);
  pf_status st = pcr_alloc(pl);
  if (!st) st = pcr_recompute(pl, s, pl->st);
  if (!st && hipStreamSynchronize(pl->st) != hipSuccess) st = fail(PF_ERR_DEVICE, "Step 1 kernel failed");
  if (st) {
    if (pl->ar.base) (void)hipFree(pl->ar.base);
    delete pl;
    return st;
  }
  *out = pl;
  return PF_OK;
}

pf_status pcr_prepare_rows(pf_pcr_plan **out, int32_t n, const double *lower, const double *diag,
                           const double *upper, double s, int32_t precision, int32_t chunk_rows, void *stream) {
  if (!out) return fail(PF_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n < 4) return fail(PF_ERR_ARG, "n must be >= 4 (got %d)", n);
  if (!lower || !diag || !upper) return fail(PF_ERR_ARG, "row arrays must be host pointers");
  if (lower[0] != 0.0 || upper[n - 1] != 0.0) return fail(PF_ERR_ARG, "lower[0] and upper[n-1] must be 0");
  // rows of L_z: lower, upper >= 0 and a diagonal no larger than -(lower +
  // upper); the excess -(lower + diag + upper) is clamped at zero within
  // rounding of the three terms
  std::vector<double> al(n), ga(n), ex(n);
  for (int r = 0; r < n; ++r) {
    const double A = lower[r], B = diag[r], C = upper[r];
    if (!std::isfinite(A) || !std::isfinite(B) || !std::isfinite(C))
      return fail(PF_ERR_ARG, "row %d is not finite", r);
    if (A < 0.0 || C < 0.0)
      return fail(PF_ERR_UNSUPPORTED, "row %d: negative off-diagonal of L_z (not an M-matrix form)", r);
    const double e = -(A + B + C);
    const double tol = 16.0 * 2.220446049250313e-16 * (A + std::fabs(B) + C);
    if (e < -tol)
      return fail(PF_ERR_UNSUPPORTED, "row %d: diagonal of -L_z below the off-diagonal sum (not an M-matrix)", r);
    al[r] = A;
    ga[r] = C;
    ex[r] = e > tol ? e : 0.0;
  }
  return pcr_prepare(out, n, al.data(), ga.data(), ex.data(), s, precision, chunk_rows, stream);
}

pf_status pcr_update_coef(pf_pcr_plan *pl, double s) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  if (!(s >= 0.0) || !std::isfinite(s)) return fail(PF_ERR_ARG, "s must be finite and >= 0");
  pl->s = s;
  return pcr_recompute(pl, s, pl->st);
}

pf_status pcr_set_shape(pf_pcr_plan *pl, int32_t chunk_rows, int32_t cw_in) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  const bool staged = cw_in < 0;
  const int cw = staged ? -cw_in : cw_in;
  const int M = chunk_rows;
  if (M != 8 && M != 16 && M != 32) return fail(PF_ERR_UNSUPPORTED, "chunk_rows must be 8, 16 or 32");
  if (cw != 16 && cw != 32 && cw != 64) return fail(PF_ERR_UNSUPPORTED, "columns per chunk must be 16, 32 or 64");
  const int P = (pl->n + M - 1) / M;
  if (P > 32 || P * cw > (staged ? 512 : 1024))
    return fail(PF_ERR_UNSUPPORTED, "%d chunks of %d columns exceed a workgroup", P, cw);
  PF_HIP(hipStreamSynchronize(pl->st));
  pl->staged = staged;
  char *old = pl->ar.base;
  pl->M = M;
  pl->P = P;
  pl->cw = cw;
  pl->steps = 0;
  while ((1 << pl->steps) < 2 * P) ++pl->steps;
  pf_status st = pcr_alloc(pl);
  if (!st) st = pcr_recompute(pl, pl->s, pl->st);
  if (!st && hipStreamSynchronize(pl->st) != hipSuccess) st = fail(PF_ERR_DEVICE, "Step 1 kernel failed");
  if (old) (void)hipFree(old);
  return st;
}

pf_status pcr_get_shape(pf_pcr_plan *pl, int32_t *chunk_rows, int32_t *cw) {
  if (!pl || !chunk_rows || !cw) return fail(PF_ERR_ARG, "NULL argument");
  *chunk_rows = pl->M;
  *cw = pl->staged ? -pl->cw : pl->cw;
  return PF_OK;
}

pf_status pcr_set_stream(pf_pcr_plan *pl, void *stream) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  pl->st = (hipStream_t)stream;
  return PF_OK;
}

// Validates a group of Helmholtz fields for one fused launch and fills its
// job table and launch shape.
struct HelmGroup {
  pf::HelmJob jobs[pf::kMaxHelmJobs];
  int count = 0, M = 0, cw = 1 << 30, prec = 0;
  bool staged = true;
};

static pf_status pcr_group(int32_t count, pf_pcr_plan *const *plans, void *const *fields, const int32_t *nx,
                           const int32_t *ny, HelmGroup &G) {
  if (count < 1 || count > pf::kMaxHelmJobs) return fail(PF_ERR_ARG, "count must be 1..%d", pf::kMaxHelmJobs);
  if (!plans || !fields || !nx || !ny) return fail(PF_ERR_ARG, "NULL argument array");
  pf::HelmJob *jobs = G.jobs;
  int M = 0, cw = 1 << 30;
  bool staged = true;
  for (int t = 0; t < count; ++t) {
    const pf_pcr_plan *pl = plans[t];
    if (!pl || !fields[t]) return fail(PF_ERR_ARG, "plan or field %d is NULL", t);
    if (nx[t] < 64 || nx[t] % 64 || ny[t] < 1) return fail(PF_ERR_ARG, "nx must be a positive multiple of 64, ny >= 1");
    if (pl->P * pl->cw > 1024) return fail(PF_ERR_ARG, "plan %d: chunk shape exceeds a workgroup", t);
    if (pl->M != plans[0]->M) return fail(PF_ERR_ARG, "batched plans must share chunk_rows");
    if (pl->prec != plans[0]->prec) return fail(PF_ERR_ARG, "batched plans must share precision");
    const size_t esz = pl->prec == PF_FP32 ? 4 : 8;
    if ((uintptr_t)fields[t] % esz) return fail(PF_ERR_ARG, "field %d misaligned", t);
    M = M > pl->M ? M : pl->M;
    cw = cw < pl->cw ? cw : pl->cw;
    staged = staged && pl->staged;
    jobs[t].field = fields[t];
    jobs[t].nx = nx[t];
    jobs[t].ny = ny[t];
    jobs[t].c = helm_coef(pl);
  }
  for (int t = 0; t < count; ++t)
    for (int u = t + 1; u < count; ++u) {
      const size_t a = (size_t)plans[t]->n * nx[t] * ny[t] * (plans[t]->prec == PF_FP32 ? 4 : 8);
      const size_t b = (size_t)plans[u]->n * nx[u] * ny[u] * (plans[u]->prec == PF_FP32 ? 4 : 8);
      if (overlaps(fields[t], a, fields[u], b)) return fail(PF_ERR_ARG, "fields %d and %d overlap", t, u);
    }
  G.count = count;
  G.M = M;
  G.cw = cw;
  G.staged = staged;
  G.prec = plans[0]->prec == PF_FP64 ? 0 : (plans[0]->prec == PF_FP32 ? 1 : 2);
  return PF_OK;
}

static pf_status pcr_enqueue(pf_pcr_plan *p0, const HelmGroup &G, hipStream_t st) {
  return run_stage(p0->tm, st, PF_STAGE_PCR_APPLY,
                   [&]() { return pf::launch_helm(G.prec, G.M, G.cw, G.staged, G.count, G.jobs, st); });
}

pf_status pcr_apply_batched(int32_t count, pf_pcr_plan *const *plans, void *const *fields, const int32_t *nx,
                            const int32_t *ny) {
  HelmGroup G;
  pf_status s = pcr_group(count, plans, fields, nx, ny, G);
  if (s) return s;
  return pcr_enqueue(plans[0], G, plans[0]->st);
}

pf_status pcr_apply(pf_pcr_plan *pl, void *field, int32_t nx, int32_t ny) {
  pf_pcr_plan *pls[1] = {pl};
  void *f[1] = {field};
  int32_t a[1] = {nx}, b[1] = {ny};
  return pcr_apply_batched(1, pls, f, a, b);
}

pf_status pcr_destroy(pf_pcr_plan *pl) {
  if (!pl) return PF_OK;
  pl->tm.destroy();
  if (pl->ar.base) (void)hipFree(pl->ar.base);
  delete pl;
  return PF_OK;
}

pf_status pcr_timing(pf_pcr_plan *pl, int32_t enable) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  pl->tm.on = enable != 0;
  return PF_OK;
}

pf_status pcr_timing_read(pf_pcr_plan *pl, double *ms, int32_t *count) {
  if (!pl) return fail(PF_ERR_ARG, "plan is NULL");
  return timing_read(pl->tm, pl->st, ms, count);
}

// ---------------------------------------------------------------- graphs
// ------------------------------------------------------------- task batch
// A pool of internal streams (default priority) and fork/join events per
// device, created on first use and kept until the process ends.
namespace {
constexpr int kMaxLanes = 8;
constexpr int kMaxTaskComps = 4;  // Helmholtz fields of one pf_task
struct Lanes {
  bool ready = false;
  hipStream_t s[kMaxLanes] = {};
  hipEvent_t fork = nullptr, join[kMaxLanes] = {};
};
constexpr int kMaxDevices = 64;
std::mutex g_lanes_mu;
Lanes g_lanes[kMaxDevices];
}  // namespace

static pf_status lanes_ready(int dev, Lanes *&L) {
  if (dev < 0 || dev >= kMaxDevices) return fail(PF_ERR_UNSUPPORTED, "device %d beyond the lane pool", dev);
  L = &g_lanes[dev];
  if (L->ready) return PF_OK;
  for (int l = 0; l < kMaxLanes; ++l) {
    PF_HIP(hipStreamCreateWithFlags(&L->s[l], hipStreamNonBlocking));
    PF_HIP(hipEventCreateWithFlags(&L->join[l], hipEventDisableTiming));
  }
  PF_HIP(hipEventCreateWithFlags(&L->fork, hipEventDisableTiming));
  L->ready = true;
  return PF_OK;
}

// Every task of a batch checked before anything is enqueued: its Poisson
// solve, its Helmholtz group (filled into groups[t]) and its footprint
// against every other task's (cost[t]: its points, for the lane balance).
static pf_status validate_tasks(int32_t count, const pf_task *tasks, std::vector<HelmGroup> &groups,
                                std::vector<double> &cost) {
  if (count < 0 || (count > 0 && !tasks)) return fail(PF_ERR_ARG, "bad batch arguments");
  groups.assign((size_t)count, HelmGroup{});
  cost.assign((size_t)count, 0.0);
  for (int t = 0; t < count; ++t) {
    const pf_task &T = tasks[t];
    if (T.poisson) {
      pf_status s = poisson_check_solve(T.poisson, T.rhs, T.p);
      if (s) return s;
      cost[t] += (double)T.poisson->npts();
    }
    if (T.ncomp < 0 || T.ncomp > kMaxTaskComps) return fail(PF_ERR_ARG, "task %d: ncomp must be 0..%d", t, kMaxTaskComps);
    if (!T.poisson && T.ncomp == 0) return fail(PF_ERR_ARG, "task %d is empty", t);
    if (T.ncomp) {
      pf_status s = pcr_group(T.ncomp, T.pcr, T.field, T.nx, T.ny, groups[t]);
      if (s) return s;
      for (int c = 0; c < T.ncomp; ++c) cost[t] += (double)T.pcr[c]->n * T.nx[c] * T.ny[c] / 3.0;
    }
  }
  // tasks run concurrently: no Poisson plan (its workspace and scratch
  // tables) may serve two tasks, and nothing a task writes may overlap what
  // another task reads or writes
  struct Range { const void *p; size_t n; int task; bool write; };
  std::vector<Range> rg;
  for (int t = 0; t < count; ++t) {
    const pf_task &T = tasks[t];
    if (T.poisson) {
      const size_t nb = T.poisson->npts() * sizeof(double);
      rg.push_back({T.rhs, nb, t, false});
      rg.push_back({T.p, nb, t, true});
      if (T.poisson->ws_need) rg.push_back({T.poisson->ws, T.poisson->ws_need, t, true});
      for (int u = 0; u < t; ++u)
        if (tasks[u].poisson == T.poisson) return fail(PF_ERR_ARG, "tasks %d and %d share a Poisson plan", u, t);
    }
    for (int c = 0; c < T.ncomp; ++c) {
      const size_t esz = T.pcr[c]->prec == PF_FP32 ? 4 : 8;
      rg.push_back({T.field[c], (size_t)T.pcr[c]->n * T.nx[c] * T.ny[c] * esz, t, true});
    }
  }
  for (size_t a = 0; a < rg.size(); ++a)
    for (size_t b = a + 1; b < rg.size(); ++b)
      if (rg[a].task != rg[b].task && (rg[a].write || rg[b].write) &&
          overlaps(rg[a].p, rg[a].n, rg[b].p, rg[b].n))
        return fail(PF_ERR_ARG, "tasks %d and %d overlap in device memory", rg[a].task, rg[b].task);
  return PF_OK;
}

pf_status pf_run_batched(int32_t count, const pf_task *tasks, int32_t lanes, void *stream) {
  if (lanes < 1 || lanes > kMaxLanes) return fail(PF_ERR_ARG, "lanes must be 1..%d", kMaxLanes);
  std::vector<HelmGroup> groups;
  std::vector<double> cost;
  pf_status vs = validate_tasks(count, tasks, groups, cost);
  if (vs) return vs;
  if (count == 0) return PF_OK;
  int dev = 0;
  PF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_lanes_mu);
  Lanes *L = nullptr;
  pf_status s = lanes_ready(dev, L);
  if (s) return s;
  hipStream_t origin = (hipStream_t)stream;
  const int nl = lanes < count ? lanes : count;
  PF_HIP(hipEventRecord(L->fork, origin));
  for (int l = 0; l < nl; ++l) PF_HIP(hipStreamWaitEvent(L->s[l], L->fork, 0));
  // largest tasks first, each to the least-loaded lane
  std::vector<int> order((size_t)count);
  for (int t = 0; t < count; ++t) order[t] = t;
  for (int a = 1; a < count; ++a)
    for (int b = a; b > 0 && cost[order[b]] > cost[order[b - 1]]; --b) std::swap(order[b], order[b - 1]);
  double load[kMaxLanes] = {};
  pf_status err = PF_OK;
  for (int t : order) {
    int l = 0;
    for (int u = 1; u < nl; ++u)
      if (load[u] < load[l]) l = u;
    load[l] += cost[t];
    const pf_task &T = tasks[t];
    if (!err && T.ncomp) err = pcr_enqueue(T.pcr[0], groups[t], L->s[l]);
    if (!err && T.poisson) err = poisson_enqueue(T.poisson, T.rhs, T.p, L->s[l]);
  }
  // join every lane back, also after a failed launch, so that a capture
  // on the origin stream stays well formed
  for (int l = 0; l < nl; ++l) {
    PF_HIP(hipEventRecord(L->join[l], L->s[l]));
    PF_HIP(hipStreamWaitEvent(origin, L->join[l], 0));
  }
  return err;
}

pf_status pf_graph_begin(void *stream) {
  if (!stream) return fail(PF_ERR_ARG, "capture needs a non-default stream");
  PF_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
  return PF_OK;
}

pf_status pf_graph_end(void *stream, pf_graph **out) {
  if (!stream || !out) return fail(PF_ERR_ARG, "NULL argument");
  *out = nullptr;
  hipGraph_t g = nullptr;
  PF_HIP(hipStreamEndCapture((hipStream_t)stream, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(PF_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *out = new pf_graph{g, ex};
  return PF_OK;
}

pf_status pf_graph_launch(pf_graph *gr, void *stream) {
  if (!gr) return fail(PF_ERR_ARG, "graph is NULL");
  PF_HIP(hipGraphLaunch(gr->ex, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_graph_destroy(pf_graph *gr) {
  if (!gr) return PF_OK;
  (void)hipGraphExecDestroy(gr->ex);
  (void)hipGraphDestroy(gr->g);
  delete gr;
  return PF_OK;
}

pf_status pf_copy_kernel(void *dst, const void *src, size_t bytes, void *stream) {
  if (!dst || !src || bytes % 16) return fail(PF_ERR_ARG, "copy needs device pointers and a multiple of 16 bytes");
  if (overlaps(dst, bytes, src, bytes)) return fail(PF_ERR_ARG, "copy ranges overlap");
  PF_HIP(pf::launch_copy(dst, src, bytes, (hipStream_t)stream));
  return PF_OK;
}

}  // extern "C"
