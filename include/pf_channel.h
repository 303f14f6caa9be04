/*
 * pf_channel.h -- C ABI of the MI355X channel pressure-Poisson and
 * wall-normal Helmholtz solvers (arXiv 2502.06296).
 *
 * Problem statement (paper Sec. 2.1 and 2.2.1):
 *   Poisson    L7 p = f on a channel grid periodic in x and y, with uniform
 *              spacing there, and non-uniform cell faces zf[0..nz] in z.
 *              L7 is the second-order 7-point operator of the staggered
 *              (MAC) grid, pressure at cell centres, zero normal gradient at
 *              both walls. After packed real Fourier transforms in x and y
 *              every wavenumber pair (i,j) leaves one tridiagonal system in
 *              z whose diagonal is shifted by the modified wavenumbers
 *              (eq. fijk_eq). L7 is singular: f is first projected by
 *              removing its dzf-weighted mean, and p is returned with zero
 *              dzf-weighted mean. A grid may instead put walls at both y
 *              ends (pf_grid.ybc): the y transform is then the cosine
 *              (zero-gradient walls) or sine (value-zero walls, a
 *              nonsingular L7: no projection, no pin) transform.
 *   Helmholtz  (I - s L_z) u = r in every (x,y) column (eq. proj3_impl1d,
 *              with s = alpha * nu * dt; the paper writes gamma_k nu dt / 2),
 *              solved with the reworked cyclic reduction of Algorithm 2:
 *              pcr_prepare computes the chunk coefficients once (Step 1),
 *              pcr_apply runs the reduction, the reduced boundary solve and
 *              the in-place reconstruction (Steps 2-4).
 *
 * Layout: every field is a dense C-order array of shape (nz, ny, nx), x
 * fastest: element (i,j,k) at i + nx*(j + ny*k).
 *
 * Memory: field pointers are DEVICE pointers owned by the caller; plans own
 * only small constant tables. Every call is asynchronous on the plan's HIP
 * stream (passed as void*, a hipStream_t; NULL is the default stream); no
 * call made after a plan exists allocates, synchronises or reads back, so a
 * sequence of solves may be captured in a HIP graph.
 *
 * Errors: every function returns a pf_status; 0 is success. Arguments are
 * validated on the host before anything is enqueued, so a failing call
 * enqueues nothing. pf_last_error() returns a thread-local message for the
 * last failure on the calling thread.
 */
#ifndef PF_CHANNEL_H
#define PF_CHANNEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pf_status;
#define PF_OK 0
#define PF_ERR_ARG (-1)          /* NULL pointer, bad size, aliasing      */
#define PF_ERR_UNSUPPORTED (-2)  /* length or option this build lacks     */
#define PF_ERR_DEVICE (-3)       /* a HIP runtime call failed             */
#define PF_ERR_WORKSPACE (-4)    /* workspace missing or too small        */

/* Arithmetic of a solve.
 * PF_FP64         float64 everywhere.
 * PF_FP32         float32 transforms and storage; the z systems are
 *                 eliminated in float64 registers; about 1e-7 relative.
 * PF_FP32_REFINE  PF_FP32 followed by n_refine corrections, each solving
 *                 for the float64 residual f - L7 p (Poisson) or r - (I -
 *                 s L_z) u (Helmholtz, in registers); the singular zero
 *                 mode is always solved in float64. */
typedef enum { PF_FP64 = 0, PF_FP32 = 1, PF_FP32_REFINE = 2 } pf_precision;

/* Wall-normal boundary families of the staggered grid.
 * NEUMANN           cell centres (pressure), zero gradient at the walls.
 * DIRICHLET_CENTRE  cell centres (u, v), value 0 at the walls through a
 *                   ghost value mirrored about the wall.
 * DIRICHLET_FACE    interior faces 1..nz-1 (w), w = 0 on the wall faces;
 *                   nz-1 unknowns per column. */
typedef enum { PF_BC_NEUMANN = 0, PF_BC_DIRICHLET_CENTRE = 1, PF_BC_DIRICHLET_FACE = 2 } pf_zbc;

/* Channel grid. nx and ny each one of the transform lengths this library
 * instantiates: the even 2^a 3^b from 64 to 2048, and 3072, 3200 (2^7 5^2)
 * and 3456 (2^7 3^3), the lengths of the paper's per-GPU weak-scaling share
 * and of its strong-scaling grid; any other length is PF_ERR_UNSUPPORTED.
 * 4 <= nz <= 1024. zf: host array of
 * nz+1 strictly increasing face coordinates, copied at plan time; if NULL
 * the faces are zf[k] = lz/2 (1 + tanh(beta (2k/nz - 1)) / tanh(beta))
 * (uniform when beta == 0).
 * ybc: PF_Y_PERIODIC (the channel); PF_Y_WALLS, zero-gradient walls at
 * both y ends with ny cell-centred unknowns between them: the y transform
 * is then the cosine transform (the cosine member of the Fourier-based
 * transforms of Sec. 2.2.1) with the wavenumbers 4 sin^2(pi q / 2 ny) / dy^2;
 * PF_Y_DIRICHLET, walls where the solution vanishes: the sine transform,
 * wavenumbers 4 sin^2(pi (q + 1) / 2 ny) / dy^2, a nonsingular operator (f is
 * not projected and p is not pinned). Walls are implemented for
 * poisson_plan / poisson_solve and for helmholtz3d_plan / helmholtz3d_solve
 * (a field at cell-centre y positions); poisson_project takes PF_Y_WALLS
 * (v[:, ny-1, :] is then the top wall face: no flux through it enters the
 * divergence and it is left unchanged) and returns PF_ERR_UNSUPPORTED for
 * PF_Y_DIRICHLET.
 * PF_Y_FACES (helmholtz3d_plan only; poisson_plan returns
 * PF_ERR_UNSUPPORTED): a field on the y faces between walls where it
 * vanishes, the face-located velocity v of a y-walled grid: row j of each
 * plane holds the face j + 1 (j = 0..ny-2) and row ny - 1 the top wall face,
 * where the solve leaves zero up to rounding (about 1e-16 of the field's
 * largest value: the x inverse transforms it together with row ny - 2; r
 * there is not read). The y transform is the
 * type-I sine transform of the ny - 1 interior faces (the sine member of
 * Sec. 2.2.1's transforms for face unknowns), wavenumbers
 * 4 sin^2(pi q / 2 ny) / dy^2, q = 1..ny-1; 2 ny must be a built length.
 * xbc: the same choice at both x ends (PF_X_PERIODIC, PF_X_WALLS: the cosine
 * transform along x, wavenumbers 4 sin^2(pi q / 2 nx) / dx^2; PF_X_DIRICHLET:
 * the sine transform, 4 sin^2(pi (q + 1) / 2 nx) / dx^2, nonsingular), with
 * nx cell-centred unknowns, alone or with y walls; built for poisson_plan /
 * poisson_solve and helmholtz3d_plan / helmholtz3d_solve; poisson_project
 * takes PF_X_WALLS (u[:, :, nx-1] is then the east wall face: no flux
 * through it or through the west wall face enters the divergence, and it is
 * left unchanged) and returns PF_ERR_UNSUPPORTED for PF_X_DIRICHLET.
 * PF_X_FACES (helmholtz3d_plan only): PF_Y_FACES along x, a field on the x
 * faces (the face-located velocity u of an x-walled grid): column i of each
 * row holds the face i + 1 (i = 0..nx-2), column nx - 1 the east wall face
 * (zero in the result up to rounding; r there is not read); the type-I sine
 * transform along x, wavenumbers 4 sin^2(pi q / 2 nx) / dx^2, q = 1..nx-1;
 * 2 nx must be a built length. */
enum { PF_Y_PERIODIC = 0, PF_Y_WALLS = 1, PF_Y_DIRICHLET = 2, PF_Y_FACES = 3 };
enum { PF_X_PERIODIC = 0, PF_X_WALLS = 1, PF_X_DIRICHLET = 2, PF_X_FACES = 3 };
typedef struct pf_grid {
  int32_t nx, ny, nz;
  double lx, ly, lz;
  double beta;
  const double *zf;
  int32_t ybc;
  int32_t xbc;
} pf_grid;

typedef struct pf_poisson_plan pf_poisson_plan;
typedef struct pf_pcr_plan pf_pcr_plan;
typedef struct pf_graph pf_graph;

const char *pf_last_error(void);
int32_t pf_abi_version(void); /* 3: pf_grid carries ybc and xbc */

/* Host helper: the sign-normalised rows of -L_z for boundary family bc,
 * row k = -alpha[k] x[k-1] + (alpha[k]+gamma[k]+excess[k]) x[k]
 *         - gamma[k] x[k+1], all three >= 0, alpha[0] = gamma[n-1] = 0.
 * n = nz (centres) or nz-1 (faces). Output arrays are host, length n. */
pf_status pf_zop_rows(const pf_grid *g, int32_t bc, double *alpha, double *gamma,
                      double *excess);

/* Host helper: the face coordinates the plan uses (host array, nz+1). */
pf_status pf_grid_faces(const pf_grid *g, double *zf_out);

/* ------------------------------------------------------------ Poisson
 * poisson_plan: validates the grid, builds the modified wavenumbers of the
 * packed slots, the z rows, the twiddle tables and the kernel shapes, all
 * on the device of the calling thread. n_refine: corrections for
 * PF_FP32_REFINE, 0 or 1 (one correction reaches 1e-10 relative at
 * nz <= 1024; 0 is PF_FP32), ignored otherwise. *workspace_bytes (may be NULL) receives the
 * device workspace poisson_solve needs: 0 for PF_FP64 (p doubles as the
 * spectral buffer); for PF_FP32 a float32 spectrum whose z planes are
 * padded by 64 elements, 4*nz*(nx*ny + 64) bytes; for PF_FP32_REFINE that
 * plus the float32 iterate, 4*N more. */
pf_status poisson_plan(pf_poisson_plan **out, const pf_grid *g, int32_t precision,
                       int32_t n_refine, void *stream, size_t *workspace_bytes);
/* Caller-owned device workspace of at least *workspace_bytes, 256-byte
 * aligned; kept by pointer until replaced or the plan is destroyed. */
pf_status poisson_set_workspace(pf_poisson_plan *plan, void *workspace, size_t bytes);
/* p <- L7^{-1} f. rhs: device (nz,ny,nx) float64, read only. p: device
 * (nz,ny,nx) float64, must not overlap rhs or the workspace. */
pf_status poisson_solve(pf_poisson_plan *plan, const double *rhs, double *p);
/* poisson_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the float32 work arrays come from a static device array of the library,
 * 320 MiB per GPU, held from the library's load until the process ends,
 * instead of the plan's workspace (which need not be set). The call itself
 * allocates nothing; its first call on a device looks up that device's
 * array address once. Every call on one GPU shares the array, so calls that
 * overlap in time on one GPU (several streams, or several host threads)
 * race: order them on one stream. Nothing in the array needs to start at
 * zero. PF_ERR_UNSUPPORTED when the plan needs more than 320 MiB of scratch
 * (PF_FP32_REFINE: 8 nz (nx ny + 64) bytes, about 41 M points; PF_FP32
 * half that); a PF_FP64 plan needs none. Other arguments and errors as
 * poisson_solve. */
pf_status poisson_solve_noalloc(pf_poisson_plan *plan, const double *rhs, double *p);
/* A-posteriori status of the solves of a plan (device memory, written by
 * every later poisson_solve, poisson_project and helmholtz3d_solve on the
 * plan's stream; no host readback, so it is graph-capturable). For
 * PF_FP32_REFINE, est_rel_err = (max|correction| / max|iterate|)^2 over the
 * x spectra the last pass sums: the first iterate's relative error is about
 * max|correction| / max|iterate|, and one correction squares it. flags has
 * PF_STATUS_NOT_CONVERGED when est_rel_err > tol. Solves without a
 * correction record est_rel_err = -1 and no flag. The two max words are
 * working storage (bit patterns of non-negative doubles). */
typedef struct pf_solve_status {
  uint64_t max_iterate, max_correction;
  double est_rel_err;
  uint64_t flags;
} pf_solve_status;
enum { PF_STATUS_NOT_CONVERGED = 1 };
/* dev_status: device pointer to a pf_solve_status, 8-byte aligned, or NULL
 * to stop recording; tol >= 0. Calls that share a status word must be
 * ordered (same stream). */
pf_status poisson_set_status(pf_poisson_plan *plan, void *dev_status, double tol);

/* Pressure projection of a Runge-Kutta substep on the staggered grid
 * (paper Sec. 2.1, eqs. proj1_Lphi, proj1_ukp1, proj1_Pkp1; with implicit
 * wall-normal diffusion the z part of eq. proj2_Pkp1):
 *   L7 phi = D u* / gdt,   u <- u* - gdt G phi,   p <- p + phi - c L_z phi.
 * u: x-face velocity, u[k][j][i] on face i+1/2 of cell (i,j,k); v: y-face
 * velocity, v[k][j][i] on face j+1/2; both (nz,ny,nx). w: (nz-1,ny,nx), the
 * interior z faces 1..nz-1 (w[m] between cells m and m+1; w = 0 on the
 * walls, not stored). D is the cell divergence (face fluxes over dx, dy,
 * dzf), G the face gradient (over dx, dy and the centre distances), L_z the
 * zero-gradient z operator; D G = L7. gdt = gamma_k * dt > 0; c >= 0 (0 for
 * explicit diffusion, gamma_k * nu * dt / 2 with the z-implicit Helmholtz).
 * Zero-gradient walls (PF_Y_WALLS, PF_X_WALLS) make v[:, ny-1, :] and
 * u[:, :, nx-1] wall faces: no flux, no correction. Value-zero walls
 * (PF_Y_DIRICHLET, PF_X_DIRICHLET) return PF_ERR_UNSUPPORTED: a correction
 * pressure that vanishes on a wall would push fluid through it.
 * phi: device (nz,ny,nx) float64, receives the correction pressure (zero
 * dzf-weighted mean) and serves the solve as its spectral buffer (PF_FP64)
 * or as the stash of f (PF_FP32_REFINE). u, v, w, p are updated in place.
 * All device float64, 16-byte aligned, pairwise disjoint and disjoint from
 * the workspace; the workspace rules of poisson_solve apply. */
pf_status poisson_project(pf_poisson_plan *plan, double *u, double *v, double *w, double *p,
                          double *phi, double gdt, double c);
/* The same solve for several independent problems on the first plan's
 * stream (the batches of uneven problems of the paper's use, Sec. 3: one
 * pressure solve or 3-D Helmholtz per grid). Plans in float32 with one
 * float64-residual correction (PF_FP32_REFINE), periodic in x and y, whose
 * z solve takes a separator-form shape (the default for every supported
 * size), run grouped: each stage of all of them is one launch per kernel
 * instance (one per transform length; per z-solve shape and chunk count),
 * at most 16 problems a launch; the other plans run one after another
 * afterwards. Results equal poisson_solve's bitwise. Stage timing, when
 * enabled on the first grouped plan, records the grouped launches there.
 * PF_ERR_ARG: a plan given twice, an output overlapping another entry's
 * input or output, overlapping workspaces; the per-solve checks of
 * poisson_solve apply to each entry; all checks run before anything is
 * enqueued. */
pf_status poisson_solve_batched(int32_t count, pf_poisson_plan *const *plans,
                                const double *const *rhs, double *const *p);
pf_status poisson_set_stream(pf_poisson_plan *plan, void *stream);
pf_status poisson_destroy(pf_poisson_plan *plan);

/* ------------------------------------------------- 3-D Helmholtz
 * The fully implicit diffusion of a Runge-Kutta substep (paper Sec. 2.1,
 * eq. proj2_ustar): u with (I - s L) u = r, L the 3-D second-order operator
 * of the staggered grid, periodic in x and y, with the Dirichlet z rows of
 * family bc (PF_BC_DIRICHLET_CENTRE: nz unknowns per column, u and v;
 * PF_BC_DIRICHLET_FACE: nz-1, w), s = gamma_k nu dt / 2 > 0. The solver is
 * the Poisson machinery (packed transforms in x and y, one z system per
 * slot pair) with the diagonal of every mode shifted by 1/s; no mode is
 * singular. helmholtz3d_plan takes the grid, precision, n_refine, stream
 * and workspace rules of poisson_plan (the workspace is sized by the n =
 * nz or nz-1 planes of the field); the plan is destroyed with
 * poisson_destroy and takes poisson_set_workspace, poisson_set_stream and
 * the stage timers. helmholtz3d_solve: r and u device (n, ny, nx) float64,
 * u must not overlap r or the workspace. helmholtz3d_update changes s > 0
 * for the solves enqueued after it: a kernel on the plan's stream rebuilds
 * the shifted wavenumber table (no host staging, no synchronisation), and
 * later solves take 1/s as a launch argument; capturable, and several
 * updates with solves between them may be queued or captured in one graph.
 * Errors as poisson_solve; a Helmholtz plan is refused by poisson_solve and
 * poisson_project, and a Poisson plan by helmholtz3d_solve. */
pf_status helmholtz3d_plan(pf_poisson_plan **out, const pf_grid *g, int32_t bc, double s,
                           int32_t precision, int32_t n_refine, void *stream,
                           size_t *workspace_bytes);
pf_status helmholtz3d_solve(pf_poisson_plan *plan, const double *r, double *u);
pf_status helmholtz3d_update(pf_poisson_plan *plan, double s);

/* ---------------------------------------------------------- Helmholtz
 * pcr_prepare (Algorithm 2, Step 1): host arrays alpha, gamma, excess of
 * length n in the form of pf_zop_rows describe -L_z; the plan solves
 * (I - s L_z) u = r, i.e. rows (s alpha, s gamma, 1 + s excess), s >= 0.
 * Rows are split into P chunks; chunk_rows is the
 * number of rows per chunk (0 picks it; otherwise 8, 16 or 32), at most 32
 * chunks; the last chunk is padded with identity rows. The rows are copied
 * to the device; the chunk coefficients, the reduced boundary system's
 * twisted elimination and its cyclic reduction are then computed there in
 * float64, subtraction-free, by one kernel on `stream` (the plan call waits
 * for it; pcr_update_coef reruns it).
 * precision: PF_FP64 (float64 field), PF_FP32 (float32 field), or
 * PF_FP32_REFINE (float64 field, float32 solves plus one float64-residual
 * correction in registers). n >= 4. */
pf_status pcr_prepare(pf_pcr_plan **out, int32_t n, const double *alpha, const double *gamma,
                      const double *excess, double s, int32_t precision, int32_t chunk_rows,
                      void *stream);
/* The same plan from the paper's form of the rows (the inputs A, B, C of
 * Algorithm 2, here of L_z itself): lower[k] x[k-1] + diag[k] x[k] +
 * upper[k] x[k+1] is row k of L_z, host arrays of length n, lower[0] =
 * upper[n-1] = 0; the plan solves (I - s L_z) u = r. The rows are converted
 * to the sign-normalised form (alpha = lower, gamma = upper, excess =
 * -(lower + diag + upper), set to 0 when it is within 16 ulp of the three
 * terms). PF_ERR_UNSUPPORTED when a row is not of M-matrix form (a negative
 * off-diagonal, or a diagonal smaller in magnitude than the off-diagonal sum
 * beyond rounding): the subtraction-free elimination needs it. Other
 * arguments and errors as pcr_prepare. */
pf_status pcr_prepare_rows(pf_pcr_plan **out, int32_t n, const double *lower, const double *diag,
                           const double *upper, double s, int32_t precision, int32_t chunk_rows,
                           void *stream);
/* Re-run Step 1 for a new s >= 0 (one per Runge-Kutta substep, the paper's
 * local recomputation of the chunk coefficients in Sec. 2.2.4): one kernel
 * on the plan's stream recomputes every table from the stored rows of L_z.
 * No host work, copy, allocation or synchronisation: stream-ordered with the
 * plan's applies, and capturable, so a graph may hold several substeps with
 * different s. */
pf_status pcr_update_coef(pf_pcr_plan *plan, double s);
/* In place, every column of a device (n, ny, nx) field; float64 or float32
 * per the plan's precision. nx must be a multiple of 64. */
pf_status pcr_apply(pf_pcr_plan *plan, void *field, int32_t nx, int32_t ny);
/* Several fields (1..16: for example the three velocity components, or
 * those of several independent problems) in one launch; all plans must
 * share precision, chunk rows and stream. */
pf_status pcr_apply_batched(int32_t count, pf_pcr_plan *const *plans, void *const *fields,
                            const int32_t *nx, const int32_t *ny);
pf_status pcr_set_stream(pf_pcr_plan *plan, void *stream);
pf_status pcr_destroy(pf_pcr_plan *plan);

/* ---------------------------------------------------------- HIP graphs
 * Capture every call enqueued on `stream` between begin and end into a
 * graph (stream must not be the default stream), replay it with
 * pf_graph_launch. */
pf_status pf_graph_begin(void *stream);
pf_status pf_graph_end(void *stream, pf_graph **out);
pf_status pf_graph_launch(pf_graph *graph, void *stream);
pf_status pf_graph_destroy(pf_graph *graph);

/* ------------------------------------------------------------- task batch
 * Independent work of several problems (the batch of uneven channel grids
 * of the paper's use: a pressure solve and the velocity components of each
 * problem), spread over `lanes` (1..8) internal streams forked from `stream`
 * and joined back into it, so that small problems run side by side instead
 * of leaving the GPU underfilled one after another.
 *
 * A task is an optional Poisson solve (poisson, rhs, p as for poisson_solve)
 * and an optional group of ncomp (0..4) Helmholtz fields applied in one
 * launch (pcr[], field[], nx[], ny[] as for pcr_apply_batched: the plans of
 * a group share chunk rows and precision). Tasks are assigned largest first
 * to the least-loaded lane. Every task is ordered after the work already on
 * `stream`, and work enqueued on `stream` afterwards after every task. Tasks
 * must not share Poisson plans, and nothing one task writes (p, workspace,
 * Helmholtz fields) may overlap what another reads or writes: PF_ERR_ARG
 * (Helmholtz plans, read only during an apply, may be shared). Inside pf_graph_begin/pf_graph_end on
 * `stream` the fork and join become graph edges. The lanes (default-priority
 * streams) and their events are created once per device by the first call,
 * which must not be inside a capture, and are kept until the process ends.
 * Every task is validated before anything is enqueued. Calls from several
 * host threads are serialised. Plans keep their own streams for their other
 * calls. */
typedef struct {
  pf_poisson_plan *poisson; /* NULL: no Poisson solve */
  const double *rhs;
  double *p;
  int32_t ncomp;            /* Helmholtz fields, 0..4 */
  pf_pcr_plan *pcr[4];
  void *field[4];
  int32_t nx[4], ny[4];
} pf_task;
pf_status pf_run_batched(int32_t count, const pf_task *tasks, int32_t lanes, void *stream);

/* --------------------------------------------------------- measurement
 * Stage timing in the style of the paper's per-operation GPU timers: when
 * enabled, each kernel a plan launches is bracketed by HIP events on the
 * plan's stream. pf_*_timing_read synchronises the stream and returns, per
 * stage, the summed milliseconds and the launch count since the last read
 * (arrays of PF_STAGE_COUNT). PF_STAGE_XINV is the x inverse of the FP64
 * solve, PF_STAGE_XINV_FINAL the last x inverse of the float32 solves (for
 * PF_FP32_REFINE: of iterate plus correction); PF_STAGE_XFWD_RESID is the
 * correction's right-hand side of PF_FP32_REFINE (the float64 residual
 * formed in x-spectral space); PF_STAGE_PROJECT is the velocity and pressure
 * update of poisson_project (whose first x pass, which forms the divergence,
 * counts as PF_STAGE_XFWD). */
enum {
  PF_STAGE_XFWD = 0, PF_STAGE_YFWD = 1, PF_STAGE_ZSOLVE = 2, PF_STAGE_YINV = 3,
  PF_STAGE_XINV = 4, PF_STAGE_ZERO_MODE = 5, PF_STAGE_XFWD_RESID = 6, PF_STAGE_XINV_FINAL = 7,
  PF_STAGE_PCR_APPLY = 8, PF_STAGE_PROJECT = 9, PF_STAGE_COUNT = 10
};
pf_status poisson_timing(pf_poisson_plan *plan, int32_t enable);
pf_status poisson_timing_read(pf_poisson_plan *plan, double *ms, int32_t *count);
pf_status pcr_timing(pf_pcr_plan *plan, int32_t enable);
pf_status pcr_timing_read(pf_pcr_plan *plan, double *ms, int32_t *count);

/* ------------------------------------------------------------ tuning
 * Launch-shape variants that an autotuner may choose between. For
 * PF_STAGE_ZSOLVE the variants are table entries of (rows per thread,
 * columns per workgroup, occupancy bound, reciprocal flavour, elimination
 * form, column tile through LDS, single or double-buffered reduced rows). For
 * PF_STAGE_XFWD (the x forward, the x inverse and the refinement's residual)
 * and PF_STAGE_YFWD (both y transforms) of a direction without walls they
 * are 5 transform shapes: 0 the default, 1 half the threads per line, 2
 * twice the threads per line (x) or the lines per workgroup (y), 3 the
 * radix capped at 8, 4 (y only, every length) the default shape in a
 * persistent launch that loads each workgroup's next lines while it
 * transforms the current ones; shapes 1-3 exist for the lengths 256, 512,
 * 1024 and 2048. Every variant computes the same solution to rounding. *count
 * receives the number of
 * variants; poisson_set_variant returns PF_ERR_UNSUPPORTED for a variant
 * that does not fit the plan's grid. Plans with non-default transform
 * shapes run one by one in poisson_solve_batched. Set variants only while no
 * solve of the plan is in flight. */
pf_status poisson_variant_count(pf_poisson_plan *plan, int32_t stage, int32_t *count);
pf_status poisson_set_variant(pf_poisson_plan *plan, int32_t stage, int32_t variant);
pf_status poisson_get_variant(pf_poisson_plan *plan, int32_t stage, int32_t *variant);
/* Re-shape a Helmholtz plan: rows per chunk (8, 16 or 32) and columns per
 * chunk (16, 32 or 64; negated for persistent workgroups that stage the
 * Step 1 tables in LDS, at most 512 threads); re-runs Step 1 and re-uploads
 * the tables (synchronises the plan's stream; allocates). */
pf_status pcr_set_shape(pf_pcr_plan *plan, int32_t chunk_rows, int32_t columns_per_chunk);
pf_status pcr_get_shape(pf_pcr_plan *plan, int32_t *chunk_rows, int32_t *columns_per_chunk);

/* A plain device copy of `bytes` bytes (multiple of 16), the calibration
 * kernel for hardware byte counters. */
pf_status pf_copy_kernel(void *dst, const void *src, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PF_CHANNEL_H */
