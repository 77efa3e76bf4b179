/*
 * les.h - C ABI of the MI355X large-eddy-simulation substep library.
 *
 * The library advances the filtered incompressible Navier-Stokes equations by one
 * low-storage third-order Runge-Kutta substep on a staggered (MAC) finite-difference
 * grid, as described in Xiao et al., "CaLES: A GPU-accelerated solver for large-eddy
 * simulation of wall-bounded flows" (arXiv 2411.09364):
 *   predictor            Sec. 2.2, Eq. onestar_exp (explicit viscous terms) or
 *                        Eqs. twostar_imp1d, onestar_imp1d (Crank-Nicolson in z)
 *   pressure Poisson     Eq. poi, solved by eigenfunction expansion: FFTs in the periodic
 *                        x and y directions, tridiagonal (Thomas) solves along the
 *                        non-uniform z direction (Sec. 2.2)
 *   projection           Eqs. correc, p_update_exp / p_update_imp1d
 *   eddy viscosity       Sec. 2.1: Smagorinsky with optional van Driest damping (Eq. smag),
 *                        dynamic Smagorinsky (Eqs. dsmag, cs, lij, mij), or a learned
 *                        coefficient network
 *   wall model           Sec. 2.1 Eq. wm (log law) with the coupling of Sec. 2.2
 *   boundary order       Alg. 2; substep order Alg. 1
 *
 * Axes: x and y periodic; z either periodic or bounded by walls at z = 0 and z = lz.
 * (The paper calls the wall-normal direction y; here it is z, the solver's stretched axis.)
 *
 * Memory: every device buffer is allocated by the caller (the library never allocates
 * device memory) and must stay valid while the context uses it.  Fields are dense
 * arrays of shape [nz + 2][ny][nx] (x fastest) in the storage type reported by
 * les_layout (double for LES_FP64, float for LES_MIXED).  Planes 0 and nz + 1 are ghost
 * planes.  Face positions: u[k][j][i] at x = (i+1) dx, y = (j+1/2) dy, z = zc[k];
 * v at ((i+1/2) dx, (j+1) dy, zc[k]); w at ((i+1/2) dx, (j+1/2) dy, zf[k]) where zf[k] is
 * the top face of cell k (zf[0] = 0, zf[nz] = lz); p at cell centres.
 *
 * Streams: all device work is enqueued on the HIP stream given to les_init, in order,
 * without synchronising, unless a function says it synchronises.  A context is not
 * thread-safe.  Asynchronous device faults surface as LES_EDEVICE at the next
 * synchronising call.
 *
 * Errors: every function returns les_status and never aborts.  Arguments are validated
 * before any device work is enqueued; on error nothing is enqueued and les_last_error
 * describes the problem.
 */
#ifndef LES_H
#define LES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LES_ABI_VERSION 2

typedef enum {
  LES_OK = 0,
  LES_EINVAL = -1,      /* invalid argument or configuration                         */
  LES_ENOMEM = -2,      /* caller buffer too small                                   */
  LES_EDEVICE = -3,     /* HIP runtime error (launch failure, earlier fault, ...)    */
  LES_ENOTSUP = -4,     /* valid but unsupported combination (e.g. FFT length)       */
  LES_ENONFINITE = -5,  /* non-finite value detected in the state                    */
  LES_ESTATE = -6       /* call out of order (e.g. field not bound)                  */
} les_status;

enum { LES_ZBC_PERIODIC = 0, LES_ZBC_NOSLIP = 1, LES_ZBC_WALLMODEL = 2 };
/* y boundaries (les_config.ybc): periodic, or walls at y = 0 and y = ly with the z walls'
   treatment (no-slip or the wall model): the square duct of Sec. 4.4. */
enum { LES_YBC_PERIODIC = 0, LES_YBC_WALL = 1 };
enum { LES_SGS_NONE = 0, LES_SGS_SMAG = 1, LES_SGS_SMAG_VD = 2, LES_SGS_DSM = 3, LES_SGS_MLP = 4 };
enum { LES_FP64 = 0, LES_MIXED = 1 };
/* Viscous-term treatment (les_config.implicit_z). */
enum { LES_VISC_EXPLICIT = 0, LES_VISC_CN_Z = 1, LES_VISC_CN_3D = 2 };

typedef struct les_ctx les_ctx;   /* opaque, owned by the library */

/* Problem description.  Plain data, copied by les_init. */
typedef struct {
  int32_t abi_version;  /* must be LES_ABI_VERSION                                        */
  int32_t nx, ny, nz;   /* cells; nx, ny even, of the form 2^a, 3 * 2^a, 5 * 2^a or
                           15 * 2^a, 4..1024; 4 <= nz <= 512 (wall-bounded) or, when z is
                           periodic, of that form                                          */
  double lx, ly, lz;    /* box lengths (> 0)                                             */
  int32_t zbc;          /* LES_ZBC_*                                                     */
  double beta;          /* tanh wall clustering (wall-bounded z); 0 = uniform            */
  double nu;            /* kinematic viscosity (> 0)                                     */
  int32_t sgs;          /* LES_SGS_*                                                     */
  double cs;            /* Smagorinsky constant for LES_SGS_SMAG / _SMAG_VD              */
  int32_t implicit_z;   /* LES_VISC_*: explicit viscous terms (Eq. twostar_exp); Crank-Nicolson
                           in z (Eqs. twostar_imp1d, onestar_imp1d; walls only); or Crank-
                           Nicolson in all directions (Eqs. twostar_imp3d, onestar_imp3d,
                           p_update_imp3d; the Helmholtz systems solved by FFTs in x and y
                           and FP64 Thomas in z, or FFTs in z as well when z is periodic)  */
  int32_t precision;    /* LES_FP64, or LES_MIXED: float storage, stencils and FFTs,
                           double tridiagonal solves, zero mode and reductions           */
  double ubulk;         /* > 0: constant flow rate (bulk velocity) in x; 0: off          */
  double h_wm;          /* wall-model height; 0 = first off-wall cell centre            */
  double kappa, bconst; /* log-law constants (Eq. wm); 0 selects 0.41 and 5.2            */
  int32_t ybc;          /* LES_YBC_*.  LES_YBC_WALL (square duct, Sec. 4.4) needs wall-bounded
                           z, uniform y, and explicit viscous terms or CN in z (the dynamic
                           coefficient is then averaged along x lines, the only homogeneous
                           direction, and the learned closure falls back per x line).  Fields then
                           carry two ghost rows in y after the interior rows: dims
                           [nz+2][ny+2][nx], row ny above y = ly, row ny+1 below y = 0
                           (where the periodic index j - 1 of row 0 lands).  v on row
                           ny - 1 is the wall face y = ly and stays zero.  Batches are not
                           available for ducts. */
} les_config;

/* Bindable and readable buffers. */
enum {
  LES_FIELD_U = 0, LES_FIELD_V = 1, LES_FIELD_W = 2, LES_FIELD_P = 3,
  LES_FIELD_WORKSPACE = 4,  /* scratch + internal state (RK history, |S|, spectra, ...) */
  LES_FIELD_NUT = 5,        /* readable only: eddy viscosity at cell centres, field layout */
  LES_FIELD_CS = 6,         /* readable only: per-plane model coefficient, double[nz]
                               (ducts: per x line, double[nz][ny])                         */
  LES_FIELD_TAUW = 7,       /* readable only: wall stress, double[4][ny'][nx] (ny' = the stored
                               rows): tau_x bottom, tau_y bottom, tau_x top, tau_y top     */
  LES_FIELD_ZGRID = 8,      /* readable only, host memory: double zf[nz+1], zc[nz+2]       */
  LES_FIELD_TAUWY = 9       /* readable only, ducts with the wall model: y-wall stress,
                               double[4][nz+2][nx]: tau_x at y = 0, tau_z at y = 0, tau_x at
                               y = ly, tau_z at y = ly (zero on the ghost planes and, for
                               tau_z, on the wall face k = nz)                              */
};

typedef struct {
  int64_t nx, ny, nz;        /* interior cells                                     */
  int64_t dims[3];           /* [nz+2, ny, nx] for fields ([nz+2, ny+2, nx] for ducts) */
  int64_t elem_bytes;        /* 8 (double) or 4 (float) for fields                 */
  int64_t bytes;             /* total bytes required for the requested buffer      */
} les_layout_t;

/* Diagnostics (les_diag synchronises the stream). */
typedef struct {
  double max_div;            /* max |D u| over cells                                 */
  double ubulk;              /* volume-mean u                                        */
  double max_vel;            /* max |u|, |v|, |w|                                    */
  double tauw_mean[2];       /* plane-mean tau_x at bottom / top wall (wall model)   */
  double dt;                 /* current time step in the device slot                 */
  int64_t nonfinite;         /* count of non-finite values in u, v, w, p             */
  int64_t mlp_flagged;       /* learned closure: points that fell back in the last nu_t evaluation */
} les_diag_t;

/* Validate cfg, compute the grid metrics and solver tables on the host, and create a
 * context bound to hip_stream (a hipStream_t, NULL = default stream).  No device work
 * is done.  On error *out is NULL. */
les_status les_init(const les_config* cfg, void* hip_stream, les_ctx** out);

/* Size and shape of a bindable or readable buffer (LES_FIELD_*). */
les_status les_layout(const les_ctx* ctx, int field, les_layout_t* out);

/* Bind caller-owned device memory to LES_FIELD_U/V/W/P or LES_FIELD_WORKSPACE.  The
 * pointer must be 256-byte aligned and hold les_layout(field).bytes.  Binding the
 * workspace enqueues the upload of the solver tables (grid metrics, eigenvalues,
 * twiddles) and zeroes the internal state. */
les_status les_bind(les_ctx* ctx, int field, void* device_ptr);

/* Alg. 1, line 2 and Alg. 2: fill the ghost planes of u, v, w, p, evaluate the wall
 * model (zbc = WALLMODEL) and the eddy viscosity from the bound velocity.  Must be called
 * once after the initial fields are written and before the first substep. */
les_status les_nut(les_ctx* ctx);

/* Time step: Courant-limited (cfl times the inverse of max |u|/dx + |v|/dy + |w|/dzf)
 * and viscous-limited (0.95 * 2.51 / (4 max(nu + nu_t) sum 1/h^2), z term dropped with
 * CN in z), the minimum of the two, written to the context's device time-step slot.  If
 * dt_host is not NULL the stream is synchronised and the value returned there.  After a
 * substep the advective maximum is the one the substep's correction took from the velocity
 * it wrote (the same per-cell values); les_nut, les_bind and les_project drop it, so fields
 * written by the caller are read here once les_nut has run for them.  LES_CFL_PASS=1 in the
 * environment when the context is created: always a pass over the fields. */
les_status les_dt(les_ctx* ctx, double cfl, double* dt_host);

/* Write dt into the device time-step slot (enqueued; no synchronisation). */
les_status les_set_dt(les_ctx* ctx, double dt);

/* One RK3 substep, stage = 0, 1, 2 (Alg. 1 inner loop body): predictor, optional CN-z
 * Helmholtz solves, Poisson solve, correction, pressure update, flow-rate forcing,
 * boundary conditions, wall model and eddy viscosity of the new velocity.  Uses the
 * time step in the device slot. */
les_status les_substep(les_ctx* ctx, int stage);

/* Three substeps.  use_graph != 0 records them once into a hipGraph on first use and
 * replays it afterwards (the time step is read from the device slot, so replays see
 * the current value). */
les_status les_step(les_ctx* ctx, int use_graph);

/* Solve D(G phi) = f (Eq. poi's discrete operator, zero-flux walls or periodic z) in
 * place: f_inout is a device buffer in field layout (storage type of the context); on
 * return its interior holds phi with zero dzf-weighted mean and its ghost planes are
 * filled.  Uses the workspace. */
les_status les_poisson(les_ctx* ctx, void* f_inout);

/* Initial fields: make the bound velocity discretely divergence-free by one projection with
 * the substep's own operators (Eq. poi and Eq. correc without the time factor gamma_k dt):
 * phi solves D G phi = D u with zero flux through walls (or periodic z), then u -= G phi, the
 * wall faces of w (and of v in a duct) staying zero.  With a constant flow rate (ubulk > 0) u
 * is then shifted uniformly so that its volume mean (sum u dzf / (nx ny lz)) is ubulk.  Only
 * interior values change.  Enqueued; uses the workspace (spectrum, pressure correction); call
 * les_nut afterwards (les_substep returns LES_ESTATE until then). */
les_status les_project(les_ctx* ctx);

/* Copy a readable quantity (LES_FIELD_NUT, _CS, _TAUW to device memory dst; _ZGRID to
 * host memory dst).  Enqueued, except _ZGRID which is immediate. */
les_status les_read(les_ctx* ctx, int field, void* dst);

/* Synchronise and compute diagnostics. */
les_status les_diag(les_ctx* ctx, les_diag_t* out);

/* ---------------------------------------------------------------- statistics
 * Long-run statistics of a channel run (Secs. 4.2 and 4.3 channel cases: mean velocity, resolved
 * Reynolds stresses, u_tau, Re_tau = u_tau h / nu with h = lz/2, C_f = tau_w / (u_b^2 / 2) and
 * its standard uncertainty; Eq. error for profile errors).  A sample is the plane (x-y) sums
 * of the current state, added on the device to running sums; products are taken where their
 * staggered factors meet: u v on the (x, y) edge, u w on the (x, z) edge and v w on the (y, z)
 * edge at the top face of each cell, each factor the two-point mean onto that edge; w, w^2 and
 * the products with w belong to the top face of cell k.  tau_w is the time mean of the
 * plane-mean streamwise wall stress over both walls (wall model: its stress; no-slip:
 * nu du/dz from the ghosts; 0 with periodic z); u_b is the dzf-weighted mean of the mean
 * velocity profile.  The uncertainty of C_f is plain batch means over the per-sample series:
 * nbatch equal consecutive batches (the oldest samples beyond nbatch * floor(len / nbatch)
 * dropped), std of the batch means (n - 1 norm) / sqrt(nbatch), times 2 / u_b^2. */
#define LES_STATS_NPROF 11
#define LES_STATS_SERIES_MAX 65536   /* the wall-stress series keeps the first this many samples;
                                        the running sums take every sample */
/* profile rows of les_stats_read: means, then covariances (mean product minus product of
 * the means of the two edge factors) */
enum { LES_STAT_U = 0, LES_STAT_V, LES_STAT_W, LES_STAT_P, LES_STAT_NUT, LES_STAT_UU, LES_STAT_VV, LES_STAT_WW,
       LES_STAT_UV, LES_STAT_UW, LES_STAT_VW };

typedef struct {
  int64_t samples;       /* samples accumulated since les_stats_reset                    */
  int64_t series_len;    /* samples in the wall-stress series (<= LES_STATS_SERIES_MAX)   */
  double tau_w, u_tau, re_tau;
  double u_b;
  double c_f, c_f_sigma; /* c_f_sigma NaN with fewer than 2 batches or samples < nbatch   */
} les_stats_t;

/* Clear the running sums (enqueued; also done at les_bind of the workspace). */
les_status les_stats_reset(les_ctx* ctx);
/* Add the current state as one sample (enqueued; two kernels). */
les_status les_stats_sample(les_ctx* ctx);
/* Synchronise, copy the sums to the host and finalise: out, and when profiles is not NULL
 * the host array profiles[LES_STATS_NPROF][nz] (rows LES_STAT_*).
 * Ducts (Sec. 4.4): the sums run along x lines, so profiles is [LES_STATS_NPROF][nz][ny]
 * (cross-sections); a covariance subtracts the product of the two edge factors' means, each
 * the two-point mean of the neighbouring lines' means; tau_w is the perimeter mean of the
 * streamwise wall stress (each wall's mean, the y walls' weighted by dzf, weighted by the
 * wall's length); u_b the area mean of U; Re_tau uses h = lz / 2. */
les_status les_stats_read(les_ctx* ctx, int32_t nbatch, les_stats_t* out, double* profiles);
/* Host only.  Relative profile error of Eq. error over [z0, z1]: phi and ref known at the n
 * increasing points z, both taken piecewise linear between them; the integrals are exact for
 * that interpolant.  LES_EINVAL for n < 2, non-increasing z, z1 <= z0 or a zero reference
 * integral. */
les_status les_profile_error(const double* z, const double* phi, const double* ref, int32_t n, double z0,
                             double z1, double* eps);

/* ---------------------------------------------------------------- learned closure
 * Not in the paper, which motivates SGS closures trained on data produced by the LES solver
 * itself (Sec. 1).  Network: 7 -> 64 -> 64 -> 1 with SiLU, output clipped at zero, giving the
 * coefficient c of nu_t = c Delta^2 |S| (the role c_s plays in Eq. dsmag).  Inputs per cell:
 * tr(S^2), tr(O^2), tr(S^3), tr(O^2 S), tr(O^2 S^2) of S/n and O/n (S strain, O rotation,
 * n = sqrt(S_ij S_ij + O_ij O_ij)), y+ = d u_tau/nu (d distance to the nearer wall, u_tau from
 * that wall's plane-mean stress; 0 when z is periodic; in a duct the smallest d_w u_tau,w/nu
 * over the four walls, each u_tau,w from its wall's mean stress, as in the van Driest factor)
 * and Delta (channel half-height 1), each min-max scaled with the training ranges lo, hi.
 * Parameters: 4737 floats, W1[64][7] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3, float32
 * master copy in caller-owned device memory.  W1, W2 and the inputs of the two 64-wide
 * products are rounded to bfloat16 (nearest-even) for the matrix cores, accumulation is
 * float32; the output layer is float32. */

/* Use the network for nu_t (context created with sgs = LES_SGS_MLP; until this is called such
 * a context runs the dynamic model).  params must stay valid; lo, hi: host double[7], copied.
 * Points whose scaled inputs leave [-0.05, 1.05] take the dynamic-model coefficient of their
 * plane (of their x line in a duct) instead, computed from the same velocity: the dynamic
 * model runs (on the device, without host round trip) in every nu_t evaluation in which a
 * point falls back, and only then.  A range not much wider than the rounding of its input (an input constant
 * over the grid, such as Delta on a uniform grid) makes the scaled input rounding noise:
 * give such an input a span of order one. */
les_status les_mlp_bind(les_ctx* ctx, const float* params_dev, const double* lo, const double* hi);

/* Training pairs from the current state: sample s sits at interior cell
 * e = SplitMix64(seed ^ SplitMix64(s)) mod (nz ny nx), in [k][j][i] order; x_raw_dev
 * (float[n][7]) receives its raw (unscaled) inputs and y_dev (float[n]) the dynamic-model
 * coefficient of its plane, or of its x line in a duct (context with sgs = DSM, after les_nut
 * or a substep). */
les_status les_mlp_sample(les_ctx* ctx, uint64_t seed, int64_t n_samples, float* x_raw_dev, float* y_dev);

/* The functions below need no context; they enqueue on hip_stream (NULL = default). */

/* x = (x_raw - lo)/(hi - lo) per input (device float[n][7] in and out; lo, hi host double[7]). */
les_status les_mlp_normalize(void* hip_stream, const float* x_raw_dev, int64_t n, const double* lo,
                             const double* hi, float* x_dev);

/* y_dev[n] = network(x_dev[n][7]) (scaled inputs, no clipping). */
les_status les_mlp_forward(void* hip_stream, const float* params_dev, const float* x_dev, int64_t n, float* y_dev);

/* Bytes of device workspace les_mlp_grad needs for n samples. */
int64_t les_mlp_workspace_bytes(int64_t n);

/* Gradient of the mean-squared error mean((network(x) - y)^2) over n samples: grad_dev
 * (float[4737]) and loss_dev (one float, may be NULL).  dz2 and dz1 enter the products in
 * bfloat16; per-block partial gradients are summed in a fixed order (run-to-run identical). */
les_status les_mlp_grad(void* hip_stream, const float* params_dev, const float* x_dev, const float* y_dev,
                        int64_t n, void* workspace_dev, float* grad_dev, float* loss_dev);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on params_dev with moments m_dev, v_dev
 * (float[4737] each); step is the 1-based Adam counter. */
les_status les_mlp_adam(void* hip_stream, float* params_dev, const float* grad_dev, float* m_dev, float* v_dev,
                        int step, float lr);

/* For callers that cannot allocate device memory (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): les_mlp_grad without a workspace argument.  The
 * per-block partial gradients live in a static device array of the library,
 * LES_MLP_NOALLOC_MAX_SAMPLES / 256 * 4738 floats (4.6 MiB), one per device, held until the
 * process ends; its address is looked up on the first call on each device, with the stream's
 * device current (a stream of another device: LES_EINVAL).  n above
 * LES_MLP_NOALLOC_MAX_SAMPLES returns LES_EINVAL with a message in les_last_error(NULL).
 * Results are bitwise those of les_mlp_grad for the same inputs.  Nothing is allocated.  All
 * calls on one device share the array: calls that overlap on one device (other streams,
 * other threads) race and must be ordered by the caller. */
#define LES_MLP_NOALLOC_MAX_SAMPLES 65536
les_status les_mlp_grad_noalloc(void* hip_stream, const float* params_dev, const float* x_dev, const float* y_dev,
                                int64_t n, float* grad_dev, float* loss_dev);

/* les_mlp_grad followed by les_mlp_adam. */
les_status les_mlp_train_step(void* hip_stream, float* params_dev, const float* x_dev, const float* y_dev,
                              int64_t n, void* workspace_dev, float* grad_dev, float* m_dev, float* v_dev,
                              int step, float lr, float* loss_dev);

/* Per-kernel timing.  les_timing(ctx, 1) starts recording: every kernel the context
 * enqueues afterwards is bracketed by two HIP events on the context stream and tagged with
 * its algorithmic byte count (each array the kernel reads or writes counted once).
 * les_timing(ctx, 0) stops recording.  Recording is refused inside les_step's graph
 * capture (LES_ESTATE).  les_timing_report synchronises, writes a JSON object
 * {"kernel": {"count": n, "ms": total_ms, "bytes": total_bytes}, ...} into buf (len
 * bytes, NUL-terminated; LES_ENOMEM if too short) and clears the records. */
les_status les_timing(les_ctx* ctx, int enable);
les_status les_timing_report(les_ctx* ctx, char* buf, size_t len);

/* ---------------------------------------------------------------- batched ensembles
 * Many triply periodic boxes of (possibly) different sizes, viscosities and lengths advanced
 * together: each kernel of the substep runs for all boxes in one launch (blocks assigned to
 * boxes by prefix sums of the boxes' block counts), every box keeps its own time step and
 * model coefficient, and a whole step can be replayed from one hipGraph.
 * Every box config must have zbc = PERIODIC, implicit_z = 0, ubulk = 0; all boxes share sgs
 * (NONE, SMAG or DSM) and precision.  Fields of all boxes are concatenated in one caller buffer
 * per field (box b starts at les_batch_offset), the workspace is one caller buffer. */
typedef struct les_batch les_batch;

les_status les_batch_init(const les_config* cfgs, int nbox, void* hip_stream, les_batch** out);
/* Total bytes of the concatenated U/V/W/P buffers (each) or of the workspace. */
les_status les_batch_layout(const les_batch* b, int field, les_layout_t* out);
/* Byte offset of box `box` inside the U/V/W/P buffers or the workspace. */
les_status les_batch_offset(const les_batch* b, int box, int field, int64_t* byte_offset);
les_status les_batch_bind(les_batch* b, int field, void* device_ptr);
/* Ghost planes and eddy viscosity of every box (once, after writing the initial fields). */
les_status les_batch_nut(les_batch* b);
/* Per-box CFL time step into each box's device slot (same rule as les_dt). */
les_status les_batch_dt(les_batch* b, double cfl);
les_status les_batch_set_dt(les_batch* b, double dt);
les_status les_batch_substep(les_batch* b, int stage);
/* Per-box time step (skipped when cfl = 0: the slots keep their values) and three substeps;
 * use_graph != 0 records them into a hipGraph on first use and replays it afterwards (the
 * graph keeps the cfl it was recorded with). */
les_status les_batch_step(les_batch* b, double cfl, int use_graph);
/* Time `substeps` batched substeps for each candidate of the dynamic-model chunk length and
 * of the FFT lines per block, keep the fastest, and write a JSON report into report (may be
 * NULL).  The timed substeps advance the bound state: call it before writing the initial
 * fields (the time-step slots must hold a positive value). */
les_status les_batch_autotune(les_batch* b, int substeps, char* report, size_t len);
/* Readable quantities and diagnostics of one box (as les_read / les_diag). */
les_status les_batch_read(les_batch* b, int box, int field, void* dst);
/* The ensemble as a training-data generator for the learned closure: box i draws n_per_box
 * training pairs from its current state as les_mlp_sample does with seed + i, into rows
 * [i n_per_box, (i + 1) n_per_box) of x_raw_dev (float[nbox n_per_box][7], raw inputs) and
 * y_dev (float[nbox n_per_box], the dynamic-model coefficient of the box).  Boxes with
 * sgs = DSM, after les_batch_nut or a batched substep; buffers are the caller's, on the
 * batch stream.  LES_EINVAL for n_per_box < 0 or null buffers, LES_ESTATE before the
 * batch is bound. */
les_status les_batch_mlp_sample(les_batch* b, uint64_t seed, int64_t n_per_box, float* x_raw_dev, float* y_dev);
les_status les_batch_diag(les_batch* b, int box, les_diag_t* out);
const char* les_batch_last_error(const les_batch* b);
les_status les_batch_free(les_batch* b);

/* Destroy the context (does not free caller memory). */
les_status les_free(les_ctx* ctx);

const char* les_strerror(les_status s);
/* Description of the context's last error.  With ctx NULL: the calling thread's last error of
 * les_mlp_grad_noalloc if it has failed on this thread, else "null context". */
const char* les_last_error(const les_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LES_H */
