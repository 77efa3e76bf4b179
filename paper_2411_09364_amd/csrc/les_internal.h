// Internal declarations shared by the library's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/les.h"

namespace les {

// ---------------------------------------------------------------------------- grid
// Plain-data view of the grid passed by value to every kernel.  Metric arrays live
// in the workspace (device memory) and are indexed by plane k = 0..nz+1.
struct GridP {
  int nx, ny, nz;
  int zbc;            // LES_ZBC_*
  int ywall;          // walls in y as well (square duct): two ghost rows after the interior
  int nys;            // stored rows per plane: ny, or ny + 2 with y walls
  int64_t sxy;        // plane stride nx * nys; the interior cells of a plane are its first nx * ny
  int nxp;            // row stride of the spectrum (complex values): nx/2+1 rounded up to 128 bytes
  double dx, dy, rdx, rdy;
  double lz, nu;
  const double* zc;   // [nz+2]
  const double* dzf;  // [nz+2]
  const double* dzc;  // [nz+1]
  const double* delta2;  // [nz+2] filter width squared per plane (ghosts copy neighbours)
  const double* rdzf;    // [nz+2] 1 / dzf, correctly rounded on the host (no division per wave)
  const double* rdzc;    // [nz+2] 1 / dzc
};

// Read of a table that no kernel writes while the reading kernel runs (grid metrics, plane
// coefficients, the time-step slot), through the constant address space: with a uniform
// index it becomes a scalar load, which does not wait behind the vector loads in flight.
template <typename T>
__device__ inline T ro_load(const T* p, int64_t i) {
  typedef const __attribute__((address_space(4))) T* cptr;
  return ((cptr)p)[i];
}

// Loads from one stored plane of a field through a raw buffer resource: the resource (scalar
// registers) holds the plane's base address, each lane a 32-bit element offset, so a load
// point costs one VGPR instead of a 64-bit pointer; offsets past the plane read 0.
template <typename T>
struct PlaneLoader {
  __amdgpu_buffer_rsrc_t r;
  __device__ PlaneLoader(const T* base, int64_t plane, int64_t sxy)
      : r(__builtin_amdgcn_make_buffer_rsrc((void*)(base + plane * sxy), (short)0, (int)(sxy * (int64_t)sizeof(T)),
                                            0x00020000)) {}
  __device__ T operator()(int off) const;
};
template <>
__device__ inline double PlaneLoader<double>::operator()(int off) const {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off * 8, 0, 0));
}
template <>
__device__ inline float PlaneLoader<float>::operator()(int off) const {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off * 4, 0, 0));
}

// Workgroup barrier that orders LDS only: it waits for the wave's LDS operations, not for
// its global loads and stores, so loads issued before it stay in flight.  For kernels whose
// threads exchange data through LDS only (each global location a thread reads is written by
// no other thread of the launch while it runs).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Advective time-step measure |u|/dx + |v|/dy + |w|/dzf of one cell from its face values
// (1/dzf from the table of reciprocals), every product and sum rounded on its own (no
// contraction into FMAs), so that the kernels that form it get the same bits.
__device__ inline double cfl_adv(double u, double v, double w, double rdx, double rdy, double rdzf) {
#pragma clang fp contract(off)
  return (fabs(u) * rdx + fabs(v) * rdy) + fabs(w) * rdzf;
}

// Block shape of the one-thread-per-cell tile launches (32 x 8 cells, narrower grids take
// their full width)
__host__ __device__ inline void tile_shape(int nx, int ny, int& bx, int& by) {
  bx = nx >= 32 ? 32 : nx;
  by = 256 / bx;
  if (by > 8 && bx == 32) by = 8;
  if (by > ny) by = ny;
}

__host__ __device__ inline int64_t idx3(const GridP& g, int k, int j, int i) {
  return ((int64_t)k * g.nys + j) * g.nx + i;
}
// Rows of the x-y tiles of the fused dynamic-model kernel (32 columns wide): 16 in FP64 (not in
// ducts), 8 in FP32 and in ducts.
constexpr int dsm_tile_rows(bool fp64) { return fp64 ? 16 : 8; }

// XCD-aware tile order.  Workgroups are dispatched to the 8 XCDs in turn by linear index;
// when a plane holds a multiple of 8 tiles, XCD x gets the contiguous band of tiles
// [x n/8, (x+1) n/8) of every plane, so tiles that are neighbours in y, and the same tile
// in the planes above and below, share that XCD's L2.
__device__ inline dim3 xcd_tile(dim3 bid, dim3 grid) {
  const unsigned n = grid.x * grid.y;
  if (n % 8 != 0) return bid;
  const unsigned t = bid.y * grid.x + bid.x;
  const unsigned tt = (t % 8) * (n / 8) + t / 8;
  return dim3(tt % grid.x, tt / grid.x, bid.z);
}

// Segmented-scan solve of tridiagonal chains with known factors (Thomas sweeps written as
// first-order linear recurrences: forward d_k = r_k f_k + alpha_k d_{k-1}, alpha_k = -a_k r_k,
// r_k = 1/pivot; back x_k = d_k - c'_k x_{k+1}).  The CG chains of a block are cut into
// segments of S rows, thread (cl, p) holding rows k0 = p S .. k0 + S - 1 (< n) of chain cl in
// v.  Each sweep runs over the segment from a zero start while carrying the product of its
// coefficients; the segment end values are folded in order through E, G ([segments][CG] in
// LDS) and every row is corrected by product x start value.  R(j), A(j), C(j) give r, a and
// c' of row k0 + j.  Contains barriers: every thread of the block calls it.
template <int S, int CG, class RF, class AF, class CF>
__device__ __forceinline__ void seg_scan_solve(double (&v)[S], int k0, int n, int p, int P, int cl,
                                               double (*E)[CG], double (*G)[CG], const RF& R, const AF& A,
                                               const CF& C) {
  double dl = 0.0, pr = 1.0;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    if (k0 + j < n) {
      const double al = -A(j) * R(j);
      dl = R(j) * v[j] + al * dl;
      pr = al * pr;
      v[j] = dl;
    }
  }
  E[p][cl] = dl;
  G[p][cl] = pr;
  __syncthreads();
  double D = 0.0;
  for (int q = 0; q < p; ++q) D = E[q][cl] + G[q][cl] * D;
  pr = 1.0;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    if (k0 + j < n) {
      pr *= -A(j) * R(j);
      v[j] += pr * D;
    }
  }
  double xl = 0.0, ps = 1.0;
#pragma unroll
  for (int j = S - 1; j >= 0; --j) {
    if (k0 + j < n) {
      xl = v[j] - C(j) * xl;
      ps = -C(j) * ps;
      v[j] = xl;
    }
  }
  __syncthreads();
  E[p][cl] = xl;
  G[p][cl] = ps;
  __syncthreads();
  double X = 0.0;
  for (int q = P - 1; q > p; --q) X = E[q][cl] + G[q][cl] * X;
  ps = 1.0;
#pragma unroll
  for (int j = S - 1; j >= 0; --j) {
    if (k0 + j < n) {
      ps *= -C(j);
      v[j] += ps * X;
    }
  }
}

__device__ inline int wrap_p(int i, int n) { return i + 1 == n ? 0 : i + 1; }
// y modes with their own z factors: m <= ny/2 (periodic y), every m (ducts)
__host__ __device__ inline int factor_modes(const GridP& g) { return g.ywall ? g.ny : g.ny / 2 + 1; }
__device__ inline int wrap_m(int i, int n) { return i == 0 ? n - 1 : i - 1; }

// Radix plan of an LDS Stockham FFT (radix 3 first, then 4s, then a 2).
struct FftPlan {
  int n;
  int nst;
  int rad[16];
};
FftPlan make_plan(int n);

// Device-side tables carved out of the workspace.
struct Tables {
  double* zc;       // nz+2
  double* dzf;      // nz+2
  double* dzc;      // nz+1 (padded)
  double* delta2;   // nz+2
  double* rdzf;     // nz+2: 1 / dzf
  double* rdzc;     // nz+2: 1 / dzc
  double* coef;     // nz+2: nu_t = coef[k] * nut_field (see les.cpp)
  double* cs;       // nz: dynamic coefficient per plane
  double* pa;       // nz: Poisson z rows (lower)
  double* pb;       // nz: (diagonal without eigenvalues)
  double* pc;       // nz: (upper)
  double* lamx;     // nx/2+1
  double* lamy;     // ny
  double* lamz;     // nz (periodic z)
  double* twx;      // 2*nx : cos, sin pairs of exp(-2 pi i q/nx)
  double* twy;      // 2*ny
  double* twz;      // 2*nz
  float* twx_f;     // float copies
  float* twy_f;
  float* twz_f;
  double2* hfac3;   // CN in all directions, walls: per-substep z factor pairs, u/v rows then w rows,
                    //   each [nz][ny/2+1][nxp]
  double* hfac;     // 12*nz: CN factorisation: c', 1/pivot for u/v rows and for w rows, the
                    //   flow-rate profile q, unused, sub-diagonals (u/v, w), diagonals and
                    //   super-diagonals (u/v, w)
  double* dt;       // [0] time step; [1] bulk shift s; [2..] scratch scalars
  double* red;      // reduction partials (size red_n)
  double* bulk;     // flow-rate partial sums, one per forward-x block
  double* tau;      // 4*sxy wall stresses of the z walls
  double* utau;     // 4*sxy Newton state
  double* tauy;     // ducts: 4*(nz+2)*nx stresses of the y walls (tau_x, tau_z at y = 0, then y = ly)
  double* utauy;    // ducts: their Newton state
  double* vd4;      // ducts, van Driest: friction velocity of the z bottom, z top, y = 0, y = ly walls
  double* twc;      // ducts: 2*ny cos, sin of pi m / (2 ny), the cosine transform's twiddles
  float* twc_f;
  double* dsm_part; // plane partial sums (LM, MM) per tile and wave of the fused dynamic model
  double* cflc;     // 4 per block of the last correction: max |u|/dx + |v|/dy + |w|/dzf per wave
  double* pfac;     // walls: (c', 1/pivot) of the (l, m) z systems, [nz][nm][nxp] pairs with
                    //   nm = ny/2+1 (periodic y: m and ny - m share them) or ny (ducts)
  double* stats;    // statistics: header[8], sums [11][nz], wall-stress series [cap][2]
  double* stats_part; // per-block plane partials of one sample [nz+1][nblk][11]
  int64_t red_n;
  int nblk_xy;      // number of x-y tiles used by plane reductions
};

// Per-context state (host side).
struct Ctx {
  les_config cfg;
  hipStream_t stream;
  GridP g;               // device metric pointers filled at workspace bind
  // host copies of the tables
  std::vector<double> zf, zc, dzf, dzc, delta2, pa, pb, pc, lamx, lamy, lamz, rdzf, rdzc;
  std::vector<double> twx, twy, twz, twc;
  // host staging of uploaded tables (kept alive for the asynchronous copies)
  std::vector<float> twx_f_host, twy_f_host, twz_f_host, twc_f_host;
  std::vector<double> coef_host, hfac_host;
  // bound buffers
  void* u = nullptr;
  void* v = nullptr;
  void* w = nullptr;
  void* p = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  size_t field_elems = 0;   // (nz+2)*nys*nx
  size_t elem = 8;          // storage bytes
  // workspace carving (byte offsets into ws)
  Tables t{};
  void* ru = nullptr;  void* rv = nullptr;  void* rw = nullptr;   // RK history R^{k-1}
  void* us = nullptr;  void* vs = nullptr;  void* wsf = nullptr;  // u*, v*, w*
  void* nut = nullptr;    // |S| (all Smagorinsky variants) or learned nu_t/Delta^2
  void* phi = nullptr;    // pressure correction (field layout)
  void* spec = nullptr;   // complex spectrum [nz][ny][nx/2+1]
  int dsm_kc = 8;         // planes per z chunk of the fused dynamic-model kernel
  int mlp_kc = 8;         // planes per z chunk of the learned-closure inference kernel
  int pred_kc = 8;        // planes per z chunk of the z-marching predictor
  int pred_ty = 8;        // rows of the predictor's 32-wide tiles: 8 or 16
  // time step: the advective maxima taken by the correction's blocks (unless LES_CFL_PASS=1),
  // usable while the fields are those that correction wrote
  bool cfl_fold = true;
  bool cfl_adv_ready = false;
  int bulk_nblk = 0;      // forward-x flow-rate partials awaiting the shift (spectral_solve forms it)
  // learned closure
  float* mlp_params = nullptr;   // caller-owned float32 parameters (les_mlp_bind)
  double mlp_lo[7], mlp_hi[7];    // feature ranges for min-max scaling
  int* mlp_cnt = nullptr;         // [2] fallback counters in the workspace
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool initialised = false;  // les_nut called
  // per-launch timing (HIP events on the context stream), enabled by les_timing
  struct Timed {
    const char* name;
    hipEvent_t a, b;
    double bytes;
  };
  bool timing = false;
  std::vector<Timed> timed;
  std::string err;
};

// kernel launchers (defined in the .hip files)
template <typename T> void launch_predictor(Ctx& c, int stage);
template <typename T> void launch_helmholtz(Ctx& c, int stage);
template <typename T> void launch_helmholtz_3d(Ctx& c, int stage);
template <typename T> void launch_poisson_rhs_fwd(Ctx& c, const T* us, const T* vs, const T* ws, double scale_by_gamma_dt, int stage);
template <typename T> void launch_poisson_solve_spectral(Ctx& c);
void launch_thomas_factor(Ctx& c);
template <typename T> void launch_poisson_inverse(Ctx& c, T* phi_out);
template <typename T> void launch_correct(Ctx& c, int stage);
template <typename T> void launch_bc_fill(Ctx& c, T* u, T* v, T* w, T* p);
template <typename T> void launch_wallmodel(Ctx& c);
// ducts: y-wall model, y ghost rows of u, v, w, p (Alg. 2) and of the eddy viscosity
template <typename T> void launch_wallmodel_y(Ctx& c);
template <typename T> void launch_bc_fill_y(Ctx& c, T* u, T* v, T* w, T* p);
template <typename T> void launch_fill_y_scalar(Ctx& c, T* f, double sign);
template <typename T> void launch_eddy_viscosity(Ctx& c);
template <typename T> void launch_dt(Ctx& c, double cfl);
template <typename T> void launch_poisson_field(Ctx& c, T* f);
template <typename T> void launch_project(Ctx& c);
template <typename T> void launch_read_nut(Ctx& c, T* dst);
template <typename T> void launch_diag(Ctx& c, double* out_dev);
template <typename T> void launch_mlp_sample(Ctx& c, uint64_t seed, int64_t n, float* x, float* y);
int64_t mlp_grad_blocks(int64_t n);
void launch_mlp_forward(hipStream_t st, const float* P, const float* x, int64_t n, float* y);
void launch_mlp_grad(hipStream_t st, const float* P, const float* x, const float* t, int64_t n, float* part,
                     float* grad, float* loss);
void launch_mlp_adam(hipStream_t st, float* P, const float* g, float* m, float* v, int step, float lr);
// blocks of k_mlp_grad at the largest sample count of the allocation-free gradient
constexpr int MLP_NOALLOC_BLOCKS = LES_MLP_NOALLOC_MAX_SAMPLES / 256;
// device address of this device's partial-gradient array (looked up on first use per device)
hipError_t mlp_scratch_ptr(int device, float** out);
void launch_mlp_normalize(hipStream_t st, const float* xr, int64_t n, const double* lo, const double* hi, float* x);
void launch_set_dt(Ctx& c, double dt);
int stats_blocks(int64_t sxy);
int64_t stats_words(const GridP& g);
int64_t stats_part_words(int nz, int64_t sxy);
void launch_stats_reset(Ctx& c);
template <typename T> void launch_stats_sample(Ctx& c);
void stats_finalize(const Ctx& c, const double* st, int nbatch, les_stats_t* out, double* prof);

// Kernel launch on the context stream.  With timing enabled the launch is bracketed by
// two HIP events and tagged with its algorithmic byte count (minimum HBM traffic of the
// kernel as designed: each input and output array touched once).
#define LES_LAUNCH(ctx, name, bytes, kernel, grid, block, shmem, ...)                          \
  do {                                                                                          \
    hipEvent_t les_ev_a_ = nullptr, les_ev_b_ = nullptr;                                        \
    if ((ctx).timing) {                                                                         \
      (void)hipEventCreate(&les_ev_a_);                                                         \
      (void)hipEventCreate(&les_ev_b_);                                                         \
      (void)hipEventRecord(les_ev_a_, (ctx).stream);                                            \
    }                                                                                           \
    hipLaunchKernelGGL(kernel, grid, block, shmem, (ctx).stream, __VA_ARGS__);                  \
    if ((ctx).timing) {                                                                         \
      (void)hipEventRecord(les_ev_b_, (ctx).stream);                                            \
      (ctx).timed.push_back({name, les_ev_a_, les_ev_b_, (double)(bytes)});                     \
    }                                                                                           \
  } while (0)

// launch geometry for one-thread-per-point kernels over interior planes
struct Launch3 {
  dim3 grid, block;
};
Launch3 point_launch(const GridP& g, int planes);

// ---------------------------------------------------------------------------- batches
// Kernel kinds of a batched substep; each batched launch covers all boxes, block b of the
// launch belongs to the box whose prefix range holds b.
enum BatchKind { BK_POINT = 0, BK_RFFTX, BK_FFTY, BK_FFTZ, BK_DSM, BK_DSMRED, BK_CFL, BK_PRED, BK_NKIND };

// Everything a batched kernel needs to run one box (device memory, one per box).
struct BoxDesc {
  GridP g;
  void *u, *v, *w, *p;
  void *ru, *rv, *rw, *us, *vs, *wsf, *nut, *phi, *spec;
  double *coef, *cs, *dt, *red, *dsm_part, *lamx, *lamy, *lamz, *twx, *twy, *twz;
  float *twx_f, *twy_f, *twz_f;
  FftPlan px, py, pz;
  int pbx;              // x-row pairs per forward/inverse x block
  int ly, lz;           // lines per y / z FFT block
  int kc;               // planes per dynamic-model chunk
  int pkc;              // planes per predictor chunk
  int sgs;
  double cs_smag;       // static coefficient (SMAG)
  int gdim[BK_NKIND][3];  // per-kind block grid of this box
};

// Batch lookup: prefix[kind][box] = first block of box, prefix[kind][nbox] = total.
constexpr int kMaxBox = 256;
struct BatchMap {
  const BoxDesc* desc;
  const int* prefix;    // [BK_NKIND][nbox + 1]
  int nbox;
};

__device__ inline int batch_box(const BatchMap& m, int kind, int b) {
  const int* pre = m.prefix + kind * (m.nbox + 1);
  int lo = 0, hi = m.nbox;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (pre[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Block index of block b of a batched launch inside its box's own grid.
__device__ inline dim3 batch_bid(const BatchMap& m, int kind, int b, int& box) {
  box = batch_box(m, kind, b);
  const int* pre = m.prefix + kind * (m.nbox + 1);
  const int local = b - pre[box];
  const int* gd = m.desc[box].gdim[kind];
  return dim3(local % gd[0], (local / gd[0]) % gd[1], local / (gd[0] * gd[1]));
}

// batch launchers (all boxes of a batch in one launch per kernel kind)
template <typename T> void batch_predictor(hipStream_t st, const BatchMap& m, int total, int stage);
template <typename T> void batch_correct(hipStream_t st, const BatchMap& m, int total, int stage);
template <typename T> void batch_dt(hipStream_t st, const BatchMap& m, int total_cfl, int nbox, double cfl);
void batch_set_dt(hipStream_t st, const BatchMap& m, int nbox, double dt);
template <typename T>
void batch_poisson(hipStream_t st, const BatchMap& m, const int* totals, size_t sh_x, size_t sh_y, size_t sh_z,
                   int stage);
template <typename T>
void batch_eddy_viscosity(hipStream_t st, const BatchMap& m, const int* totals, int any_dsm, int any_smag);
int fft_pairs_per_block(int nx);
int fft_lines_per_block(int n);

}  // namespace les

// opaque ABI handle of one context
struct les_ctx {
  les::Ctx c;
};
