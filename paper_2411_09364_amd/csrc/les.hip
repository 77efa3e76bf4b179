// C ABI of the substep library (declarations and argument contracts in include/les.h):
// validation, host-side grid metrics and solver tables, workspace carving, and the
// kernel schedule of one RK3 substep (Alg. 1) with the boundary order of Alg. 2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "les_internal.h"

using namespace les;

namespace {

const double kPi = 3.14159265358979323846;

bool fft_size_ok(int n) {
  if (n < 4 || n > 1024) return false;
  int m = n;
  if (m % 5 == 0) m /= 5;
  if (m % 3 == 0) m /= 3;
  while (m % 2 == 0) m /= 2;
  return m == 1;
}

les_status fail(Ctx* c, les_status s, const char* msg) {
  if (c) c->err = msg;
  return s;
}

les_status check_hip(Ctx& c, hipError_t e, const char* where) {
  if (e == hipSuccess) return LES_OK;
  c.err = std::string(where) + ": " + hipGetErrorString(e);
  return LES_EDEVICE;
}

les_status check_launch(Ctx& c, const char* where) {
  return check_hip(c, hipGetLastError(), where);
}

// Wall-normal faces: uniform, or tanh clustering zf(k) = (lz/2)[1 + tanh(beta(2k/nz - 1))/tanh(beta)]
// made exactly mirror-symmetric (the lower half is snapped so that lz - zf is exact).
void build_grid(Ctx& c) {
  const les_config& f = c.cfg;
  const int n = f.nz;
  c.zf.assign(n + 1, 0.0);
  const bool stretch = f.zbc != LES_ZBC_PERIODIC && f.beta > 0.0;
  for (int k = 0; k <= n; ++k) {
    if (stretch)
      c.zf[k] = 0.5 * f.lz * (1.0 + std::tanh(f.beta * (2.0 * k / n - 1.0)) / std::tanh(f.beta));
    else
      c.zf[k] = f.lz * k / n;
  }
  if (stretch) {
    for (int k = 0; k < (n + 1) / 2; ++k) {
      const double b = f.lz - c.zf[k];
      c.zf[n - k] = b;
      c.zf[k] = f.lz - b;
    }
    if (n % 2 == 0) c.zf[n / 2] = 0.5 * f.lz;
  }
  c.zf[0] = 0.0;
  c.zf[n] = f.lz;
  c.zc.assign(n + 2, 0.0);
  c.dzf.assign(n + 2, 0.0);
  for (int k = 1; k <= n; ++k) {
    c.zc[k] = 0.5 * (c.zf[k - 1] + c.zf[k]);
    c.dzf[k] = c.zf[k] - c.zf[k - 1];
  }
  if (f.zbc == LES_ZBC_PERIODIC) {
    c.zc[0] = c.zc[n] - f.lz;
    c.zc[n + 1] = c.zc[1] + f.lz;
    c.dzf[0] = c.dzf[n];
    c.dzf[n + 1] = c.dzf[1];
  } else {
    c.zc[0] = -c.zc[1];
    c.zc[n + 1] = 2.0 * f.lz - c.zc[n];
    c.dzf[0] = c.dzf[1];
    c.dzf[n + 1] = c.dzf[n];
  }
  c.dzc.assign(n + 2, 0.0);
  for (int k = 0; k <= n; ++k) c.dzc[k] = c.zc[k + 1] - c.zc[k];
  c.dzc[n + 1] = c.dzc[n];
  c.rdzf.assign(n + 2, 0.0);
  c.rdzc.assign(n + 2, 0.0);
  for (int k = 0; k <= n + 1; ++k) {
    c.rdzf[k] = 1.0 / c.dzf[k];
    c.rdzc[k] = 1.0 / c.dzc[k];
  }
  const double dx = f.lx / f.nx, dy = f.ly / f.ny;
  c.delta2.assign(n + 2, 0.0);
  for (int k = 0; k <= n + 1; ++k) {
    const double d = std::pow(dx * dy * c.dzf[k], 1.0 / 3.0);
    c.delta2[k] = d * d;
  }
  // Poisson rows of D G along z (zero flux through walls)
  c.pa.assign(n, 0.0);
  c.pb.assign(n, 0.0);
  c.pc.assign(n, 0.0);
  for (int k = 1; k <= n; ++k) {
    double a = 1.0 / (c.dzc[k - 1] * c.dzf[k]);
    double cc = 1.0 / (c.dzc[k] * c.dzf[k]);
    if (f.zbc != LES_ZBC_PERIODIC) {
      if (k == 1) a = 0.0;
      if (k == n) cc = 0.0;
    }
    c.pa[k - 1] = a;
    c.pc[k - 1] = cc;
    c.pb[k - 1] = -(a + cc);
  }
  // eigenvalues of the periodic second difference, -(4/h^2) sin^2(pi l/n)
  auto eig = [](int nn, double h, int l) {
    const double s = std::sin(kPi * l / nn);
    return -(4.0 / (h * h)) * s * s;
  };
  c.lamx.resize(f.nx / 2 + 1);
  for (int l = 0; l <= f.nx / 2; ++l) c.lamx[l] = eig(f.nx, dx, l);
  c.lamy.resize(f.ny);
  if (f.ybc == LES_YBC_WALL) {
    // walls in y: the cosine modes of the zero-flux second difference,
    // -(4/dy^2) sin^2(pi m / (2 ny)), m = 0..ny-1
    for (int m = 0; m < f.ny; ++m) {
      const double s = std::sin(kPi * m / (2.0 * f.ny));
      c.lamy[m] = -(4.0 / (dy * dy)) * s * s;
    }
  } else {
    // y modes m and ny - m share their eigenvalue exactly (mirrored), so their z systems and
    // factors coincide
    for (int m = 0; m <= f.ny / 2; ++m) c.lamy[m] = eig(f.ny, dy, m);
    for (int m = f.ny / 2 + 1; m < f.ny; ++m) c.lamy[m] = c.lamy[f.ny - m];
  }
  c.lamz.assign(n, 0.0);
  if (f.zbc == LES_ZBC_PERIODIC)
    for (int q = 0; q < n; ++q) c.lamz[q] = eig(n, f.lz / n, q);
  auto tw = [](int nn, std::vector<double>& t) {
    t.resize(2 * nn);
    for (int q = 0; q < nn; ++q) {
      t[2 * q] = std::cos(2.0 * kPi * q / nn);
      t[2 * q + 1] = std::sin(2.0 * kPi * q / nn);
    }
  };
  tw(f.nx, c.twx);
  tw(f.ny, c.twy);
  tw(n, c.twz);
  // cosine transform (ducts): cos, sin of pi m / (2 ny)
  c.twc.resize(2 * f.ny);
  for (int m = 0; m < f.ny; ++m) {
    c.twc[2 * m] = std::cos(kPi * m / (2.0 * f.ny));
    c.twc[2 * m + 1] = std::sin(kPi * m / (2.0 * f.ny));
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace layout.  With base == nullptr only the size is computed.
size_t carve(Ctx& c, char* base) {
  const les_config& f = c.cfg;
  const int n = f.nz;
  const size_t F = c.field_elems, E = c.elem;
  const int64_t sxy = c.g.sxy;   // stored rows (ghost rows of ducts included)
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = align256(off + bytes);
    return p;
  };
  Tables& t = c.t;
  t.zc = (double*)take((n + 2) * 8);
  t.dzf = (double*)take((n + 2) * 8);
  t.dzc = (double*)take((n + 2) * 8);
  t.delta2 = (double*)take((n + 2) * 8);
  t.rdzf = (double*)take((n + 2) * 8);
  t.rdzc = (double*)take((n + 2) * 8);
  t.coef = (double*)take((n + 2) * 8);
  t.cs = (double*)take((f.ybc == LES_YBC_WALL ? (size_t)n * f.ny : n) * 8);   // per plane, or per x line
  t.pa = (double*)take(n * 8);
  t.pb = (double*)take(n * 8);
  t.pc = (double*)take(n * 8);
  t.lamx = (double*)take((f.nx / 2 + 1) * 8);
  t.lamy = (double*)take(f.ny * 8);
  t.lamz = (double*)take(n * 8);
  t.twx = (double*)take(2 * f.nx * 8);
  t.twy = (double*)take(2 * f.ny * 8);
  t.twz = (double*)take(2 * n * 8);
  t.twx_f = (float*)take(2 * f.nx * 4);
  t.twy_f = (float*)take(2 * f.ny * 4);
  t.twz_f = (float*)take(2 * n * 4);
  t.hfac = (double*)take(14 * n * 8);
  t.dt = (double*)take(16 * 8);
  c.mlp_cnt = (int*)take(4 * sizeof(int));   // [0, 1] fallback counters, [2] wall-mean ticket
  t.red_n = 4096;
  t.red = (double*)take(t.red_n * 8);
  const int64_t npairs = (int64_t)n * (f.ny / 2);
  t.bulk = (double*)take((size_t)std::max<int64_t>(npairs, 1) * 8);
  t.tau = (double*)take(4 * sxy * 8);
  t.utau = (double*)take(4 * sxy * 8);
  const bool duct = f.ybc == LES_YBC_WALL;
  t.tauy = (double*)take(duct ? 4 * (size_t)(n + 2) * f.nx * 8 : 0);
  t.utauy = (double*)take(duct ? 4 * (size_t)(n + 2) * f.nx * 8 : 0);
  t.vd4 = (double*)take(4 * 8);
  t.twc = (double*)take(2 * f.ny * 8);
  t.twc_f = (float*)take(2 * f.ny * 4);
  // plane partial sums (LM, MM): one per wave of each x-y tile of the fused dynamic-model
  // kernel (32 x 8 cells, 4 waves)
  t.nblk_xy = ((f.nx + 31) / 32) * ((f.ny + 7) / 8);
  {
    // z chunk lengths in units of 32 x 8 tiles on 256 CUs: whole rounds of resident blocks, at
    // least 8 planes (the dynamic model's FP64 block covers two such tiles, one block per CU;
    // the learned-closure inference runs four blocks per CU on chunks sized for three, which
    // measured faster than chunks for four)
    auto chunk = [&](int64_t slots) {
      const int64_t want = ((int64_t)n * t.nblk_xy + slots - 1) / slots;
      return (int)std::max<int64_t>(std::min<int64_t>(8, n), std::min<int64_t>(n, want));
    };
    // the fewest chunks that make the launch a whole number of rounds (at least one), when
    // their length stays at 8 planes or more (0 if there are none); chunk_rounds falls back
    // to chunk
    auto whole_rounds = [&](int64_t slots) {
      for (int64_t nch = 1; nch <= n; ++nch) {
        const int64_t blocks = nch * t.nblk_xy;
        if (blocks < slots || blocks % slots != 0) continue;
        const int64_t kc = (n + nch - 1) / nch;
        if (kc < std::min<int64_t>(8, n)) break;
        return (int)kc;
      }
      return 0;
    };
    auto chunk_rounds = [&](int64_t slots) {
      const int kc = whole_rounds(slots);
      return kc > 0 ? kc : chunk(slots);
    };
    c.dsm_kc = chunk(512);
    c.mlp_kc = chunk(768);
    // z-marching predictor: 32 x 16 tiles, at one 512-thread block per CU in FP64 and two in
    // FP32, fetch less halo than 32 x 8 tiles at three (FP64) or four (FP32) blocks per CU
    // (measured faster on 3, 17 and 134 M-cell channels) and are taken when their launch makes
    // whole rounds; else 32 x 8.  LES_PRED_TILE_ROWS (8 or 16) overrides.  Slots in units of
    // 32 x 8 tiles: a 32 x 16 block covers two.
    const bool mixed = f.precision == LES_MIXED;
    const int slots16 = mixed ? 1024 : 512;
    c.pred_ty = f.ny % 16 == 0 && whole_rounds(slots16) > 0 ? 16 : 8;
    // LES_CFL_PASS=1: the time step's advective maxima always take a pass of their own
    if (const char* e = std::getenv("LES_CFL_PASS")) c.cfl_fold = std::atoi(e) != 1;
    if (const char* e = std::getenv("LES_PRED_TILE_ROWS")) {
      const int r = std::atoi(e);
      if (r == 8 || r == 16) c.pred_ty = r;
    }
    c.pred_kc = chunk_rounds(c.pred_ty == 16 ? slots16 : (mixed ? 1024 : 768));
  }
  // ducts: one partial per x line and x tile, [nz][ny][nx/32]
  // per (plane, tile, wave) of the fused dynamic-model kernel, or per (plane, row, x tile)
  const int dty = dsm_tile_rows(f.precision != LES_MIXED);
  const size_t dsm_waves = (size_t)((f.nx + 31) / 32) * ((f.ny + dty - 1) / dty) * (32 * dty / 64);
  t.dsm_part = (double*)take(std::max((size_t)2 * n * dsm_waves, (size_t)2 * n * f.ny * ((f.nx + 31) / 32)) * 8);
  {
    int bx, by;
    tile_shape(f.nx, f.ny, bx, by);
    t.cflc = (double*)take((size_t)4 * ((f.nx + bx - 1) / bx) * ((f.ny + by - 1) / by) * n * 8);
  }
  c.ru = take(F * E);
  c.rv = take(F * E);
  c.rw = take(F * E);
  c.us = take(F * E);
  c.vs = take(F * E);
  c.wsf = take(F * E);
  c.nut = take(F * E);
  c.phi = take(F * E);
  const size_t rq = f.precision == LES_MIXED ? 16 : 8;
  const size_t nxp = ((size_t)(f.nx / 2 + 1) + rq - 1) / rq * rq;
  // one spectrum buffer; three with CN in all directions (the components are solved together)
  c.spec = take(nxp * f.ny * n * 2 * E * (f.implicit_z == LES_VISC_CN_3D ? 3 : 1));
  // factor pairs of the z systems of every (l, m) column with its own factors (walls only)
  t.pfac = (double*)take(f.zbc == LES_ZBC_PERIODIC ? 0 : nxp * factor_modes(c.g) * n * 2 * 8);
  // long-run statistics: running sums and series, per-sample partials
  t.stats = (double*)take(8 * stats_words(c.g));
  t.stats_part = (double*)take(8 * stats_part_words(n, (int64_t)f.nx * f.ny));
  // per-substep factor pairs of the Helmholtz z systems (CN in all directions, walls)
  t.hfac3 = (double2*)take(f.zbc != LES_ZBC_PERIODIC && f.implicit_z == LES_VISC_CN_3D
                               ? 2 * nxp * (f.ny / 2 + 1) * n * 16 : 0);
  return off;
}

// After an update of u, v, w, p (Alg. 2, then Alg. 1's last line): the wall stresses from the
// interior values, the wall-model ghosts, the y ghost rows of ducts, and the eddy viscosity
// with its ghosts.  Both wall models read interior values and wall faces only, so the stale
// y ghost rows they see do not matter.
template <typename T>
void boundary_and_model(Ctx& c) {
  if (c.cfg.zbc == LES_ZBC_WALLMODEL) {
    launch_wallmodel<T>(c);
    if (c.g.ywall) launch_wallmodel_y<T>(c);
  }
  if (c.g.ywall) launch_bc_fill_y<T>(c, (T*)c.u, (T*)c.v, (T*)c.w, (T*)c.p);
  launch_eddy_viscosity<T>(c);
  if (c.g.ywall) launch_fill_y_scalar<T>(c, (T*)c.nut, -1.0);
}

template <typename T>
les_status substep_body(Ctx& c, int stage) {
  static const double G[3] = {8.0 / 15.0, 2.0 / 15.0, 1.0 / 3.0};
  launch_predictor<T>(c, stage);
  if (c.cfg.implicit_z == LES_VISC_CN_Z) launch_helmholtz<T>(c, stage);
  if (c.cfg.implicit_z == LES_VISC_CN_3D) launch_helmholtz_3d<T>(c, stage);
  launch_poisson_rhs_fwd<T>(c, (const T*)c.us, (const T*)c.vs, (const T*)c.wsf, G[stage], stage);
  launch_poisson_solve_spectral<T>(c);
  launch_poisson_inverse<T>(c, (T*)c.phi);
  launch_correct<T>(c, stage);
  boundary_and_model<T>(c);
  return check_launch(c, "les_substep");
}

les_status substep_any(Ctx& c, int stage) {
  return c.cfg.precision == LES_MIXED ? substep_body<float>(c, stage) : substep_body<double>(c, stage);
}

les_status ready(Ctx& c, bool need_init) {
  if (!c.u || !c.v || !c.w || !c.p || !c.ws) return fail(&c, LES_ESTATE, "fields and workspace must be bound");
  if (need_init && !c.initialised) return fail(&c, LES_ESTATE, "les_nut must be called before stepping");
  return LES_OK;
}

}  // namespace

extern "C" {

const char* les_strerror(les_status s) {
  switch (s) {
    case LES_OK: return "ok";
    case LES_EINVAL: return "invalid argument";
    case LES_ENOMEM: return "buffer too small";
    case LES_EDEVICE: return "device error";
    case LES_ENOTSUP: return "unsupported configuration";
    case LES_ENONFINITE: return "non-finite state";
    case LES_ESTATE: return "call out of order";
  }
  return "unknown status";
}

// last error of a context-free call that reports one (les_mlp_grad_noalloc), per thread
static thread_local std::string t_free_err;

const char* les_last_error(const les_ctx* ctx) {
  if (ctx) return ctx->c.err.c_str();
  return t_free_err.empty() ? "null context" : t_free_err.c_str();
}

les_status les_init(const les_config* cfg, void* hip_stream, les_ctx** out) {
  if (!out) return LES_EINVAL;
  *out = nullptr;
  if (!cfg) return LES_EINVAL;
  if (cfg->abi_version != LES_ABI_VERSION) return LES_EINVAL;
  const les_config& f = *cfg;
  if (!fft_size_ok(f.nx) || !fft_size_ok(f.ny) || f.nx % 2 || f.ny % 2) return LES_ENOTSUP;
  if (f.zbc < 0 || f.zbc > 2) return LES_EINVAL;
  if (f.zbc == LES_ZBC_PERIODIC) {
    if (!fft_size_ok(f.nz)) return LES_ENOTSUP;
  } else if (f.nz < 4 || f.nz > 512) {
    return LES_EINVAL;
  }
  auto pos = [](double x) { return std::isfinite(x) && x > 0.0; };
  if (!pos(f.lx) || !pos(f.ly) || !pos(f.lz) || !pos(f.nu)) return LES_EINVAL;
  if (!(std::isfinite(f.beta) && f.beta >= 0.0 && f.beta < 20.0)) return LES_EINVAL;
  if (f.sgs < 0 || f.sgs > 4) return LES_EINVAL;
  if (!(std::isfinite(f.cs) && f.cs >= 0.0)) return LES_EINVAL;
  if (f.implicit_z < LES_VISC_EXPLICIT || f.implicit_z > LES_VISC_CN_3D) return LES_EINVAL;
  if (f.implicit_z == LES_VISC_CN_Z && f.zbc == LES_ZBC_PERIODIC) return LES_ENOTSUP;
  if (f.precision != LES_FP64 && f.precision != LES_MIXED) return LES_EINVAL;
  if (!(std::isfinite(f.ubulk) && f.ubulk >= 0.0)) return LES_EINVAL;
  if (!(std::isfinite(f.h_wm) && f.h_wm >= 0.0)) return LES_EINVAL;
  if (!(std::isfinite(f.kappa) && f.kappa >= 0.0) || !std::isfinite(f.bconst)) return LES_EINVAL;
  if (f.ybc != LES_YBC_PERIODIC && f.ybc != LES_YBC_WALL) return LES_EINVAL;
  if (f.ybc == LES_YBC_WALL) {
    // square duct: walls in z as well, no implicit y solve
    if (f.zbc == LES_ZBC_PERIODIC || f.implicit_z == LES_VISC_CN_3D || f.ny < 4)
      return LES_ENOTSUP;
    if (f.zbc == LES_ZBC_WALLMODEL && f.h_wm > 0.0) {
      const double dy = f.ly / f.ny;
      if (f.h_wm < 0.5 * dy || f.h_wm > (f.ny / 2 - 0.5) * dy) return LES_EINVAL;
    }
  }
  les_ctx* h = new (std::nothrow) les_ctx();
  if (!h) return LES_ENOMEM;
  Ctx& c = h->c;
  c.cfg = f;
  if (c.cfg.kappa == 0.0) c.cfg.kappa = 0.41;
  if (c.cfg.bconst == 0.0) c.cfg.bconst = 5.2;
  c.stream = (hipStream_t)hip_stream;
  c.elem = f.precision == LES_MIXED ? 4 : 8;
  const int nys = f.ybc == LES_YBC_WALL ? f.ny + 2 : f.ny;
  c.field_elems = (size_t)(f.nz + 2) * nys * f.nx;
  build_grid(c);
  if (f.zbc == LES_ZBC_WALLMODEL && f.h_wm > 0.0) {
    if (f.h_wm < c.zc[1] || f.h_wm > c.zc[f.nz / 2]) {
      delete h;
      return LES_EINVAL;
    }
  }
  GridP& g = c.g;
  g.nx = f.nx;
  g.ny = f.ny;
  g.nz = f.nz;
  g.zbc = f.zbc;
  g.ywall = f.ybc == LES_YBC_WALL ? 1 : 0;
  g.nys = nys;
  g.sxy = (int64_t)f.nx * nys;
  // 128-byte spectrum rows: 8 double or 16 float complex values
  const int rq = f.precision == LES_MIXED ? 16 : 8;
  g.nxp = ((f.nx / 2 + 1) + rq - 1) / rq * rq;
  g.dx = f.lx / f.nx;
  g.dy = f.ly / f.ny;
  g.rdx = 1.0 / g.dx;
  g.rdy = 1.0 / g.dy;
  g.lz = f.lz;
  g.nu = f.nu;
  c.ws_bytes = carve(c, nullptr);
  *out = h;
  return LES_OK;
}

les_status les_layout(const les_ctx* ctx, int field, les_layout_t* out) {
  if (!ctx || !out) return LES_EINVAL;
  const Ctx& c = ctx->c;
  const les_config& f = c.cfg;
  std::memset(out, 0, sizeof(*out));
  out->nx = f.nx;
  out->ny = f.ny;
  out->nz = f.nz;
  out->dims[0] = f.nz + 2;
  out->dims[1] = c.g.nys;
  out->dims[2] = f.nx;
  out->elem_bytes = (int64_t)c.elem;
  switch (field) {
    case LES_FIELD_U: case LES_FIELD_V: case LES_FIELD_W: case LES_FIELD_P: case LES_FIELD_NUT:
      out->bytes = (int64_t)(c.field_elems * c.elem);
      return LES_OK;
    case LES_FIELD_WORKSPACE:
      out->bytes = (int64_t)c.ws_bytes;
      out->elem_bytes = 1;
      return LES_OK;
    case LES_FIELD_CS:
      out->bytes = 8LL * f.nz * (f.ybc == LES_YBC_WALL ? f.ny : 1);
      out->elem_bytes = 8;
      return LES_OK;
    case LES_FIELD_TAUW:
      out->bytes = 8LL * 4 * c.g.sxy;
      out->elem_bytes = 8;
      return LES_OK;
    case LES_FIELD_TAUWY:
      if (f.ybc != LES_YBC_WALL) return LES_EINVAL;
      out->bytes = 8LL * 4 * (f.nz + 2) * f.nx;
      out->elem_bytes = 8;
      return LES_OK;
    case LES_FIELD_ZGRID:
      out->bytes = 8LL * (2 * f.nz + 3);
      out->elem_bytes = 8;
      return LES_OK;
  }
  return LES_EINVAL;
}

les_status les_bind(les_ctx* ctx, int field, void* ptr) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  if (!ptr) return fail(&c, LES_EINVAL, "null pointer");
  if (((uintptr_t)ptr) & 255) return fail(&c, LES_EINVAL, "pointer must be 256-byte aligned");
  c.cfl_adv_ready = false;   // fields not written by the last correction
  switch (field) {
    case LES_FIELD_U: c.u = ptr; break;
    case LES_FIELD_V: c.v = ptr; break;
    case LES_FIELD_W: c.w = ptr; break;
    case LES_FIELD_P: c.p = ptr; break;
    case LES_FIELD_WORKSPACE: {
      c.ws = ptr;
      carve(c, (char*)ptr);
      GridP& g = c.g;
      g.zc = c.t.zc;
      g.dzf = c.t.dzf;
      g.dzc = c.t.dzc;
      g.delta2 = c.t.delta2;
      g.rdzf = c.t.rdzf;
      g.rdzc = c.t.rdzc;
      const les_config& f = c.cfg;
      const int n = f.nz;
      les_status s = check_hip(c, hipMemsetAsync(ptr, 0, c.ws_bytes, c.stream), "zero workspace");
      if (s != LES_OK) return s;
      auto up = [&](void* dst, const void* src, size_t bytes) {
        return check_hip(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.stream), "upload tables");
      };
      // host staging kept in the context so the asynchronous copies stay valid
      c.twx_f_host.clear();
      for (double x : c.twx) c.twx_f_host.push_back((float)x);
      c.twy_f_host.clear();
      for (double x : c.twy) c.twy_f_host.push_back((float)x);
      c.twz_f_host.clear();
      for (double x : c.twz) c.twz_f_host.push_back((float)x);
      c.twc_f_host.clear();
      for (double x : c.twc) c.twc_f_host.push_back((float)x);
      c.coef_host.assign(n + 2, 0.0);
      if (f.sgs == LES_SGS_MLP && c.mlp_params != nullptr) c.coef_host = c.delta2;
      if ((f.sgs == LES_SGS_DSM || f.sgs == LES_SGS_MLP) && f.ybc == LES_YBC_WALL)
        c.coef_host = c.delta2;   // field c_s(j, k) |S|
      if (f.sgs == LES_SGS_SMAG || f.sgs == LES_SGS_SMAG_VD)
        for (int k = 0; k <= n + 1; ++k) {
          const double d = std::pow((f.lx / f.nx) * (f.ly / f.ny) * c.dzf[k], 1.0 / 3.0);
          c.coef_host[k] = (f.cs * d) * (f.cs * d);
        }
      c.hfac_host.assign(14 * n, 0.0);
      for (int k = 0; k < n; ++k) c.hfac_host[4 * n + k] = 1.0;
      if ((s = up(c.t.zc, c.zc.data(), (n + 2) * 8)) != LES_OK) return s;
      if ((s = up(c.t.dzf, c.dzf.data(), (n + 2) * 8)) != LES_OK) return s;
      if ((s = up(c.t.dzc, c.dzc.data(), (n + 2) * 8)) != LES_OK) return s;
      if ((s = up(c.t.delta2, c.delta2.data(), (n + 2) * 8)) != LES_OK) return s;
      if ((s = up(c.t.rdzf, c.rdzf.data(), (n + 2) * 8)) != LES_OK) return s;
      if ((s = up(c.t.rdzc, c.rdzc.data(), (n + 2) * 8)) != LES_OK) return s;
      if ((s = up(c.t.coef, c.coef_host.data(), (n + 2) * 8)) != LES_OK) return s;
      if ((s = up(c.t.pa, c.pa.data(), n * 8)) != LES_OK) return s;
      if ((s = up(c.t.pb, c.pb.data(), n * 8)) != LES_OK) return s;
      if ((s = up(c.t.pc, c.pc.data(), n * 8)) != LES_OK) return s;
      if ((s = up(c.t.lamx, c.lamx.data(), c.lamx.size() * 8)) != LES_OK) return s;
      if ((s = up(c.t.lamy, c.lamy.data(), c.lamy.size() * 8)) != LES_OK) return s;
      if ((s = up(c.t.lamz, c.lamz.data(), c.lamz.size() * 8)) != LES_OK) return s;
      if ((s = up(c.t.twx, c.twx.data(), c.twx.size() * 8)) != LES_OK) return s;
      if ((s = up(c.t.twy, c.twy.data(), c.twy.size() * 8)) != LES_OK) return s;
      if ((s = up(c.t.twz, c.twz.data(), c.twz.size() * 8)) != LES_OK) return s;
      if ((s = up(c.t.twx_f, c.twx_f_host.data(), c.twx_f_host.size() * 4)) != LES_OK) return s;
      if ((s = up(c.t.twy_f, c.twy_f_host.data(), c.twy_f_host.size() * 4)) != LES_OK) return s;
      if ((s = up(c.t.twz_f, c.twz_f_host.data(), c.twz_f_host.size() * 4)) != LES_OK) return s;
      if ((s = up(c.t.twc, c.twc.data(), c.twc.size() * 8)) != LES_OK) return s;
      if ((s = up(c.t.twc_f, c.twc_f_host.data(), c.twc_f_host.size() * 4)) != LES_OK) return s;
      if ((s = up(c.t.hfac, c.hfac_host.data(), c.hfac_host.size() * 8)) != LES_OK) return s;
      // learned closure: fallback counters (cleared again by every evaluation)
      static const int cnt_init[4] = {0, 0, 0, 0};
      if ((s = up(c.mlp_cnt, cnt_init, sizeof(cnt_init))) != LES_OK) return s;
      if (f.zbc != LES_ZBC_PERIODIC) {
        launch_thomas_factor(c);
        if ((s = check_hip(c, hipGetLastError(), "thomas factorisation")) != LES_OK) return s;
      }
      c.initialised = false;
      if (c.graph_exec) {
        hipGraphExecDestroy(c.graph_exec);
        c.graph_exec = nullptr;
      }
      if (c.graph) {
        hipGraphDestroy(c.graph);
        c.graph = nullptr;
      }
      break;
    }
    default:
      return fail(&c, LES_EINVAL, "field is not bindable");
  }
  return LES_OK;
}

les_status les_nut(les_ctx* ctx) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  les_status s = ready(c, false);
  if (s != LES_OK) return s;
  c.cfl_adv_ready = false;   // called after the fields are written: the correction's maxima are stale
  if (c.cfg.precision == LES_MIXED) {
    launch_bc_fill<float>(c, (float*)c.u, (float*)c.v, (float*)c.w, (float*)c.p);
    if (c.g.ywall) launch_bc_fill_y<float>(c, (float*)c.u, (float*)c.v, (float*)c.w, (float*)c.p);
    boundary_and_model<float>(c);
  } else {
    launch_bc_fill<double>(c, (double*)c.u, (double*)c.v, (double*)c.w, (double*)c.p);
    if (c.g.ywall) launch_bc_fill_y<double>(c, (double*)c.u, (double*)c.v, (double*)c.w, (double*)c.p);
    boundary_and_model<double>(c);
  }
  s = check_launch(c, "les_nut");
  if (s == LES_OK) c.initialised = true;
  return s;
}

les_status les_dt(les_ctx* ctx, double cfl, double* dt_host) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  les_status s = ready(c, true);
  if (s != LES_OK) return s;
  if (!(std::isfinite(cfl) && cfl > 0.0)) return fail(&c, LES_EINVAL, "cfl must be positive");
  if (c.cfg.precision == LES_MIXED) launch_dt<float>(c, cfl);
  else launch_dt<double>(c, cfl);
  if ((s = check_launch(c, "les_dt")) != LES_OK) return s;
  if (dt_host) {
    if ((s = check_hip(c, hipMemcpyAsync(dt_host, c.t.dt, 8, hipMemcpyDeviceToHost, c.stream), "dt copy")) != LES_OK)
      return s;
    if ((s = check_hip(c, hipStreamSynchronize(c.stream), "dt sync")) != LES_OK) return s;
  }
  return LES_OK;
}

les_status les_set_dt(les_ctx* ctx, double dt) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  if (!c.ws) return fail(&c, LES_ESTATE, "workspace not bound");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(&c, LES_EINVAL, "dt must be positive");
  launch_set_dt(c, dt);
  return check_launch(c, "les_set_dt");
}

les_status les_substep(les_ctx* ctx, int stage) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  les_status s = ready(c, true);
  if (s != LES_OK) return s;
  if (stage < 0 || stage > 2) return fail(&c, LES_EINVAL, "stage must be 0, 1 or 2");
  return substep_any(c, stage);
}

les_status les_step(les_ctx* ctx, int use_graph) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  les_status s = ready(c, true);
  if (s != LES_OK) return s;
  if (!use_graph) {
    for (int k = 0; k < 3; ++k)
      if ((s = substep_any(c, k)) != LES_OK) return s;
    return LES_OK;
  }
  if (!c.stream) return fail(&c, LES_EINVAL, "graph replay needs a non-default stream");
  if (c.timing) return fail(&c, LES_ESTATE, "timing cannot be recorded into a graph");
  if (!c.graph_exec) {
    if ((s = check_hip(c, hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal), "begin capture")) != LES_OK)
      return s;
    les_status body = LES_OK;
    for (int k = 0; k < 3 && body == LES_OK; ++k) body = substep_any(c, k);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c.stream, &graph);
    if (body != LES_OK) {
      if (graph) hipGraphDestroy(graph);
      return body;
    }
    if ((s = check_hip(c, e, "end capture")) != LES_OK) return s;
    c.graph = graph;
    if ((s = check_hip(c, hipGraphInstantiate(&c.graph_exec, c.graph, nullptr, nullptr, 0), "instantiate")) != LES_OK)
      return s;
  }
  return check_hip(c, hipGraphLaunch(c.graph_exec, c.stream), "graph launch");
}

les_status les_poisson(les_ctx* ctx, void* f) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  if (!c.ws) return fail(&c, LES_ESTATE, "workspace not bound");
  if (!f) return fail(&c, LES_EINVAL, "null buffer");
  if (c.cfg.precision == LES_MIXED) launch_poisson_field<float>(c, (float*)f);
  else launch_poisson_field<double>(c, (double*)f);
  return check_launch(c, "les_poisson");
}

les_status les_project(les_ctx* ctx) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  les_status s = ready(c, false);
  if (s != LES_OK) return s;
  if (c.cfg.precision == LES_MIXED) launch_project<float>(c);
  else launch_project<double>(c);
  c.initialised = false;   // the eddy viscosity and ghosts of the new velocity come from les_nut
  c.cfl_adv_ready = false;
  return check_launch(c, "les_project");
}

les_status les_read(les_ctx* ctx, int field, void* dst) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  if (!dst) return fail(&c, LES_EINVAL, "null destination");
  const les_config& f = c.cfg;
  if (field == LES_FIELD_ZGRID) {
    std::memcpy(dst, c.zf.data(), (f.nz + 1) * 8);
    std::memcpy((double*)dst + f.nz + 1, c.zc.data(), (f.nz + 2) * 8);
    return LES_OK;
  }
  if (!c.ws) return fail(&c, LES_ESTATE, "workspace not bound");
  switch (field) {
    case LES_FIELD_NUT:
      if (f.precision == LES_MIXED) launch_read_nut<float>(c, (float*)dst);
      else launch_read_nut<double>(c, (double*)dst);
      return check_launch(c, "les_read");
    case LES_FIELD_CS:
      return check_hip(c, hipMemcpyAsync(dst, c.t.cs, 8 * (size_t)f.nz * (f.ybc == LES_YBC_WALL ? f.ny : 1),
                                         hipMemcpyDeviceToDevice, c.stream),
                       "read cs");
    case LES_FIELD_TAUW:
      return check_hip(c, hipMemcpyAsync(dst, c.t.tau, 8 * 4 * c.g.sxy, hipMemcpyDeviceToDevice, c.stream),
                       "read tau");
    case LES_FIELD_TAUWY:
      if (f.ybc != LES_YBC_WALL) return fail(&c, LES_EINVAL, "no y walls");
      return check_hip(c, hipMemcpyAsync(dst, c.t.tauy, 8 * 4 * (size_t)(f.nz + 2) * f.nx, hipMemcpyDeviceToDevice,
                                         c.stream),
                       "read tauy");
  }
  return fail(&c, LES_EINVAL, "field is not readable");
}

les_status les_stats_reset(les_ctx* ctx) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  if (!c.ws) return fail(&c, LES_ESTATE, "workspace not bound");
  launch_stats_reset(c);
  return check_launch(c, "les_stats_reset");
}

les_status les_stats_sample(les_ctx* ctx) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  les_status s = ready(c, false);
  if (s != LES_OK) return s;
  if (c.cfg.precision == LES_MIXED) launch_stats_sample<float>(c);
  else launch_stats_sample<double>(c);
  return check_launch(c, "les_stats_sample");
}

les_status les_stats_read(les_ctx* ctx, int32_t nbatch, les_stats_t* out, double* profiles) {
  if (!ctx || !out) return LES_EINVAL;
  Ctx& c = ctx->c;
  if (!c.ws) return fail(&c, LES_ESTATE, "workspace not bound");
  std::vector<double> host((size_t)stats_words(c.g));
  les_status s = check_hip(c, hipMemcpyAsync(host.data(), c.t.stats, host.size() * 8, hipMemcpyDeviceToHost, c.stream),
                           "read statistics");
  if (s != LES_OK) return s;
  s = check_hip(c, hipStreamSynchronize(c.stream), "read statistics");
  if (s != LES_OK) return s;
  stats_finalize(c, host.data(), nbatch, out, profiles);
  return LES_OK;
}

les_status les_diag(les_ctx* ctx, les_diag_t* out) {
  if (!ctx || !out) return LES_EINVAL;
  Ctx& c = ctx->c;
  les_status s = ready(c, false);
  if (s != LES_OK) return s;
  double* dev = c.t.red;
  if (c.cfg.precision == LES_MIXED) launch_diag<float>(c, dev);
  else launch_diag<double>(c, dev);
  if ((s = check_launch(c, "les_diag")) != LES_OK) return s;
  double h[8] = {0};
  double dt = 0.0;
  if ((s = check_hip(c, hipMemcpyAsync(h, dev, 6 * 8, hipMemcpyDeviceToHost, c.stream), "diag copy")) != LES_OK)
    return s;
  if ((s = check_hip(c, hipMemcpyAsync(&dt, c.t.dt, 8, hipMemcpyDeviceToHost, c.stream), "diag copy")) != LES_OK)
    return s;
  int cnt[2] = {0, 0};
  if ((s = check_hip(c, hipMemcpyAsync(cnt, c.mlp_cnt, sizeof(cnt), hipMemcpyDeviceToHost, c.stream), "diag copy")) !=
      LES_OK)
    return s;
  if ((s = check_hip(c, hipStreamSynchronize(c.stream), "diag sync")) != LES_OK) return s;
  std::memset(out, 0, sizeof(*out));
  out->max_div = h[0];
  const double cells_xy = (double)c.g.nx * c.g.ny;   // interior cells per plane
  out->ubulk = h[1] / (cells_xy * c.cfg.lz);
  out->max_vel = h[2];
  out->nonfinite = (int64_t)h[3];
  out->tauw_mean[0] = h[4] / cells_xy;
  out->tauw_mean[1] = h[5] / cells_xy;
  out->dt = dt;
  out->mlp_flagged = cnt[1];
  return out->nonfinite ? LES_ENONFINITE : LES_OK;
}

les_status les_mlp_bind(les_ctx* ctx, const float* params, const double* lo, const double* hi) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  if (c.cfg.sgs != LES_SGS_MLP) return fail(&c, LES_ESTATE, "context was not created with sgs = LES_SGS_MLP");
  if (!c.ws) return fail(&c, LES_ESTATE, "workspace not bound");
  if (!params || !lo || !hi) return fail(&c, LES_EINVAL, "null argument");
  for (int a = 0; a < 7; ++a)
    if (!(std::isfinite(lo[a]) && std::isfinite(hi[a]) && hi[a] > lo[a]))
      return fail(&c, LES_EINVAL, "feature ranges must satisfy lo < hi");
  c.mlp_params = const_cast<float*>(params);
  for (int a = 0; a < 7; ++a) {
    c.mlp_lo[a] = lo[a];
    c.mlp_hi[a] = hi[a];
  }
  // nu_t = Delta^2 * (c |S|) for the learned closure
  les_status s = check_hip(c, hipMemcpyAsync(c.t.coef, c.delta2.data(), (c.cfg.nz + 2) * 8, hipMemcpyHostToDevice,
                                             c.stream), "mlp coef");
  if (s != LES_OK) return s;
  static const int cnt_init[2] = {0, 0};
  s = check_hip(c, hipMemcpyAsync(c.mlp_cnt, cnt_init, sizeof(cnt_init), hipMemcpyHostToDevice, c.stream), "mlp cnt");
  if (s != LES_OK) return s;
  if (c.graph_exec) {
    hipGraphExecDestroy(c.graph_exec);
    c.graph_exec = nullptr;
  }
  if (c.graph) {
    hipGraphDestroy(c.graph);
    c.graph = nullptr;
  }
  return LES_OK;
}

les_status les_mlp_sample(les_ctx* ctx, uint64_t seed, int64_t n, float* x, float* y) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  les_status s = ready(c, true);
  if (s != LES_OK) return s;
  if (c.cfg.sgs != LES_SGS_DSM && c.cfg.sgs != LES_SGS_MLP)
    return fail(&c, LES_ESTATE, "sampling needs the dynamic-model coefficient (sgs = DSM)");
  if (n <= 0 || !x || !y) return fail(&c, LES_EINVAL, "bad sample buffers");
  if (c.cfg.precision == LES_MIXED) launch_mlp_sample<float>(c, seed, n, x, y);
  else launch_mlp_sample<double>(c, seed, n, x, y);
  return check_launch(c, "les_mlp_sample");
}

int64_t les_mlp_workspace_bytes(int64_t n) {
  if (n <= 0) return 0;
  return mlp_grad_blocks(n) * (int64_t)(4737 + 1) * 4;
}

static les_status mlp_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LES_OK : LES_EDEVICE;
}

les_status les_mlp_forward(void* stream, const float* params, const float* x, int64_t n, float* y) {
  if (!params || !x || !y || n <= 0) return LES_EINVAL;
  launch_mlp_forward((hipStream_t)stream, params, x, n, y);
  return mlp_status();
}

les_status les_mlp_normalize(void* stream, const float* x_raw, int64_t n, const double* lo, const double* hi,
                             float* x) {
  if (!x_raw || !x || !lo || !hi || n <= 0) return LES_EINVAL;
  for (int a = 0; a < 7; ++a)
    if (!(std::isfinite(lo[a]) && std::isfinite(hi[a]) && hi[a] > lo[a])) return LES_EINVAL;
  launch_mlp_normalize((hipStream_t)stream, x_raw, n, lo, hi, x);
  return mlp_status();
}

les_status les_mlp_grad(void* stream, const float* params, const float* x, const float* y, int64_t n, void* ws,
                        float* grad, float* loss) {
  if (!params || !x || !y || !ws || !grad || n <= 0) return LES_EINVAL;
  launch_mlp_grad((hipStream_t)stream, params, x, y, n, (float*)ws, grad, loss);
  return mlp_status();
}

les_status les_mlp_grad_noalloc(void* stream, const float* params, const float* x, const float* y, int64_t n,
                                float* grad, float* loss) {
  if (!params || !x || !y || !grad || n <= 0) {
    t_free_err = "les_mlp_grad_noalloc: null pointer or n <= 0";
    return LES_EINVAL;
  }
  if (n > LES_MLP_NOALLOC_MAX_SAMPLES) {
    t_free_err = "les_mlp_grad_noalloc: n = " + std::to_string(n) + " exceeds LES_MLP_NOALLOC_MAX_SAMPLES = " +
                 std::to_string(LES_MLP_NOALLOC_MAX_SAMPLES) + "; use les_mlp_grad with a workspace";
    return LES_EINVAL;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    t_free_err = "les_mlp_grad_noalloc: no current device";
    return LES_EDEVICE;
  }
  if (stream != nullptr) {
    hipDevice_t sdev = -1;
    if (hipStreamGetDevice((hipStream_t)stream, &sdev) != hipSuccess) {
      t_free_err = "les_mlp_grad_noalloc: cannot query the stream's device";
      return LES_EDEVICE;
    }
    if (sdev != dev) {
      t_free_err = "les_mlp_grad_noalloc: the stream belongs to device " + std::to_string(sdev) + " but device " +
                   std::to_string(dev) + " is current";
      return LES_EINVAL;
    }
  }
  float* part = nullptr;
  const hipError_t e = mlp_scratch_ptr(dev, &part);
  if (e != hipSuccess) {
    t_free_err = std::string("les_mlp_grad_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e);
    return LES_EDEVICE;
  }
  launch_mlp_grad((hipStream_t)stream, params, x, y, n, part, grad, loss);
  return mlp_status();
}

les_status les_mlp_adam(void* stream, float* params, const float* grad, float* m, float* v, int step, float lr) {
  if (!params || !grad || !m || !v || step < 1 || !(lr > 0.0f)) return LES_EINVAL;
  launch_mlp_adam((hipStream_t)stream, params, grad, m, v, step, lr);
  return mlp_status();
}

les_status les_mlp_train_step(void* stream, float* params, const float* x, const float* y, int64_t n, void* ws,
                              float* grad, float* m, float* v, int step, float lr, float* loss) {
  les_status s = les_mlp_grad(stream, params, x, y, n, ws, grad, loss);
  if (s != LES_OK) return s;
  return les_mlp_adam(stream, params, grad, m, v, step, lr);
}

static void clear_timing(Ctx& c) {
  for (auto& t : c.timed) {
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  c.timed.clear();
}

les_status les_timing(les_ctx* ctx, int enable) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  if (enable && !c.timing) clear_timing(c);
  c.timing = enable != 0;
  return LES_OK;
}

les_status les_timing_report(les_ctx* ctx, char* buf, size_t len) {
  if (!ctx || !buf || len == 0) return LES_EINVAL;
  Ctx& c = ctx->c;
  les_status s = check_hip(c, hipStreamSynchronize(c.stream), "timing sync");
  if (s != LES_OK) return s;
  struct Acc {
    std::string name;
    long count;
    double ms, bytes;
  };
  std::vector<Acc> acc;
  for (auto& t : c.timed) {
    float ms = 0.f;
    if ((s = check_hip(c, hipEventElapsedTime(&ms, t.a, t.b), "event time")) != LES_OK) return s;
    auto it = std::find_if(acc.begin(), acc.end(), [&](const Acc& a) { return a.name == t.name; });
    if (it == acc.end()) {
      acc.push_back({t.name, 0, 0.0, 0.0});
      it = acc.end() - 1;
    }
    it->count += 1;
    it->ms += ms;
    it->bytes += t.bytes;
  }
  std::string out = "{";
  for (size_t i = 0; i < acc.size(); ++i) {
    char tmp[256];
    std::snprintf(tmp, sizeof(tmp), "%s\"%s\": {\"count\": %ld, \"ms\": %.6f, \"bytes\": %.0f}", i ? ", " : "",
                  acc[i].name.c_str(), acc[i].count, acc[i].ms, acc[i].bytes);
    out += tmp;
  }
  out += "}";
  clear_timing(c);
  if (out.size() + 1 > len) return fail(&c, LES_ENOMEM, "timing report buffer too small");
  std::memcpy(buf, out.c_str(), out.size() + 1);
  return LES_OK;
}

les_status les_free(les_ctx* ctx) {
  if (!ctx) return LES_EINVAL;
  Ctx& c = ctx->c;
  clear_timing(c);
  if (c.graph_exec) hipGraphExecDestroy(c.graph_exec);
  if (c.graph) hipGraphDestroy(c.graph);
  delete ctx;
  return LES_OK;
}

}  // extern "C"
