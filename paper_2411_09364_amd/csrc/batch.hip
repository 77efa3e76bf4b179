// Batched ensembles of triply periodic boxes (declarations in include/les.h): every box is
// an ordinary context (own grid, tables and workspace slice), and each kernel of the
// substep runs for all boxes in one launch, the block -> box assignment given by per-kernel
// prefix sums of the boxes' block counts.  A step (per-box time step + three substeps) can
// be recorded once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "les_internal.h"

using namespace les;

struct les_batch {
  std::vector<les_ctx*> box;
  hipStream_t stream = nullptr;
  int nbox = 0;
  int prec = LES_FP64;
  int sgs = LES_SGS_NONE;
  std::vector<size_t> foff, woff;   // byte offsets of each box in the field / workspace buffers
  size_t ftotal = 0, wtotal = 0, desc_off = 0;
  void* fptr[4] = {nullptr, nullptr, nullptr, nullptr};
  void* ws = nullptr;
  std::vector<BoxDesc> hdesc;
  std::vector<int> hprefix;
  BoxDesc* ddesc = nullptr;
  int* dprefix = nullptr;
  int totals[BK_NKIND] = {0};
  size_t sh_x = 0, sh_y = 0, sh_z = 0;
  bool dirty = true;
  int tune_kc = 0;   // 0: per-box default; else planes per dynamic-model chunk
  int tune_l = 0;    // 0: default lines per FFT block; else this power of two
  double tune_cfl_graph = -1.0;   // cfl the recorded graph was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string err;
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

les_status bfail(les_batch* b, les_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}

void drop_graph(les_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

int pow2_at_most(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}

// Descriptors and prefix tables of the current tuning; uploaded into the workspace tail.
les_status prepare(les_batch* b) {
  if (!b->dirty) return LES_OK;
  for (int q = 0; q < 4; ++q)
    if (!b->fptr[q]) return bfail(b, LES_ESTATE, "batch fields not bound");
  if (!b->ws) return bfail(b, LES_ESTATE, "batch workspace not bound");
  const size_t E = b->prec == LES_MIXED ? 4 : 8;
  b->hdesc.assign(b->nbox, BoxDesc{});
  b->hprefix.assign((size_t)BK_NKIND * (b->nbox + 1), 0);
  b->sh_x = b->sh_y = b->sh_z = 0;
  for (int i = 0; i < b->nbox; ++i) {
    Ctx& c = b->box[i]->c;
    BoxDesc& d = b->hdesc[i];
    d.g = c.g;
    d.u = c.u;
    d.v = c.v;
    d.w = c.w;
    d.p = c.p;
    d.ru = c.ru;
    d.rv = c.rv;
    d.rw = c.rw;
    d.us = c.us;
    d.vs = c.vs;
    d.wsf = c.wsf;
    d.nut = c.nut;
    d.phi = c.phi;
    d.spec = c.spec;
    d.coef = c.t.coef;
    d.cs = c.t.cs;
    d.dt = c.t.dt;
    d.red = c.t.red;
    d.dsm_part = c.t.dsm_part;
    d.lamx = c.t.lamx;
    d.lamy = c.t.lamy;
    d.lamz = c.t.lamz;
    d.twx = c.t.twx;
    d.twy = c.t.twy;
    d.twz = c.t.twz;
    d.twx_f = c.t.twx_f;
    d.twy_f = c.t.twy_f;
    d.twz_f = c.t.twz_f;
    const int nx = c.g.nx, ny = c.g.ny, nz = c.g.nz, nxh = nx / 2 + 1;
    d.px = make_plan(nx);
    d.py = make_plan(ny);
    d.pz = make_plan(nz);
    d.pbx = fft_pairs_per_block(nx);
    d.ly = b->tune_l ? std::min(b->tune_l, pow2_at_most(std::max(1, 2048 / ny))) : fft_lines_per_block(ny);
    d.lz = b->tune_l ? std::min(b->tune_l, pow2_at_most(std::max(1, 2048 / nz))) : fft_lines_per_block(nz);
    d.kc = b->tune_kc ? std::min(b->tune_kc, nz) : c.dsm_kc;
    d.pkc = c.pred_kc;
    d.sgs = c.cfg.sgs;
    auto set = [&](int kind, int x, int y, int z) {
      d.gdim[kind][0] = x;
      d.gdim[kind][1] = y;
      d.gdim[kind][2] = z;
    };
    set(BK_POINT, (nx + 31) / 32, (ny + 7) / 8, nz);
    set(BK_RFFTX, (int)(((int64_t)nz * (ny / 2) + d.pbx - 1) / d.pbx), 1, 1);
    set(BK_FFTY, (nxh + d.ly - 1) / d.ly, nz, 1);
    set(BK_FFTZ, (nxh + d.lz - 1) / d.lz, ny, 1);
    const int dty = dsm_tile_rows(b->prec != LES_MIXED);
    set(BK_DSM, (nx + 31) / 32, (ny + dty - 1) / dty, (nz + d.kc - 1) / d.kc);
    set(BK_DSMRED, nz, 1, 1);
    set(BK_CFL, 64, 1, 1);
    set(BK_PRED, (nx + 31) / 32, (ny + 7) / 8, (nz + d.pkc - 1) / d.pkc);
    b->sh_x = std::max(b->sh_x, 2 * (size_t)d.pbx * nx * 2 * E);
    b->sh_y = std::max(b->sh_y, 2 * (size_t)d.ly * (ny + 1) * 2 * E);
    b->sh_z = std::max(b->sh_z, 2 * (size_t)d.lz * (nz + 1) * 2 * E);
  }
  for (int k = 0; k < BK_NKIND; ++k) {
    int* pre = &b->hprefix[(size_t)k * (b->nbox + 1)];
    pre[0] = 0;
    for (int i = 0; i < b->nbox; ++i) {
      const int* gd = b->hdesc[i].gdim[k];
      pre[i + 1] = pre[i] + gd[0] * gd[1] * gd[2];
    }
    b->totals[k] = pre[b->nbox];
  }
  char* tail = (char*)b->ws + b->desc_off;
  b->ddesc = (BoxDesc*)tail;
  b->dprefix = (int*)(tail + al256(sizeof(BoxDesc) * b->nbox));
  hipError_t e = hipMemcpyAsync(b->ddesc, b->hdesc.data(), sizeof(BoxDesc) * b->nbox, hipMemcpyHostToDevice,
                                b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->dprefix, b->hprefix.data(), sizeof(int) * b->hprefix.size(), hipMemcpyHostToDevice,
                       b->stream);
  if (e != hipSuccess) return bfail(b, LES_EDEVICE, std::string("descriptor upload: ") + hipGetErrorString(e));
  b->dirty = false;
  drop_graph(b);
  return LES_OK;
}

BatchMap map_of(const les_batch* b) { return BatchMap{b->ddesc, b->dprefix, b->nbox}; }

template <typename T>
void substep_batch(les_batch* b, int stage) {
  const BatchMap m = map_of(b);
  batch_predictor<T>(b->stream, m, b->totals[BK_PRED], stage);
  batch_poisson<T>(b->stream, m, b->totals, b->sh_x, b->sh_y, b->sh_z, stage);
  batch_correct<T>(b->stream, m, b->totals[BK_POINT], stage);
  batch_eddy_viscosity<T>(b->stream, m, b->totals, b->sgs == LES_SGS_DSM, b->sgs == LES_SGS_SMAG);
}

les_status run_substep(les_batch* b, int stage) {
  if (b->prec == LES_MIXED) substep_batch<float>(b, stage);
  else substep_batch<double>(b, stage);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LES_OK : bfail(b, LES_EDEVICE, std::string("batch substep: ") + hipGetErrorString(e));
}

les_status run_dt(les_batch* b, double cfl) {
  const BatchMap m = map_of(b);
  if (b->prec == LES_MIXED) batch_dt<float>(b->stream, m, b->totals[BK_CFL], b->nbox, cfl);
  else batch_dt<double>(b->stream, m, b->totals[BK_CFL], b->nbox, cfl);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LES_OK : bfail(b, LES_EDEVICE, std::string("batch dt: ") + hipGetErrorString(e));
}

}  // namespace

extern "C" {

les_status les_batch_init(const les_config* cfgs, int nbox, void* hip_stream, les_batch** out) {
  if (!out) return LES_EINVAL;
  *out = nullptr;
  if (!cfgs || nbox < 1 || nbox > kMaxBox) return LES_EINVAL;
  for (int i = 0; i < nbox; ++i) {
    const les_config& f = cfgs[i];
    if (f.zbc != LES_ZBC_PERIODIC || f.implicit_z || f.ubulk != 0.0) return LES_ENOTSUP;
    if (f.sgs != LES_SGS_NONE && f.sgs != LES_SGS_SMAG && f.sgs != LES_SGS_DSM) return LES_ENOTSUP;
    if (f.sgs != cfgs[0].sgs || f.precision != cfgs[0].precision) return LES_EINVAL;
  }
  les_batch* b = new (std::nothrow) les_batch();
  if (!b) return LES_ENOMEM;
  b->stream = (hipStream_t)hip_stream;
  b->nbox = nbox;
  b->prec = cfgs[0].precision;
  b->sgs = cfgs[0].sgs;
  for (int i = 0; i < nbox; ++i) {
    les_ctx* c = nullptr;
    const les_status s = les_init(&cfgs[i], hip_stream, &c);
    if (s != LES_OK) {
      for (auto* x : b->box) les_free(x);
      delete b;
      return s;
    }
    b->box.push_back(c);
  }
  size_t fo = 0, wo = 0;
  for (int i = 0; i < nbox; ++i) {
    les_layout_t lf, lw;
    les_layout(b->box[i], LES_FIELD_U, &lf);
    les_layout(b->box[i], LES_FIELD_WORKSPACE, &lw);
    b->foff.push_back(fo);
    b->woff.push_back(wo);
    fo = al256(fo + (size_t)lf.bytes);
    wo = al256(wo + (size_t)lw.bytes);
  }
  b->ftotal = fo;
  b->desc_off = wo;
  b->wtotal = wo + al256(sizeof(BoxDesc) * nbox) + al256(sizeof(int) * BK_NKIND * (nbox + 1));
  *out = b;
  return LES_OK;
}

les_status les_batch_layout(const les_batch* b, int field, les_layout_t* out) {
  if (!b || !out) return LES_EINVAL;
  std::memset(out, 0, sizeof(*out));
  switch (field) {
    case LES_FIELD_U: case LES_FIELD_V: case LES_FIELD_W: case LES_FIELD_P:
      out->bytes = (int64_t)b->ftotal;
      out->elem_bytes = b->prec == LES_MIXED ? 4 : 8;
      return LES_OK;
    case LES_FIELD_WORKSPACE:
      out->bytes = (int64_t)b->wtotal;
      out->elem_bytes = 1;
      return LES_OK;
  }
  return LES_EINVAL;
}

les_status les_batch_offset(const les_batch* b, int box, int field, int64_t* byte_offset) {
  if (!b || !byte_offset || box < 0 || box >= b->nbox) return LES_EINVAL;
  if (field >= LES_FIELD_U && field <= LES_FIELD_P) {
    *byte_offset = (int64_t)b->foff[box];
    return LES_OK;
  }
  if (field == LES_FIELD_WORKSPACE) {
    *byte_offset = (int64_t)b->woff[box];
    return LES_OK;
  }
  return LES_EINVAL;
}

les_status les_batch_bind(les_batch* b, int field, void* ptr) {
  if (!b || !ptr) return LES_EINVAL;
  if (((uintptr_t)ptr) & 255) return bfail(b, LES_EINVAL, "pointer must be 256-byte aligned");
  if (field >= LES_FIELD_U && field <= LES_FIELD_P) {
    for (int i = 0; i < b->nbox; ++i) {
      const les_status s = les_bind(b->box[i], field, (char*)ptr + b->foff[i]);
      if (s != LES_OK) return bfail(b, s, les_last_error(b->box[i]));
    }
    b->fptr[field] = ptr;
  } else if (field == LES_FIELD_WORKSPACE) {
    for (int i = 0; i < b->nbox; ++i) {
      const les_status s = les_bind(b->box[i], field, (char*)ptr + b->woff[i]);
      if (s != LES_OK) return bfail(b, s, les_last_error(b->box[i]));
    }
    b->ws = ptr;
  } else {
    return bfail(b, LES_EINVAL, "field is not bindable");
  }
  b->dirty = true;
  return LES_OK;
}

les_status les_batch_nut(les_batch* b) {
  if (!b) return LES_EINVAL;
  les_status s = prepare(b);
  if (s != LES_OK) return s;
  for (int i = 0; i < b->nbox; ++i)
    if ((s = les_nut(b->box[i])) != LES_OK) return bfail(b, s, les_last_error(b->box[i]));
  return LES_OK;
}

les_status les_batch_dt(les_batch* b, double cfl) {
  if (!b) return LES_EINVAL;
  if (!(std::isfinite(cfl) && cfl > 0.0)) return bfail(b, LES_EINVAL, "cfl must be positive");
  les_status s = prepare(b);
  if (s != LES_OK) return s;
  return run_dt(b, cfl);
}

les_status les_batch_set_dt(les_batch* b, double dt) {
  if (!b) return LES_EINVAL;
  if (!(std::isfinite(dt) && dt > 0.0)) return bfail(b, LES_EINVAL, "dt must be positive");
  les_status s = prepare(b);
  if (s != LES_OK) return s;
  batch_set_dt(b->stream, map_of(b), b->nbox, dt);
  return hipGetLastError() == hipSuccess ? LES_OK : bfail(b, LES_EDEVICE, "batch set dt");
}

les_status les_batch_substep(les_batch* b, int stage) {
  if (!b) return LES_EINVAL;
  if (stage < 0 || stage > 2) return bfail(b, LES_EINVAL, "stage must be 0, 1 or 2");
  les_status s = prepare(b);
  if (s != LES_OK) return s;
  return run_substep(b, stage);
}

les_status les_batch_step(les_batch* b, double cfl, int use_graph) {
  if (!b) return LES_EINVAL;
  if (!(std::isfinite(cfl) && cfl >= 0.0)) return bfail(b, LES_EINVAL, "cfl must be >= 0");
  les_status s = prepare(b);
  if (s != LES_OK) return s;
  auto body = [&]() -> les_status {
    les_status r = LES_OK;
    if (cfl > 0.0) r = run_dt(b, cfl);
    for (int k = 0; k < 3 && r == LES_OK; ++k) r = run_substep(b, k);
    return r;
  };
  if (!use_graph) return body();
  if (!b->stream) return bfail(b, LES_EINVAL, "graph replay needs a non-default stream");
  if (!b->exec) {
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(b, LES_EDEVICE, std::string("begin capture: ") + hipGetErrorString(e));
    const les_status r = body();
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->stream, &g);
    if (r != LES_OK) {
      if (g) hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return bfail(b, LES_EDEVICE, std::string("end capture: ") + hipGetErrorString(e));
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return bfail(b, LES_EDEVICE, std::string("instantiate: ") + hipGetErrorString(e));
    b->tune_cfl_graph = cfl;
  } else if (b->tune_cfl_graph != cfl) {
    return bfail(b, LES_EINVAL, "graph was recorded with another cfl");
  }
  const hipError_t e = hipGraphLaunch(b->exec, b->stream);
  return e == hipSuccess ? LES_OK : bfail(b, LES_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
}

les_status les_batch_autotune(les_batch* b, int substeps, char* report, size_t len) {
  if (!b || substeps < 1) return LES_EINVAL;
  const int kcs[] = {4, 8, 16, 32};
  const int ls[] = {4, 8, 16, 32};
  auto time_now = [&]() -> double {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, b->stream);
    for (int i = 0; i < substeps; ++i) run_substep(b, i % 3);
    (void)hipEventRecord(e1, b->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
  };
  std::string rep = "{\"kc\": {";
  double best = 1e300;
  int best_kc = 0;
  b->tune_l = 0;
  for (int q = 0; q < 4; ++q) {
    b->tune_kc = kcs[q];
    b->dirty = true;
    les_status s = prepare(b);
    if (s != LES_OK) return s;
    run_substep(b, 0);   // warm
    const double ms = time_now();
    char tmp[64];
    std::snprintf(tmp, sizeof(tmp), "%s\"%d\": %.4f", q ? ", " : "", kcs[q], ms / substeps);
    rep += tmp;
    if (ms < best) {
      best = ms;
      best_kc = kcs[q];
    }
  }
  b->tune_kc = best_kc;
  rep += "}, \"lines\": {";
  best = 1e300;
  int best_l = 0;
  for (int q = 0; q < 4; ++q) {
    b->tune_l = ls[q];
    b->dirty = true;
    les_status s = prepare(b);
    if (s != LES_OK) return s;
    run_substep(b, 0);
    const double ms = time_now();
    char tmp[64];
    std::snprintf(tmp, sizeof(tmp), "%s\"%d\": %.4f", q ? ", " : "", ls[q], ms / substeps);
    rep += tmp;
    if (ms < best) {
      best = ms;
      best_l = ls[q];
    }
  }
  b->tune_l = best_l;
  b->dirty = true;
  les_status s = prepare(b);
  if (s != LES_OK) return s;
  char tmp[96];
  std::snprintf(tmp, sizeof(tmp), "}, \"chosen\": {\"kc\": %d, \"lines\": %d}}", best_kc, best_l);
  rep += tmp;
  const hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, LES_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
  if (report && len) {
    if (rep.size() + 1 > len) return bfail(b, LES_ENOMEM, "report buffer too small");
    std::memcpy(report, rep.c_str(), rep.size() + 1);
  }
  return LES_OK;
}

les_status les_batch_read(les_batch* b, int box, int field, void* dst) {
  if (!b || box < 0 || box >= b->nbox) return LES_EINVAL;
  return les_read(b->box[box], field, dst);
}

les_status les_batch_mlp_sample(les_batch* b, uint64_t seed, int64_t n, float* x, float* y) {
  if (!b) return LES_EINVAL;
  if (n < 0) return bfail(b, LES_EINVAL, "n_per_box must be non-negative");
  if (n > 0 && (!x || !y)) return bfail(b, LES_EINVAL, "null buffer");
  les_status s = prepare(b);
  if (s != LES_OK) return s;
  // one launch per box on the batch stream: sampling is not on the timed path
  for (int i = 0; i < b->nbox && n > 0; ++i) {
    s = les_mlp_sample(b->box[i], seed + (uint64_t)i, n, x + (int64_t)i * n * 7, y + (int64_t)i * n);
    if (s != LES_OK) return bfail(b, s, les_last_error(b->box[i]));
  }
  return LES_OK;
}

les_status les_batch_diag(les_batch* b, int box, les_diag_t* out) {
  if (!b || box < 0 || box >= b->nbox) return LES_EINVAL;
  return les_diag(b->box[box], out);
}

const char* les_batch_last_error(const les_batch* b) { return b ? b->err.c_str() : "null batch"; }

les_status les_batch_free(les_batch* b) {
  if (!b) return LES_EINVAL;
  drop_graph(b);
  for (auto* c : b->box) les_free(c);
  delete b;
  return LES_OK;
}

}  // extern "C"
