// Long-run statistics of a channel run (Secs. 4.2 and 4.3 channel cases): per-sample plane sums of
// the mean-velocity and resolved-stress quantities accumulated on the device, the per-sample
// plane-mean wall stress kept as a series, and the host finalisation into profiles,
// tau_w, u_tau, Re_tau, C_f with its batch-means uncertainty and the profile error of
// Eq. error.  Discrete forms: every product is taken where its staggered factors meet (u v on
// the (x, y) edge, u w on the (x, z) edge, v w on the (y, z) edge, each factor the two-point
// mean onto that edge); covariances are the mean product minus the product of the means.
#include <cmath>
#include <vector>

#include "les_internal.h"

namespace les {

namespace {
constexpr int NQ = LES_STATS_NPROF;   // u, v, w, p, nu_t, uu, vv, ww, uv, uw, vw
}

int stats_blocks(int64_t sxy) {
  int64_t nb = sxy / 4096;
  return (int)(nb < 1 ? 1 : (nb > 64 ? 64 : nb));
}

// One block per (x-y chunk, plane): plane k < nz sums the NQ quantities of interior plane
// k + 1 (w and the products with w on its top face); row k = nz sums the streamwise wall
// stress at the bottom and top walls (wall model: its stress; no-slip: nu du/dz from the
// ghosts).  Per-block partials in a fixed order: wave shuffle trees, then the waves in order.
template <typename T>
__global__ void __launch_bounds__(256) k_stats_partial(GridP g, const T* __restrict__ u, const T* __restrict__ v,
                                                       const T* __restrict__ w, const T* __restrict__ p,
                                                       const T* __restrict__ nut, const double* __restrict__ coef,
                                                       const double* __restrict__ tau, double* __restrict__ part,
                                                       int nb) {
  __shared__ double wsum[4][NQ];
  const int k = blockIdx.y, b = blockIdx.x;
  const int64_t sxy = g.sxy;
  const int64_t chunk = (sxy + nb - 1) / nb;
  const int64_t r0 = b * chunk, r1 = r0 + chunk < sxy ? r0 + chunk : sxy;
  double acc[NQ];
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  if (k < g.nz) {
    const int kk = k + 1;
    const int64_t base = (int64_t)kk * sxy;
    const T cf = (T)coef[kk];
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      const int rr = (int)r;   // in-plane index (nx ny < 2^31)
      const int i = rr % g.nx, j = rr / g.nx;
      const int64_t c = base + r;
      const int64_t cip = base + (int64_t)j * g.nx + wrap_p(i, g.nx);
      const int64_t cjp = base + (int64_t)wrap_p(j, g.ny) * g.nx + i;
      const double uc = (double)u[c], vc = (double)v[c], wc = (double)w[c];
      const double ue_xy = 0.5 * (uc + (double)u[cjp]), ve_xy = 0.5 * (vc + (double)v[cip]);
      const double ue_xz = 0.5 * (uc + (double)u[c + sxy]), we_xz = 0.5 * (wc + (double)w[cip]);
      const double ve_yz = 0.5 * (vc + (double)v[c + sxy]), we_yz = 0.5 * (wc + (double)w[cjp]);
      acc[0] += uc;
      acc[1] += vc;
      acc[2] += wc;
      acc[3] += (double)p[c];
      acc[4] += (double)(cf * nut[c]);
      acc[5] += uc * uc;
      acc[6] += vc * vc;
      acc[7] += wc * wc;
      acc[8] += ue_xy * ve_xy;
      acc[9] += ue_xz * we_xz;
      acc[10] += ve_yz * we_yz;
    }
  } else if (g.zbc != LES_ZBC_PERIODIC) {
    const int n = g.nz;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      if (g.zbc == LES_ZBC_WALLMODEL) {
        acc[0] += tau[r];
        acc[1] += tau[2 * sxy + r];
      } else {
        acc[0] += g.nu * ((double)u[sxy + r] - (double)u[r]) / g.dzc[0];
        acc[1] += g.nu * ((double)u[(int64_t)n * sxy + r] - (double)u[(int64_t)(n + 1) * sxy + r]) / g.dzc[n];
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q = 0; q < NQ; ++q) {
    double s = acc[q];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) wsum[wv][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    const int q = threadIdx.x;
    part[((int64_t)q * (g.nz + 1) + k) * nb + b] = ((wsum[0][q] + wsum[1][q]) + wsum[2][q]) + wsum[3][q];
  }
}

// Adds the plane sums of one sample to the running sums and appends the sample's plane-mean
// wall stresses to the series.  One wave per (quantity, plane): lane b takes block b's
// partial (nb <= 64), a shuffle tree sums them in a fixed order; the wave after the last
// one does the wall-stress row and the header.  Layout of st: [0] samples, [1] sum of bottom
// stresses, [2] sum of top stresses, [3..7] unused, [8 .. 8 + NQ nz) sums [q][k], then the
// series [cap][2].
__global__ void __launch_bounds__(256) k_stats_final(GridP g, const double* __restrict__ part, int nb,
                                                     double* __restrict__ st, int cap) {
  const int n = g.nz;
  const int64_t wv = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wv > (int64_t)NQ * n) return;
  double* sums = st + 8;
  auto tree = [&](int64_t row) {
    double x = lane < nb ? part[row * nb + lane] : 0.0;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
  };
  if (wv < (int64_t)NQ * n) {
    const int q = (int)(wv / n), k = (int)(wv % n);
    const double s = tree((int64_t)q * (n + 1) + k);
    if (lane == 0) sums[(int64_t)q * n + k] += s;
    return;
  }
  const double tb = tree(n) / (double)g.sxy;               // quantity 0, row nz
  const double tt = tree((int64_t)(n + 1) + n) / (double)g.sxy;   // quantity 1, row nz
  if (lane == 0) {
    const int64_t idx = (int64_t)st[0];
    if (idx < cap) {
      double* ser = sums + (int64_t)NQ * n;
      ser[2 * idx] = tb;
      ser[2 * idx + 1] = tt;
    }
    st[0] += 1.0;
    st[1] += tb;
    st[2] += tt;
  }
}

// ---------------------------------------------------------------- square duct
// x is the only homogeneous direction: one wave per x line (k, j) sums the NQ quantities over
// i (lane i, i + 64, ...; shuffle tree) and adds them to the running sums [q][k][j] (each line
// owned by one wave: deterministic).  Edge neighbours as in the channel; row j + 1 of the last
// row is the stored ghost row (its product meets v = 0 on the wall face).
template <typename T>
__global__ void __launch_bounds__(256) k_stats_lines(GridP g, const T* __restrict__ u, const T* __restrict__ v,
                                                     const T* __restrict__ w, const T* __restrict__ p,
                                                     const T* __restrict__ nut, const double* __restrict__ coef,
                                                     double* __restrict__ sums) {
  const int64_t line = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (line >= (int64_t)g.nz * g.ny) return;
  const int k = (int)(line / g.ny), j = (int)(line % g.ny);
  const int kk = k + 1;
  const int64_t sxy = g.sxy;
  const T cf = (T)coef[kk];
  double acc[NQ];
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int i = lane; i < g.nx; i += 64) {
    const int64_t c = idx3(g, kk, j, i);
    const int64_t cip = idx3(g, kk, j, wrap_p(i, g.nx));
    const int64_t cjp = idx3(g, kk, j + 1, i);
    const double uc = (double)u[c], vc = (double)v[c], wc = (double)w[c];
    const double ue_xy = 0.5 * (uc + (double)u[cjp]), ve_xy = 0.5 * (vc + (double)v[cip]);
    const double ue_xz = 0.5 * (uc + (double)u[c + sxy]), we_xz = 0.5 * (wc + (double)w[cip]);
    const double ve_yz = 0.5 * (vc + (double)v[c + sxy]), we_yz = 0.5 * (wc + (double)w[cjp]);
    acc[0] += uc;
    acc[1] += vc;
    acc[2] += wc;
    acc[3] += (double)p[c];
    acc[4] += (double)(cf * nut[c]);
    acc[5] += uc * uc;
    acc[6] += vc * vc;
    acc[7] += wc * wc;
    acc[8] += ue_xy * ve_xy;
    acc[9] += ue_xz * we_xz;
    acc[10] += ve_yz * we_yz;
  }
  for (int q = 0; q < NQ; ++q) {
    double x = acc[q];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) sums[((int64_t)q * g.nz + k) * g.ny + j] += x;
  }
}

// Perimeter-mean streamwise wall stress of a duct sample: stage 1, DUCT_WALL_BLOCKS blocks of
// fixed-order partials (z bottom and top over (j, i); the y walls over (k, i) weighted by
// dzf_k); stage 2, one thread combines them in block order, weights each wall's mean by its
// length in the cross-section and appends the sample to the series (both slots).
constexpr int DUCT_WALL_BLOCKS = 64;

template <typename T>
__global__ void __launch_bounds__(256) k_stats_duct_wall(GridP g, const T* u, const double* tau, const double* tauy,
                                                         int wallmodel, double* part) {
  __shared__ double sm[4][256];
  double a[4] = {0, 0, 0, 0};
  const int n = g.nz, ny = g.ny, nx = g.nx;
  const int64_t s = g.sxy, sy = (int64_t)(n + 2) * nx;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t c = t0; c < (int64_t)nx * ny; c += stride) {
    if (wallmodel) {
      a[0] += tau[c];
      a[1] += tau[2 * s + c];
    } else {
      a[0] += g.nu * ((double)u[s + c] - (double)u[c]) / g.dzc[0];
      a[1] += g.nu * ((double)u[(int64_t)n * s + c] - (double)u[(int64_t)(n + 1) * s + c]) / g.dzc[n];
    }
  }
  for (int64_t e = t0; e < (int64_t)nx * n; e += stride) {
    const int k = (int)(e / nx) + 1, i = (int)(e % nx);
    const double dz = g.dzf[k];
    if (wallmodel) {
      const int64_t o = (int64_t)k * nx + i;
      a[2] += tauy[o] * dz;
      a[3] += tauy[2 * sy + o] * dz;
    } else {
      a[2] += g.nu * ((double)u[idx3(g, k, 0, i)] - (double)u[idx3(g, k, ny + 1, i)]) / g.dy * dz;
      a[3] += g.nu * ((double)u[idx3(g, k, ny - 1, i)] - (double)u[idx3(g, k, ny, i)]) / g.dy * dz;
    }
  }
  for (int q = 0; q < 4; ++q) sm[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int q = 0; q < 4; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ void k_stats_duct_final(GridP g, const double* part, double ly, double* st, int64_t series_off, int cap) {
  if (threadIdx.x != 0) return;
  double a[4] = {0, 0, 0, 0};
  for (int b = 0; b < DUCT_WALL_BLOCKS; ++b)
    for (int q = 0; q < 4; ++q) a[q] += part[b * 4 + q];
  const double nx = g.nx, ny = g.ny, lz = g.lz;
  const double zb = a[0] / (nx * ny), zt = a[1] / (nx * ny), yl = a[2] / (nx * lz), yh = a[3] / (nx * lz);
  const double t = (ly * (zb + zt) + lz * (yl + yh)) / (2.0 * (ly + lz));
  const int64_t idx = (int64_t)st[0];
  if (idx < cap) {
    st[series_off + 2 * idx] = t;
    st[series_off + 2 * idx + 1] = t;
  }
  st[0] += 1.0;
  st[1] += t;
  st[2] += t;
}

__global__ void k_fill_zero(double* a, int64_t n) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) a[e] = 0.0;
}

// profile lines per quantity: nz planes, or nz * ny x lines for ducts
static int64_t stats_lines(const GridP& g) { return (int64_t)g.nz * (g.ywall ? g.ny : 1); }
int64_t stats_words(const GridP& g) { return 8 + (int64_t)NQ * stats_lines(g) + 2 * (int64_t)LES_STATS_SERIES_MAX; }
int64_t stats_part_words(int nz, int64_t sxy) { return (int64_t)(nz + 1) * stats_blocks(sxy) * NQ; }

void launch_stats_reset(Ctx& c) {
  const int64_t n = 8 + (int64_t)NQ * stats_lines(c.g);   // the series is overwritten as samples arrive
  LES_LAUNCH(c, "stats_reset", 8.0 * n, k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.t.stats, n);
}

template <typename T>
void launch_stats_sample(Ctx& c) {
  if (c.g.ywall) {
    const int64_t lines = (int64_t)c.g.nz * c.g.ny;
    const double bytes = 5.0 * c.g.nx * lines * sizeof(T);
    LES_LAUNCH(c, "stats_partial", bytes, k_stats_lines<T>, dim3((unsigned)((lines + 3) / 4)), dim3(256), 0, c.g,
               (const T*)c.u, (const T*)c.v, (const T*)c.w, (const T*)c.p, (const T*)c.nut, c.t.coef, c.t.stats + 8);
    static_assert(DUCT_WALL_BLOCKS * 4 <= 4096, "partials fit the reduction area");
    LES_LAUNCH(c, "stats_wall", 0, k_stats_duct_wall<T>, dim3(DUCT_WALL_BLOCKS), dim3(256), 0, c.g, (const T*)c.u,
               c.t.tau, c.t.tauy, c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0, c.t.red);
    LES_LAUNCH(c, "stats_final", 0, k_stats_duct_final, dim3(1), dim3(64), 0, c.g, c.t.red, c.cfg.ly, c.t.stats,
               8 + (int64_t)NQ * lines, (int)LES_STATS_SERIES_MAX);
    return;
  }
  const int nb = stats_blocks(c.g.sxy);
  // algorithmic bytes: u, v, w, p and the eddy-viscosity field once per interior point
  const double bytes = 5.0 * c.g.sxy * c.g.nz * sizeof(T);
  LES_LAUNCH(c, "stats_partial", bytes, k_stats_partial<T>, dim3(nb, c.g.nz + 1), dim3(256), 0, c.g, (const T*)c.u,
             (const T*)c.v, (const T*)c.w, (const T*)c.p, (const T*)c.nut, c.t.coef, c.t.tau, c.t.stats_part, nb);
  const int64_t waves = (int64_t)NQ * c.g.nz + 1;
  LES_LAUNCH(c, "stats_final", 0, k_stats_final, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, c.g,
             c.t.stats_part, nb, c.t.stats, (int)LES_STATS_SERIES_MAX);
}
template void launch_stats_sample<double>(Ctx&);
template void launch_stats_sample<float>(Ctx&);

// Host finalisation of the copied statistics buffer (see k_stats_final for its layout).
static void stats_finalize_duct(const Ctx& c, const double* st, double* prof, double& ub);

void stats_finalize(const Ctx& c, const double* st, int nbatch, les_stats_t* out, double* prof) {
  const int n = c.cfg.nz;
  const double samples = st[0];
  const int64_t nl = stats_lines(c.g);
  const double N = samples * (double)c.cfg.nx * (double)c.cfg.ny;
  const double* sums = st + 8;
  std::vector<double> m(NQ * n, 0.0);
  for (int e = 0; e < NQ * n; ++e) m[e] = N > 0.0 ? sums[e] / N : 0.0;
  const double* U = m.data();
  const double* V = m.data() + n;
  const double* W = m.data() + 2 * n;
  const bool per = c.cfg.zbc == LES_ZBC_PERIODIC;
  double ub = 0.0;
  if (c.g.ywall) {
    stats_finalize_duct(c, st, prof, ub);
  } else if (prof) {
    for (int q = 0; q < 5; ++q)
      for (int k = 0; k < n; ++k) prof[q * n + k] = m[q * n + k];
    for (int k = 0; k < n; ++k) {
      // z-mean of u and v onto face k (cells k, k+1); the top face of a wall run has w = 0
      const int ku = k + 1 < n ? k + 1 : (per ? 0 : n - 1);
      prof[LES_STAT_UU * n + k] = m[5 * n + k] - U[k] * U[k];
      prof[LES_STAT_VV * n + k] = m[6 * n + k] - V[k] * V[k];
      prof[LES_STAT_WW * n + k] = m[7 * n + k] - W[k] * W[k];
      prof[LES_STAT_UV * n + k] = m[8 * n + k] - U[k] * V[k];
      prof[LES_STAT_UW * n + k] = m[9 * n + k] - 0.5 * (U[k] + U[ku]) * W[k];
      prof[LES_STAT_VW * n + k] = m[10 * n + k] - 0.5 * (V[k] + V[ku]) * W[k];
    }
  }
  if (!c.g.ywall) {
    double sud = 0.0, sd = 0.0;
    for (int k = 0; k < n; ++k) {
      sud += U[k] * c.dzf[k + 1];
      sd += c.dzf[k + 1];
    }
    ub = sud / sd;
  }
  const double tau_w = samples > 0.0 ? 0.5 * (st[1] + st[2]) / samples : 0.0;
  const double utau = std::sqrt(tau_w > 0.0 ? tau_w : 0.0);
  // batch means over the kept series (the oldest samples beyond nbatch * L dropped)
  const int64_t len = samples < LES_STATS_SERIES_MAX ? (int64_t)samples : (int64_t)LES_STATS_SERIES_MAX;
  double sigma = NAN;
  if (nbatch >= 2 && len >= nbatch) {
    const double* ser = sums + NQ * nl;
    const int64_t L = len / nbatch, s0 = len - (int64_t)nbatch * L;
    std::vector<double> bm(nbatch, 0.0);
    for (int b = 0; b < nbatch; ++b) {
      double s = 0.0;
      for (int64_t t = 0; t < L; ++t) {
        const int64_t i = s0 + (int64_t)b * L + t;
        s += 0.5 * (ser[2 * i] + ser[2 * i + 1]);
      }
      bm[b] = s / (double)L;
    }
    double mean = 0.0;
    for (double x : bm) mean += x;
    mean /= nbatch;
    double var = 0.0;
    for (double x : bm) var += (x - mean) * (x - mean);
    sigma = std::sqrt(var / (nbatch - 1)) / std::sqrt((double)nbatch);
  }
  out->samples = (int64_t)samples;
  out->series_len = len;
  out->tau_w = tau_w;
  out->u_tau = utau;
  out->re_tau = utau * 0.5 * c.cfg.lz / c.cfg.nu;
  out->u_b = ub;
  out->c_f = ub != 0.0 ? 2.0 * tau_w / (ub * ub) : NAN;
  out->c_f_sigma = ub != 0.0 ? 2.0 * sigma / (ub * ub) : NAN;
}

// Duct (x-line sums): cross-section means and covariances, prof[q][k][j]; the product of the
// means of two edge factors takes the two-point mean of the neighbouring lines' means (beyond
// the last row or plane the factor it multiplies is zero: v on the y wall face, w on the z
// wall face).  ub = the area mean of U.
static void stats_finalize_duct(const Ctx& c, const double* st, double* prof, double& ub) {
  const int n = c.cfg.nz, ny = c.cfg.ny;
  const int64_t nl = (int64_t)n * ny;
  const double N = st[0] * (double)c.cfg.nx;
  const double* sums = st + 8;
  auto M = [&](int q, int k, int j) { return N > 0.0 ? sums[(q * (int64_t)n + k) * ny + j] / N : 0.0; };
  double sud = 0.0, sd = 0.0;
  for (int k = 0; k < n; ++k) {
    double row = 0.0;
    for (int j = 0; j < ny; ++j) row += M(0, k, j);
    sud += row / ny * c.dzf[k + 1];
    sd += c.dzf[k + 1];
  }
  ub = sud / sd;
  if (!prof) return;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < ny; ++j) {
      const int jp = j + 1 < ny ? j + 1 : j, kp = k + 1 < n ? k + 1 : k;
      const double U = M(0, k, j), V = M(1, k, j), W = M(2, k, j);
      const int64_t o = (int64_t)k * ny + j;
      for (int q = 0; q < 5; ++q) prof[q * nl + o] = M(q, k, j);
      prof[LES_STAT_UU * nl + o] = M(5, k, j) - U * U;
      prof[LES_STAT_VV * nl + o] = M(6, k, j) - V * V;
      prof[LES_STAT_WW * nl + o] = M(7, k, j) - W * W;
      prof[LES_STAT_UV * nl + o] = M(8, k, j) - 0.5 * (U + M(0, k, jp)) * V;
      prof[LES_STAT_UW * nl + o] = M(9, k, j) - 0.5 * (U + M(0, kp, j)) * W;
      prof[LES_STAT_VW * nl + o] = M(10, k, j) - 0.5 * (V + M(1, kp, j)) * 0.5 * (W + M(2, k, jp));
    }
}

}  // namespace les

extern "C" les_status les_profile_error(const double* z, const double* phi, const double* ref, int32_t n, double z0,
                                        double z1, double* eps) {
  if (!z || !phi || !ref || !eps || n < 2 || !(z1 > z0)) return LES_EINVAL;
  for (int a = 0; a + 1 < n; ++a)
    if (!(z[a + 1] > z[a])) return LES_EINVAL;
  double num = 0.0, den = 0.0;
  for (int a = 0; a + 1 < n; ++a) {
    const double za = z[a], zb = z[a + 1];
    const double lo = za > z0 ? za : z0, hi = zb < z1 ? zb : z1;
    if (hi <= lo) continue;
    const double ta = (lo - za) / (zb - za), tb = (hi - za) / (zb - za);
    const double d0 = phi[a] - ref[a], d1 = phi[a + 1] - ref[a + 1];
    const double da = d0 + ta * (d1 - d0), db = d0 + tb * (d1 - d0);
    const double ra = ref[a] + ta * (ref[a + 1] - ref[a]), rb = ref[a] + tb * (ref[a + 1] - ref[a]);
    num += (hi - lo) * (da * da + da * db + db * db) / 3.0;
    den += (hi - lo) * 0.5 * (ra + rb);
  }
  if (den == 0.0) return LES_EINVAL;
  *eps = std::sqrt(num) / std::fabs(den);
  return LES_OK;
}
