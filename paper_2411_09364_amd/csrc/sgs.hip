// Eddy viscosity (Sec. 2.1, Eqs. smag, dsmag, cs, lij, mij; Sec. 2.2 SGS paragraph).
//
// Every Smagorinsky variant is stored as nu_t = coef[k] * S(k, j, i) where S = |S| at the
// cell centre and coef a per-plane factor:
//   static         coef = (C_s Delta_k)^2
//   van Driest     coef = (C_s Delta_k D_k)^2, D_k = 1 - exp(-y*/25) from the plane-mean
//                  wall stress of the nearer wall
//   dynamic        coef = c_s(k) Delta_k^2 with c_s from the plane-averaged Germano-Lilly
//                  identity (clipped at zero)
// so the predictor reads one field plus an nz-long vector.
//
// Strain ghosts: with the wall model, wall-parallel velocity ghosts for the strain are the
// linear extrapolation in z of the first two interior values (one-sided wall-normal
// derivative in the first layer, Sec. 2.2); otherwise the stored ghosts are used.
#include "les_internal.h"

namespace les {

template <typename T>
struct VelView {
  const T* u;
  const T* v;
  const T* w;
};

// u or v at (k, j, i) with the strain ghost rule.
template <typename T>
__device__ inline T sval(const GridP& g, const T* f, int k, int j, int i) {
  if (g.zbc == LES_ZBC_WALLMODEL) {
    if (k == 0) {
      const T a1 = f[idx3(g, 1, j, i)], a2 = f[idx3(g, 2, j, i)];
      return a1 - (T)g.dzc[0] * ((a2 - a1) / (T)g.dzc[1]);
    }
    if (k == g.nz + 1) {
      const int n = g.nz;
      const T a1 = f[idx3(g, n, j, i)], a0 = f[idx3(g, n - 1, j, i)];
      return a1 + (T)g.dzc[n] * ((a1 - a0) / (T)g.dzc[n - 1]);
    }
  }
  return f[idx3(g, k, j, i)];
}

// Strain rate at the centre of cell (k, j, i): s[0..5] = S11 S22 S33 S12 S13 S23.
template <typename T>
__device__ inline void centre_strain(const GridP& g, const T* u, const T* v, const T* w, int k, int j, int i, T s[6]) {
  const int ip = wrap_p(i, g.nx), im = wrap_m(i, g.nx), jp = wrap_p(j, g.ny), jm = wrap_m(j, g.ny);
  const T rdx = (T)g.rdx, rdy = (T)g.rdy, h = (T)0.5, q = (T)0.25;
  const T rdzc = (T)(1.0 / g.dzc[k]), rdzcm = (T)(1.0 / g.dzc[k - 1]);
#define US(kk, jj, ii) sval(g, u, kk, jj, ii)
#define VS(kk, jj, ii) sval(g, v, kk, jj, ii)
#define W(kk, jj, ii) w[idx3(g, kk, jj, ii)]
  const T u0 = US(k, j, i), uim = US(k, j, im), ujp = US(k, jp, i), ujm = US(k, jm, i);
  const T ujp_im = US(k, jp, im), ujm_im = US(k, jm, im);
  const T v0 = VS(k, j, i), vjm = VS(k, jm, i), vip = VS(k, j, ip), vim = VS(k, j, im);
  const T vjm_ip = VS(k, jm, ip), vjm_im = VS(k, jm, im);
  s[0] = (u0 - uim) * rdx;
  s[1] = (v0 - vjm) * rdy;
  s[2] = (W(k, j, i) - W(k - 1, j, i)) * (T)(1.0 / g.dzf[k]);
  const T e_a = h * ((ujp - u0) * rdy + (vip - v0) * rdx);           // (j, i)
  const T e_b = h * ((ujp_im - uim) * rdy + (v0 - vim) * rdx);       // (j, i-1)
  const T e_c = h * ((u0 - ujm) * rdy + (vjm_ip - vjm) * rdx);       // (j-1, i)
  const T e_d = h * ((uim - ujm_im) * rdy + (vjm - vjm_im) * rdx);   // (j-1, i-1)
  s[3] = q * (e_a + e_b + e_c + e_d);
  const T ukp = US(k + 1, j, i), ukm = US(k - 1, j, i), ukp_im = US(k + 1, j, im), ukm_im = US(k - 1, j, im);
  const T f_a = h * ((ukp - u0) * rdzc + (W(k, j, ip) - W(k, j, i)) * rdx);
  const T f_b = h * ((ukp_im - uim) * rdzc + (W(k, j, i) - W(k, j, im)) * rdx);
  const T f_c = h * ((u0 - ukm) * rdzcm + (W(k - 1, j, ip) - W(k - 1, j, i)) * rdx);
  const T f_d = h * ((uim - ukm_im) * rdzcm + (W(k - 1, j, i) - W(k - 1, j, im)) * rdx);
  s[4] = q * (f_a + f_b + f_c + f_d);
  const T vkp = VS(k + 1, j, i), vkm = VS(k - 1, j, i), vkp_jm = VS(k + 1, jm, i), vkm_jm = VS(k - 1, jm, i);
  const T g_a = h * ((vkp - v0) * rdzc + (W(k, jp, i) - W(k, j, i)) * rdy);
  const T g_b = h * ((vkp_jm - vjm) * rdzc + (W(k, j, i) - W(k, jm, i)) * rdy);
  const T g_c = h * ((v0 - vkm) * rdzcm + (W(k - 1, jp, i) - W(k - 1, j, i)) * rdy);
  const T g_d = h * ((vjm - vkm_jm) * rdzcm + (W(k - 1, j, i) - W(k - 1, jm, i)) * rdy);
  s[5] = q * (g_a + g_b + g_c + g_d);
#undef US
#undef VS
#undef W
}

template <typename T>
__device__ inline T strain_mag(const T s[6]) {
  return sqrt((T)2 * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]) + (T)4 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
}

// Writes a cell-centred value and, on the first/last plane, the ghost plane of the
// eddy-viscosity field (odd about walls, R12; periodic copy otherwise).
template <typename T>
__device__ inline void store_nut(const GridP& g, T* nut, int k, int j, int i, T val) {
  nut[idx3(g, k, j, i)] = val;
  const int n = g.nz;
  if (g.zbc == LES_ZBC_PERIODIC) {
    if (k == n) nut[idx3(g, 0, j, i)] = val;
    if (k == 1) nut[idx3(g, n + 1, j, i)] = val;
  } else {
    if (k == 1) nut[idx3(g, 0, j, i)] = -val;
    if (k == n) nut[idx3(g, n + 1, j, i)] = -val;
  }
}

// ============================================================================ |S|
template <typename T>
__global__ void __launch_bounds__(256) k_strain_mag(GridP g, const T* __restrict__ u, const T* __restrict__ v,
                                                    const T* __restrict__ w, T* __restrict__ nut) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z + 1;
  if (i >= g.nx || j >= g.ny) return;
  T s[6];
  centre_strain(g, u, v, w, k, j, i, s);
  store_nut(g, nut, k, j, i, strain_mag(s));
}

// van Driest coefficient: plane-mean wall stresses -> u_tau per wall -> coef[k].
// tau = wall-model stresses, or (no-slip) nu (u_1 - u_0)/dzc_0 from the ghosts.
template <typename T>
__global__ void k_vd_coef(GridP g, const T* u, const T* v, const double* tau, int wallmodel, double cs,
                          double* coef) {
  __shared__ double sm[4][256];
  double a[4] = {0, 0, 0, 0};
  const int64_t s = g.sxy;
  const int n = g.nz;
  for (int64_t c = threadIdx.x; c < s; c += blockDim.x) {
    if (wallmodel) {
      for (int q = 0; q < 4; ++q) a[q] += tau[q * s + c];
    } else {
      a[0] += g.nu * ((double)u[s + c] - (double)u[c]) / g.dzc[0];
      a[1] += g.nu * ((double)v[s + c] - (double)v[c]) / g.dzc[0];
      a[2] += g.nu * ((double)u[(int64_t)n * s + c] - (double)u[(int64_t)(n + 1) * s + c]) / g.dzc[n];
      a[3] += g.nu * ((double)v[(int64_t)n * s + c] - (double)v[(int64_t)(n + 1) * s + c]) / g.dzc[n];
    }
  }
  for (int q = 0; q < 4; ++q) sm[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int q = 0; q < 4; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ub = sqrt(hypot(sm[0][0] / s, sm[1][0] / s));
    const double ut = sqrt(hypot(sm[2][0] / s, sm[3][0] / s));
    for (int k = 1; k <= n; ++k) {
      const double zc = g.zc[k];
      const bool lower = zc <= 0.5 * g.lz;
      const double d = lower ? zc : g.lz - zc;
      const double utk = lower ? ub : ut;
      const double damp = 1.0 - exp(-d * utk / g.nu / 25.0);
      const double f = cs * sqrt(g.delta2[k]) * damp;
      coef[k] = f * f;
    }
    coef[0] = coef[1];
    coef[n + 1] = coef[n];
  }
}

// ============================================================================ dynamic model
// Sweep 1: centre velocities and |S| S_ij (9 fields), |S| into the eddy-viscosity field.
template <typename T>
__global__ void __launch_bounds__(256) k_dsm_centre(GridP g, const T* __restrict__ u, const T* __restrict__ v,
                                                    const T* __restrict__ w, T* __restrict__ nut, T* __restrict__ q9,
                                                    int64_t fstride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z + 1;
  if (i >= g.nx || j >= g.ny) return;
  T s[6];
  centre_strain(g, u, v, w, k, j, i, s);
  const T sm = strain_mag(s);
  store_nut(g, nut, k, j, i, sm);
  const int64_t c = idx3(g, k, j, i);
  const T h = (T)0.5;
  q9[c] = h * (u[c] + u[idx3(g, k, j, wrap_m(i, g.nx))]);
  q9[fstride + c] = h * (v[c] + v[idx3(g, k, wrap_m(j, g.ny), i)]);
  q9[2 * fstride + c] = h * (w[c] + w[c - g.sxy]);
  for (int a = 0; a < 6; ++a) q9[(3 + a) * fstride + c] = sm * s[a];
}

// x-y trapezoidal filter (1/4, 1/2, 1/4)^2 of field f at plane kk around (j, i).
template <typename T>
__device__ inline T filt_xy(const GridP& g, const T* f, int kk, int j, int i) {
  const int ip = wrap_p(i, g.nx), im = wrap_m(i, g.nx), jp = wrap_p(j, g.ny), jm = wrap_m(j, g.ny);
  const T a = (T)0.25, b = (T)0.5;
  auto row = [&](int jj) {
    return a * f[idx3(g, kk, jj, im)] + b * f[idx3(g, kk, jj, i)] + a * f[idx3(g, kk, jj, ip)];
  };
  return a * row(jm) + b * row(j) + a * row(jp);
}

// z-neighbour plane indices of a z-centred quantity (periodic wrap) or -1 for the
// extrapolated wall ghost.
__device__ inline int znb(const GridP& g, int k) {
  if (g.zbc == LES_ZBC_PERIODIC) {
    if (k == 0) return g.nz;
    if (k == g.nz + 1) return 1;
    return k;
  }
  if (k == 0 || k == g.nz + 1) return -1;
  return k;
}

// 3-D test filter of a z-centred field at (k, j, i): xy filter on planes k-1, k, k+1, then
// (1/4, 1/2, 1/4) in z; at a wall the missing plane is the extrapolation 2 q_1 - q_2 (R9).
template <typename T>
__device__ inline T filt3_centre(const GridP& g, const T* f, int k, int j, int i) {
  const T c = filt_xy(g, f, k, j, i);
  const int km = znb(g, k - 1), kp = znb(g, k + 1);
  T lo, hi;
  if (km >= 0) lo = filt_xy(g, f, km, j, i);
  if (kp >= 0) hi = filt_xy(g, f, kp, j, i);
  if (km < 0) lo = (T)2 * c - hi;
  if (kp < 0) hi = (T)2 * c - lo;
  return (T)0.25 * lo + (T)0.5 * c + (T)0.25 * hi;
}

// Sweep 2: test-filtered staggered velocity, each component on its own grid, with the
// ghost planes the strain routine expects.
template <typename T>
__global__ void __launch_bounds__(256) k_dsm_fvel(GridP g, const T* __restrict__ u, const T* __restrict__ v,
                                                  const T* __restrict__ w, T* __restrict__ uf, T* __restrict__ vf,
                                                  T* __restrict__ wf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z + 1;
  if (i >= g.nx || j >= g.ny) return;
  const int n = g.nz;
  const bool per = g.zbc == LES_ZBC_PERIODIC;
  const T a = filt3_centre(g, u, k, j, i);
  const T b = filt3_centre(g, v, k, j, i);
  T cw;
  if (!per && k == n) cw = (T)0;
  else cw = (T)0.25 * filt_xy(g, w, k - 1, j, i) + (T)0.5 * filt_xy(g, w, k, j, i) + (T)0.25 * filt_xy(g, w, k + 1, j, i);
  const int64_t c = idx3(g, k, j, i);
  uf[c] = a;
  vf[c] = b;
  wf[c] = cw;
  const int64_t c2 = (int64_t)j * g.nx + i, s = g.sxy;
  if (per) {
    if (k == n) { uf[c2] = a; vf[c2] = b; wf[c2] = cw; }
    if (k == 1) { uf[(n + 1) * s + c2] = a; vf[(n + 1) * s + c2] = b; wf[(n + 1) * s + c2] = cw; }
  } else {
    if (k == 1) { uf[c2] = -a; vf[c2] = -b; wf[c2] = (T)0; }
    if (k == n) { uf[(n + 1) * s + c2] = -a; vf[(n + 1) * s + c2] = -b; wf[(n + 1) * s + c2] = (T)0; }
  }
}

// Sweep 3: L_ij and M_ij at each cell, L_ij M_ij and M_ij M_ij summed per block and plane.
template <typename T>
__global__ void __launch_bounds__(256) k_dsm_lm(GridP g, const T* __restrict__ q9, int64_t fstride,
                                                const T* __restrict__ uf, const T* __restrict__ vf,
                                                const T* __restrict__ wf, double* __restrict__ part) {
  __shared__ double red[2][256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z + 1;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nthr = blockDim.x * blockDim.y;
  for (int t = tid; t < 256; t += nthr) red[0][t] = red[1][t] = 0.0;
  __syncthreads();
  double lm = 0.0, mm = 0.0;
  if (i < g.nx && j < g.ny) {
    const int n = g.nz;
    const bool wall_layer = g.zbc != LES_ZBC_PERIODIC && (k == 1 || k == n);
    const T alpha2 = wall_layer ? (T)2.5198420997897464 : (T)4;   // 4^(2/3) or 2^2
    const T d2 = (T)g.delta2[k];
    // filtered centre quantities; products formed point-wise before filtering
    const int ip = wrap_p(i, g.nx), im = wrap_m(i, g.nx), jp = wrap_p(j, g.ny), jm = wrap_m(j, g.ny);
    const int is[3] = {im, i, ip}, js[3] = {jm, j, jp};
    const T wgt[3] = {(T)0.25, (T)0.5, (T)0.25};
    T acc[3][15];
    const int kmn = znb(g, k - 1), kpn = znb(g, k + 1);
    const int planes[3] = {kmn, k, kpn};
    for (int pz = 0; pz < 3; ++pz) {
      for (int a = 0; a < 15; ++a) acc[pz][a] = (T)0;
      const int kk = planes[pz];
      if (kk < 0) continue;
      for (int dy = 0; dy < 3; ++dy) {
        T row[15];
        for (int a = 0; a < 15; ++a) row[a] = (T)0;
        for (int dx = 0; dx < 3; ++dx) {
          const int64_t c = idx3(g, kk, js[dy], is[dx]);
          const T uc = q9[c], vc = q9[fstride + c], wc = q9[2 * fstride + c];
          const T val[15] = {uc, vc, wc, uc * uc, vc * vc, wc * wc, uc * vc, uc * wc, vc * wc,
                             q9[3 * fstride + c], q9[4 * fstride + c], q9[5 * fstride + c],
                             q9[6 * fstride + c], q9[7 * fstride + c], q9[8 * fstride + c]};
          for (int a = 0; a < 15; ++a) row[a] = row[a] + wgt[dx] * val[a];
        }
        for (int a = 0; a < 15; ++a) acc[pz][a] = acc[pz][a] + wgt[dy] * row[a];
      }
    }
    if (kmn < 0)
      for (int a = 0; a < 15; ++a) acc[0][a] = (T)2 * acc[1][a] - acc[2][a];
    if (kpn < 0)
      for (int a = 0; a < 15; ++a) acc[2][a] = (T)2 * acc[1][a] - acc[0][a];
    T F[15];
    for (int a = 0; a < 15; ++a) F[a] = (T)0.25 * acc[0][a] + (T)0.5 * acc[1][a] + (T)0.25 * acc[2][a];
    T st[6];
    centre_strain(g, uf, vf, wf, k, j, i, st);
    const T stm = strain_mag(st);
    // component order 11 22 33 12 13 23
    const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int c = 0; c < 6; ++c) {
      const T L = F[3 + c] - F[pa[c]] * F[pb[c]];
      const T M = (T)2 * d2 * (F[9 + c] - alpha2 * stm * st[c]);
      const double wgt2 = c < 3 ? 1.0 : 2.0;
      lm += wgt2 * (double)L * (double)M;
      mm += wgt2 * (double)M * (double)M;
    }
  }
  red[0][tid] = lm;
  red[1][tid] = mm;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] += red[0][tid + s];
      red[1][tid] += red[1][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int64_t tile = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int64_t o = ((int64_t)(k - 1) * gridDim.x * gridDim.y + tile) * 2;
    part[o] = red[0][0];
    part[o + 1] = red[1][0];
  }
}

// Plane sums in a fixed order -> c_s(k) = max(0, <LM>/<MM>) (0 if <MM> = 0), whole box
// when z is periodic; coef[k] = c_s Delta_k^2 with ghost copies.
__global__ void k_dsm_reduce(GridP g, const double* part, int ntile, double* cs, double* coef) {
  const int n = g.nz;
  const bool per = g.zbc == LES_ZBC_PERIODIC;
  __shared__ double tot[2];
  if (per) {
    if (threadIdx.x == 0) {
      double a = 0.0, b = 0.0;
      for (int k = 0; k < n; ++k) {
        double pl = 0.0, pm = 0.0;
        for (int t = 0; t < ntile; ++t) {
          pl += part[((int64_t)k * ntile + t) * 2];
          pm += part[((int64_t)k * ntile + t) * 2 + 1];
        }
        a += pl;
        b += pm;
      }
      tot[0] = a;
      tot[1] = b;
    }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    double a = 0.0, b = 0.0;
    if (per) {
      a = tot[0];
      b = tot[1];
    } else {
      for (int t = 0; t < ntile; ++t) {
        a += part[((int64_t)k * ntile + t) * 2];
        b += part[((int64_t)k * ntile + t) * 2 + 1];
      }
    }
    const double c = b > 0.0 ? fmax(a / b, 0.0) : 0.0;
    cs[k] = c;
    coef[k + 1] = c * g.delta2[k + 1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double c1 = g.delta2[1] * cs[0], cn = g.delta2[n] * cs[n - 1];
    coef[0] = per ? cn : c1;
    coef[n + 1] = per ? c1 : cn;
  }
}

// ============================================================================ launcher
template <typename T>
void launch_eddy_viscosity(Ctx& c) {
  const GridP& g = c.g;
  Launch3 L = point_launch(g, g.nz);
  const int model = c.cfg.sgs;
  if (model == LES_SGS_NONE) return;
  const double pts = (double)g.sxy * g.nz;
  if (model == LES_SGS_SMAG || model == LES_SGS_SMAG_VD) {
    LES_LAUNCH(c, "strain_mag", 4 * pts * sizeof(T), k_strain_mag<T>, L.grid, L.block, 0, g, (const T*)c.u, (const T*)c.v,
                       (const T*)c.w, (T*)c.nut);
    if (model == LES_SGS_SMAG_VD && c.cfg.zbc != LES_ZBC_PERIODIC)
      LES_LAUNCH(c, "vd_coef", 0, k_vd_coef<T>, dim3(1), dim3(256), 0, g, (const T*)c.u, (const T*)c.v, c.t.tau,
                         c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0, c.cfg.cs, c.t.coef);
    return;
  }
  if (model == LES_SGS_DSM || model == LES_SGS_MLP) {
    const int64_t fs = (int64_t)c.field_elems;
    T* q9 = (T*)c.q9;
    T* fv = (T*)c.fvel;
    LES_LAUNCH(c, "dsm_centre", 13 * pts * sizeof(T), k_dsm_centre<T>, L.grid, L.block, 0, g, (const T*)c.u, (const T*)c.v, (const T*)c.w,
                       (T*)c.nut, q9, fs);
    LES_LAUNCH(c, "dsm_fvel", 6 * pts * sizeof(T), k_dsm_fvel<T>, L.grid, L.block, 0, g, (const T*)c.u, (const T*)c.v, (const T*)c.w,
                       fv, fv + fs, fv + 2 * fs);
    LES_LAUNCH(c, "dsm_lm", 12 * pts * sizeof(T), k_dsm_lm<T>, L.grid, L.block, 0, g, (const T*)q9, fs, (const T*)fv,
                       (const T*)(fv + fs), (const T*)(fv + 2 * fs), c.t.dsm_part);
    const int ntile = (int)(L.grid.x * L.grid.y);
    LES_LAUNCH(c, "dsm_reduce", 0, k_dsm_reduce, dim3(1), dim3(256), 0, g, c.t.dsm_part, ntile, c.t.cs, c.t.coef);
  }
}

template <typename T>
__global__ void k_read_nut(GridP g, const T* nut, const double* coef, T* dst, int64_t n) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int k = (int)(e / g.sxy);
  dst[e] = (T)coef[k] * nut[e];
}

template <typename T>
void launch_read_nut(Ctx& c, T* dst) {
  const int64_t n = (int64_t)c.field_elems;
  LES_LAUNCH(c, "read_nut", 2.0 * n * sizeof(T), k_read_nut<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.g,
                     (const T*)c.nut, c.t.coef, dst, n);
}

template void launch_eddy_viscosity<double>(Ctx&);
template void launch_eddy_viscosity<float>(Ctx&);
template void launch_read_nut<double>(Ctx&, double*);
template void launch_read_nut<float>(Ctx&, float*);

}  // namespace les
