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
// derivative in the first layer, Sec. 2.2), and in a duct those of u and w in y as well;
// otherwise the stored ghosts are used.
//
// Ducts (walls in y too, Sec. 4.4): the van Driest factor takes y* as the smallest of
// d_w u_tau,w / nu over the four walls and is folded into the stored field (|S| D^2), so
// the plane coefficient stays (C_s Delta_k)^2.
#include "les_internal.h"
#include "mlp_core.h"

#include <algorithm>

namespace les {

template <typename T>
struct VelView {
  const T* u;
  const T* v;
  const T* w;
};

// u or v at (k, j, i) with the z strain ghost rule.
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

// u or w of a duct with the wall model on a y ghost row: the linear extrapolation in y of the
// first two interior rows (uniform dy), taken after the z rule (zr: apply it, for u).
template <typename T>
__device__ inline T sval_y(const GridP& g, const T* f, int k, int j, int i, bool zr) {
  auto at = [&](int jj) { return zr ? sval(g, f, k, jj, i) : f[idx3(g, k, jj, i)]; };
  if (g.ywall && g.zbc == LES_ZBC_WALLMODEL && j >= g.ny) {
    if (j == g.ny + 1) {
      const T a0 = at(0), a1 = at(1);
      return a0 - (a1 - a0);
    }
    const T a0 = at(g.ny - 1), a1 = at(g.ny - 2);
    return a0 + (a0 - a1);
  }
  return at(j);
}

// Strain rate at the centre of cell (k, j, i): s[0..5] = S11 S22 S33 S12 S13 S23.
template <typename T>
__device__ inline void centre_strain(const GridP& g, const T* u, const T* v, const T* w, int k, int j, int i, T s[6]) {
  const int ip = wrap_p(i, g.nx), im = wrap_m(i, g.nx), jp = wrap_p(j, g.nys), jm = wrap_m(j, g.nys);
  const T rdx = (T)g.rdx, rdy = (T)g.rdy, h = (T)0.5, q = (T)0.25;
  const T rdzc = (T)g.rdzc[k], rdzcm = (T)g.rdzc[k - 1];
#define US(kk, jj, ii) sval_y(g, u, kk, jj, ii, true)
#define VS(kk, jj, ii) sval(g, v, kk, jj, ii)
#define W(kk, jj, ii) sval_y(g, w, kk, jj, ii, false)
  const T u0 = US(k, j, i), uim = US(k, j, im), ujp = US(k, jp, i), ujm = US(k, jm, i);
  const T ujp_im = US(k, jp, im), ujm_im = US(k, jm, im);
  const T v0 = VS(k, j, i), vjm = VS(k, jm, i), vip = VS(k, j, ip), vim = VS(k, j, im);
  const T vjm_ip = VS(k, jm, ip), vjm_im = VS(k, jm, im);
  s[0] = (u0 - uim) * rdx;
  s[1] = (v0 - vjm) * rdy;
  s[2] = (W(k, j, i) - W(k - 1, j, i)) * (T)g.rdzf[k];
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
                                                    const T* __restrict__ w, T* __restrict__ nut,
                                                    const double* __restrict__ vd4, double ly) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z + 1;
  if (i >= g.nx || j >= g.ny) return;
  T s[6];
  centre_strain(g, u, v, w, k, j, i, s);
  T val = strain_mag(s);
  if (vd4 != nullptr) {
    // duct van Driest factor (four walls): y* the smallest d_w u_tau,w / nu
    const double zc = g.zc[k], yc = (j + 0.5) * g.dy;
    const double ys = fmin(fmin(zc * vd4[0], (g.lz - zc) * vd4[1]), fmin(yc * vd4[2], (ly - yc) * vd4[3])) / g.nu;
    const double d = 1.0 - exp(-ys / 25.0);
    val = (T)((double)val * (d * d));
  }
  store_nut(g, nut, k, j, i, val);
}

// Friction velocities of the four duct walls for the van Driest factor: sqrt(|(<tau_1>,
// <tau_2>)|) per wall, each component averaged over its own points on that wall that are not
// wall faces (z walls: rows j < ny, the v stress over j < ny - 1; y walls: planes 1..nz, the w
// stress over faces 1..nz-1).  Stresses from the wall models, or nu times the wall-normal
// difference across the no-slip ghosts.  Stage 1: VD_BLOCKS blocks, each a fixed-order tree
// of its strided share into 8 partials (part[b][8]); stage 2: one block sums them in block
// order and writes vd4 = (z bottom, z top, y = 0, y = ly).
constexpr int VD_BLOCKS = 64;

template <typename T>
__global__ void __launch_bounds__(256) k_vd_duct_partial(GridP g, const T* u, const T* v, const T* w,
                                                         const double* tau, const double* tauy, int wallmodel,
                                                         double* part) {
  __shared__ double sm[8][256];
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int n = g.nz, ny = g.ny, nx = g.nx;
  const int64_t s = g.sxy, sy = (int64_t)(n + 2) * nx;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t c = t0; c < (int64_t)nx * ny; c += stride) {
    const bool vrow = c < (int64_t)nx * (ny - 1);   // v rows off the wall face y = ly
    if (wallmodel) {
      a[0] += tau[c];
      a[2] += tau[2 * s + c];
      if (vrow) {
        a[1] += tau[s + c];
        a[3] += tau[3 * s + c];
      }
    } else {
      a[0] += g.nu * ((double)u[s + c] - (double)u[c]) / g.dzc[0];
      a[2] += g.nu * ((double)u[(int64_t)n * s + c] - (double)u[(int64_t)(n + 1) * s + c]) / g.dzc[n];
      if (vrow) {
        a[1] += g.nu * ((double)v[s + c] - (double)v[c]) / g.dzc[0];
        a[3] += g.nu * ((double)v[(int64_t)n * s + c] - (double)v[(int64_t)(n + 1) * s + c]) / g.dzc[n];
      }
    }
  }
  for (int64_t e = t0; e < (int64_t)nx * n; e += stride) {
    const int k = (int)(e / nx) + 1, i = (int)(e % nx);
    const bool wface = k < n;   // w faces off the wall face k = nz
    if (wallmodel) {
      const int64_t o = (int64_t)k * nx + i;
      a[4] += tauy[o];
      a[6] += tauy[2 * sy + o];
      if (wface) {
        a[5] += tauy[sy + o];
        a[7] += tauy[3 * sy + o];
      }
    } else {
      a[4] += g.nu * ((double)u[idx3(g, k, 0, i)] - (double)u[idx3(g, k, ny + 1, i)]) / g.dy;
      a[6] += g.nu * ((double)u[idx3(g, k, ny - 1, i)] - (double)u[idx3(g, k, ny, i)]) / g.dy;
      if (wface) {
        a[5] += g.nu * ((double)w[idx3(g, k, 0, i)] - (double)w[idx3(g, k, ny + 1, i)]) / g.dy;
        a[7] += g.nu * ((double)w[idx3(g, k, ny - 1, i)] - (double)w[idx3(g, k, ny, i)]) / g.dy;
      }
    }
  }
  for (int q = 0; q < 8; ++q) sm[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int q = 0; q < 8; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 8) part[blockIdx.x * 8 + threadIdx.x] = sm[threadIdx.x][0];
}

// sums of q-strided block partials (nq per block, VD_BLOCKS = 64 blocks: one lane each) by a
// fixed-order shuffle tree within one wave; lane 0 holds the totals
__device__ inline void wave_block_sums(const double* part, int nq, double* a) {
  const int lane = threadIdx.x & 63;
  for (int q = 0; q < nq; ++q) {
    double x = lane < VD_BLOCKS ? part[lane * nq + q] : 0.0;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    a[q] = x;
  }
}

// cnt (learned closure, may be null): the fallback counters are cleared here, ahead of the
// inference kernel that adds to them.
__global__ void k_vd_duct_final(GridP g, const double* part, double* vd4, int* cnt) {
  static_assert(VD_BLOCKS <= 64, "one lane per block partial");
  double a[8];
  wave_block_sums(part, 8, a);
  if (threadIdx.x != 0) return;
  if (cnt != nullptr) {
    cnt[0] = 0;
    cnt[1] = 0;
  }
  const double nx = g.nx, ny = g.ny, n = g.nz;
  const double cz = nx * ny, cv = nx * (ny - 1), cy = nx * n, cw = nx * (n - 1);
  vd4[0] = sqrt(hypot(a[0] / cz, a[1] / cv));
  vd4[1] = sqrt(hypot(a[2] / cz, a[3] / cv));
  vd4[2] = sqrt(hypot(a[4] / cy, a[5] / cw));
  vd4[3] = sqrt(hypot(a[6] / cy, a[7] / cw));
}

// van Driest coefficient: plane-mean wall stresses -> u_tau per wall -> coef[k].
// tau = wall-model stresses, or (no-slip) nu (u_1 - u_0)/dzc_0 from the ghosts.  Stage 1:
// VD_BLOCKS blocks of fixed-order partials of the four plane sums (part[b][4]); stage 2, one
// block: the sums in block order, u_tau per wall, then coef[k] for every plane.
template <typename T>
__global__ void __launch_bounds__(256) k_vd_coef_partial(GridP g, const T* u, const T* v, const double* tau,
                                                         int wallmodel, double* part) {
  __shared__ double sm[4][256];
  double a[4] = {0, 0, 0, 0};
  const int64_t s = g.sxy;
  const int n = g.nz;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < s; c += stride) {
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
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_vd_coef_final(GridP g, const double* part, double cs,
                                                       double* coef) {
  __shared__ double ut[2];
  const int n = g.nz;
  double a[4];
  if (threadIdx.x < 64) wave_block_sums(part, 4, a);
  if (threadIdx.x == 0) {
    const double s = (double)g.sxy;
    ut[0] = sqrt(hypot(a[0] / s, a[1] / s));
    ut[1] = sqrt(hypot(a[2] / s, a[3] / s));
  }
  __syncthreads();
  for (int k = threadIdx.x + 1; k <= n; k += blockDim.x) {
    const double zc = g.zc[k];
    const bool lower = zc <= 0.5 * g.lz;
    const double d = lower ? zc : g.lz - zc;
    const double utk = lower ? ut[0] : ut[1];
    const double damp = 1.0 - exp(-d * utk / g.nu / 25.0);
    const double f = cs * sqrt(g.delta2[k]) * damp;
    coef[k] = f * f;
    if (k == 1) coef[0] = f * f;
    if (k == n) coef[n + 1] = f * f;
  }
}

// ============================================================================ dynamic model
// Plane sums in a fixed order -> c_s(k) = max(0, <LM>/<MM>) (0 if <MM> = 0), whole box
// when z is periodic; coef[k] = c_s Delta_k^2 with ghost copies.  One block per plane:
// strided partial sums over the tiles, then a fixed-order tree.  With periodic z every block
// forms the total over all planes itself (same order in every block).
template <typename T>
__device__ __forceinline__ void dsm_reduce_body(int k, GridP g, const double* part, int ntile, double* cs,
                                                double* coef, const int* gate, T* fnut) {
  if (gate != nullptr && gate[0] == 0) return;
  __shared__ double sm[2][256];
  const int n = g.nz;
  const bool per = g.zbc == LES_ZBC_PERIODIC;
  double a = 0.0, b = 0.0;
  if (per) {
    for (int64_t e = threadIdx.x; e < (int64_t)n * ntile; e += 256) {
      a += part[2 * e];
      b += part[2 * e + 1];
    }
  } else {
    for (int t = threadIdx.x; t < ntile; t += 256) {
      a += part[((int64_t)k * ntile + t) * 2];
      b += part[((int64_t)k * ntile + t) * 2 + 1];
    }
  }
  sm[0][threadIdx.x] = a;
  sm[1][threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + st];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  const double sa = sm[0][0], sb = sm[1][0];
  const double c = sb > 0.0 ? fmax(sa / sb, 0.0) : 0.0;
  if (threadIdx.x == 0) {
    cs[k] = c;
    if (coef != nullptr) {
      coef[k + 1] = c * g.delta2[k + 1];
      if (k == 0) coef[per ? n + 1 : 0] = c * g.delta2[1];
      if (k == n - 1) coef[per ? 0 : n + 1] = c * g.delta2[n];
    }
  }
  if (fnut != nullptr) {
    // learned closure: the cells of this plane that the network left to the dynamic model
    // (stored -|S|) take c |S|
    const int64_t nxy = (int64_t)g.nx * g.ny;
    for (int64_t r = threadIdx.x; r < nxy; r += blockDim.x) {
      const int j = (int)(r / g.nx), i = (int)(r % g.nx);
      const T val = fnut[idx3(g, k + 1, j, i)];
      if (val < (T)0) store_nut(g, fnut, k + 1, j, i, (T)c * -val);
    }
  }
}

// fnut (learned closure, may be null): also the fallback of the plane's flagged cells
template <typename T>
__global__ void __launch_bounds__(256) k_dsm_reduce(GridP g, const double* part, int ntile, double* cs,
                                                    double* coef, const int* gate, T* fnut) {
  dsm_reduce_body<T>(blockIdx.x, g, part, ntile, cs, coef, gate, fnut);
}

// ============================================================================ fused dynamic model
// One z-marching pass per (32 x 8 tile, chunk of planes) computing |S| and the plane sums
// of L_ij M_ij and M_ij M_ij, reading u, v, w once (halo 2) and writing |S| once.
//   LDS: velocity of planes p, p + 1 on the tile + 2 halo (strain ghosts substituted),
//        the 15 filter inputs (u_i, u_i u_j, |S| S_ij at cell centres) of plane p on the
//        tile + 1 halo, stored in pairs (one 16-byte read per pair in the filter), the
//        test-filtered staggered velocity of two planes on the tile + 1 halo.
//   Registers: the z pass of the test filter as running sums over the thread's cell; the
//        upper z-edge terms of the off-diagonal strain and w of the previous plane at the
//        thread's points, which are the lower terms of the plane above (so only planes k and
//        k + 1 are needed to form the strain of plane k).
// The stage of plane p forms the filter inputs of plane p from velocity planes p, p + 1 and
// completes the filtered velocity of plane p - 1; once stage p is done the cell values of plane
// p - 1 are final (z pass of the test filter, S~ from the filtered velocity, L and M).
// Wall rules as in the rest of the dynamic model: on the first off-wall layers the z pass of
// the filter is the identity (the index-space extrapolation of the neighbour reduces to it),
// filtered-velocity ghosts follow the strain ghost rule, alpha^2 = 4^(2/3) there.
// Tiles of 32 x 16 cells in FP64 (one 512-thread block per CU: the LDS of a block is about
// 140 KB, and the halo is a smaller share of the tile) and 32 x 8 in FP32 (three 256-thread
// blocks per CU) and in the duct variant (YW; two blocks per CU in FP64).
namespace fused {
constexpr int TX = 32;
constexpr int NQ = 15;   // filter inputs per cell
template <typename T, bool YW = false>
struct Tile {
  static constexpr int TY = dsm_tile_rows(sizeof(T) == 8 && !YW), NT = TX * TY, WV = NT / 64;
  static constexpr int RX2 = TX + 4, RY2 = TY + 4, N2 = RX2 * RY2;  // halo 2
  static constexpr int RX1 = TX + 2, RY1 = TY + 2, N1 = RX1 * RY1;  // halo 1
  static constexpr int NHALO = 2 * (RX1 + TY);                       // halo-1 points around the tile
  static constexpr int MINB = sizeof(T) == 8 ? (YW ? 2 : 1) : 3;     // blocks per CU
};
}  // namespace fused

// Upper z-edge terms at a cell of plane k: (du/dz + dw/dx) / 2 on the x-z edges of the cell's
// two x faces (fa: the face of u_i, fb: of u_{i-1}), (dv/dz + dw/dy) / 2 on the y-z edges of
// its two y faces (ga, gb), all on the face between planes k and k + 1, and w on that face.
// They are the lower edge terms of the cell above.
template <typename T>
struct ZEdges {
  T fa, fb, ga, gb, w;
};

// from an accessor A(c, dz, o): component c (0 u, 1 v, 2 w) of plane k + dz (dz in {0, 1}) at
// plane offset o; sy is one step in y, rdzc the reciprocal centre spacing above plane k
template <typename T, typename Acc>
__device__ inline ZEdges<T> zedges(const Acc& A, int o, int sy, T rdx, T rdy, T rdzc) {
  const T h = (T)0.5;
  ZEdges<T> E;
  const T w0 = A(2, 0, o);
  E.fa = h * ((A(0, 1, o) - A(0, 0, o)) * rdzc + (A(2, 0, o + 1) - w0) * rdx);
  E.fb = h * ((A(0, 1, o - 1) - A(0, 0, o - 1)) * rdzc + (w0 - A(2, 0, o - 1)) * rdx);
  E.ga = h * ((A(1, 1, o) - A(1, 0, o)) * rdzc + (A(2, 0, o + sy) - w0) * rdy);
  E.gb = h * ((A(1, 1, o - sy) - A(1, 0, o - sy)) * rdzc + (w0 - A(2, 0, o - sy)) * rdy);
  E.w = w0;
  return E;
}

// strain at a cell of plane k (Sec. 2.2: diagonal terms from face differences, off-diagonal
// terms as means of four edge values) from the accessor over plane k, the lower edge terms P
// (the upper terms of plane k - 1) and the cell's own upper terms E
template <typename T, typename Acc>
__device__ inline void strain_zm(const Acc& A, int o, int sy, T rdx, T rdy, T rdzf, const ZEdges<T>& P,
                                 const ZEdges<T>& E, T s[6]) {
  const T h = (T)0.5, q = (T)0.25;
  const T u0 = A(0, 0, o), uim = A(0, 0, o - 1), ujp = A(0, 0, o + sy), ujm = A(0, 0, o - sy);
  const T ujp_im = A(0, 0, o + sy - 1), ujm_im = A(0, 0, o - sy - 1);
  const T v0 = A(1, 0, o), vjm = A(1, 0, o - sy), vip = A(1, 0, o + 1), vim = A(1, 0, o - 1);
  const T vjm_ip = A(1, 0, o - sy + 1), vjm_im = A(1, 0, o - sy - 1);
  s[0] = (u0 - uim) * rdx;
  s[1] = (v0 - vjm) * rdy;
  s[2] = (E.w - P.w) * rdzf;
  const T e_a = h * ((ujp - u0) * rdy + (vip - v0) * rdx);
  const T e_b = h * ((ujp_im - uim) * rdy + (v0 - vim) * rdx);
  const T e_c = h * ((u0 - ujm) * rdy + (vjm_ip - vjm) * rdx);
  const T e_d = h * ((uim - ujm_im) * rdy + (vjm - vjm_im) * rdx);
  s[3] = q * (e_a + e_b + e_c + e_d);
  s[4] = q * (E.fa + E.fb + P.fa + P.fb);
  s[5] = q * (E.ga + E.gb + P.ga + P.gb);
}

// x of another lane of the same row of 16 lanes, by a DPP lane pattern
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false));
}
// sum over each row of 16 lanes, a 4-level tree (partners at lane distance 1 and 2 in a quad,
// then the mirrored half-row and row): every lane of a row holds the same bits
__device__ inline double row_sum(double x) {
  x = x + dpp_f64<0xB1>(x);    // quad permutation 1 0 3 2
  x = x + dpp_f64<0x4E>(x);    // quad permutation 2 3 0 1
  x = x + dpp_f64<0x141>(x);   // half-row mirror
  x = x + dpp_f64<0x140>(x);   // row mirror
  return x;
}
// lane L's value of x, uniform across the wave
__device__ inline double lane_f64(double x, int L) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), L),
                          __builtin_amdgcn_readlane(__double2loint(x), L));
}
template <typename T>
__device__ inline T strain_norm(const T s[6]) {
  return sqrt((T)2 * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]) + (T)4 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
}

// YW (ducts, walls in y too): the y pass of the test filter is the identity on the first and
// last rows for y-centred quantities (u, w and the 15 cell quantities), v~ vanishes on and
// beyond the y wall faces, the y ghost rows of u~ and w~ follow the strain ghost rule, alpha^2
// counts the filter's dimensions per cell, and the partial sums are per x line (one per row
// of each wave: 32 lanes) instead of per wave.
template <typename T, bool YW = false, int ZBC = -1>
__device__ __forceinline__ void dsm_fused_body(dim3 bid, int gdx, int gdy, GridP g, const T* __restrict__ u,
                                               const T* __restrict__ v, const T* __restrict__ w,
                                               T* __restrict__ nut, double* __restrict__ part, int kc,
                                               const int* __restrict__ gate) {
  using TL = fused::Tile<T, YW>;
  constexpr int TX = fused::TX, TY = TL::TY, NT = TL::NT, WV = TL::WV, NQ = fused::NQ;
  constexpr int RX2 = TL::RX2, N2 = TL::N2, RX1 = TL::RX1, RY1 = TL::RY1, N1 = TL::N1, NHALO = TL::NHALO;
  if (gate != nullptr && gate[0] == 0) return;   // learned closure: no point fell back
  constexpr int NL = (N2 + NT - 1) / NT;          // halo-2 points per thread (loads)
  constexpr int NH = (N1 + NT - 1) / NT;          // halo-1 points per thread (velocity filter)
  __shared__ T vel[2][3][N2];   // [plane & 1][component][R2]
  typedef HIP_vector_type<T, 2> T2;
  __shared__ T2 qb[(NQ + 1) / 2][N1];   // filter inputs of the current stage plane, in pairs
  __shared__ T ut[2][3][N1];    // filtered velocity [plane & 1][component][R1]
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int i0 = bid.x * TX, j0 = bid.y * TY;
  const int nz = g.nz;
  const int kb = 1 + bid.z * kc;
  const int ke = min(nz, kb + kc - 1);
  const int zbc = ZBC < 0 ? g.zbc : ZBC;   // ZBC >= 0: the z boundary fixed at compile time
  const bool per = zbc == LES_ZBC_PERIODIC;
  const bool wm = zbc == LES_ZBC_WALLMODEL;
  const int ntile = gdx * gdy;
  const int tile = bid.y * gdx + bid.x;
  const T rdx = (T)g.rdx, rdy = (T)g.rdy;
  const T W0 = (T)0.25, W1 = (T)0.5;
  const int64_t sxy = g.sxy;
  auto phys = [&](int q) {  // logical plane -> stored plane (periodic wrap of interior planes)
    if (!per) return q;
    int m = (q - 1) % nz;
    if (m < 0) m += nz;
    return m + 1;
  };
  // the z spacing above plane q as the plane above sees it (they differ only across the
  // periodic wrap, where the stored spacings at both ends are separately rounded)
  auto rdzc_above = [&](int q) { return (T)ro_load(g.rdzc, phys(q + 1) - 1); };
  // in-plane offsets of the thread's halo-2 load points (tiles may exceed the grid: wrap)
  int lofs[NL];
  for (int r = 0; r < NL; ++r) {
    const int e = tid + r * NT;
    const int rx = e % RX2, ry = e / RX2;
    int i = (i0 - 2 + rx) % g.nx, j = (j0 - 2 + ry) % g.nys;
    if (i < 0) i += g.nx;
    if (j < 0) j += g.nys;
    lofs[r] = e < N2 ? j * g.nx + i : 0;
  }
  // global row of a load point before the wrap (ducts)
  auto lrow = [&](int r) { return j0 - 2 + (tid + r * NT) / RX2; };
  // velocity of one plane held in registers between its fetch and its commit to LDS, so that
  // the global loads of plane p + 2 overlap the work on plane p: the loads are raw and
  // unconditional (points past the halo read offset 0 and are not committed)
  T ra[NL], rb[NL], rc[NL];
  auto fetch = [&](int q) {
    const int pq = phys(q);
    const PlaneLoader<T> lu(u, pq, sxy), lv(v, pq, sxy), lw(w, pq, sxy);
    for (int r = 0; r < NL; ++r) {
      ra[r] = lu(lofs[r]);
      rb[r] = lv(lofs[r]);
      rc[r] = lw(lofs[r]);
    }
    if (YW && wm) {
      const int64_t bw = (int64_t)pq * sxy;
      for (int r = 0; r < NL; ++r) {
        if (tid + r * NT < N2 && (lrow(r) == -1 || lrow(r) == g.ny)) {
          // duct: strain ghosts of u and w on the y ghost rows, extrapolated in y
          const int64_t o0 = bw + (lofs[r] % g.nx) + (int64_t)(lrow(r) < 0 ? 0 : g.ny - 1) * g.nx;
          const int64_t o1 = o0 + (lrow(r) < 0 ? g.nx : -g.nx);
          const T a0 = u[o0], a1 = u[o1], c0 = w[o0], c1 = w[o1];
          ra[r] = a0 - (a1 - a0);
          rc[r] = c0 - (c1 - c0);
        }
      }
    }
  };
  auto yghost = [&](int r) { return YW && (lrow(r) == -1 || lrow(r) == g.ny); };
  // commit plane q to its ring slot; with the wall model the top ghost plane's u, v are the
  // linear extrapolation in z of planes nz and nz - 1 (the thread's own entries; plane nz - 1
  // sits in the slot being replaced, read before it is overwritten)
  auto commit = [&](int q) {
    const int sl = q & 1;
    if (wm && phys(q) == nz + 1) {
      const int s1 = (q - 1) & 1;
      const T ca = (T)ro_load(g.dzc, nz), cb = (T)ro_load(g.dzc, nz - 1);
      for (int r = 0; r < NL; ++r) {
        const int e = tid + r * NT;
        if (e < N2) {
          const T b1 = vel[s1][1][e], b2 = vel[sl][1][e];
          rb[r] = b1 + ca * ((b1 - b2) / cb);
          // ducts: u on a y ghost row keeps its y extrapolation of the stored plane (corner rule)
          if (!yghost(r)) {
            const T a1 = vel[s1][0][e], a2 = vel[sl][0][e];
            ra[r] = a1 + ca * ((a1 - a2) / cb);
          }
        }
      }
    }
    for (int r = 0; r < NL; ++r) {
      const int e = tid + r * NT;
      if (e < N2) {
        vel[sl][0][e] = ra[r];
        vel[sl][1][e] = rb[r];
        vel[sl][2][e] = rc[r];
      }
    }
  };
  // z pass of the velocity filter by partial sums: G1 holds plane p's sum without its upper
  // neighbour, G2 plane p + 1's lower-neighbour term; z weights per plane (lower, centre,
  // upper) are (0, 1, 0) for u, v on the first off-wall layers and 0 for w on the top wall face
  T G1[NH][3], G2[NH][3];
  auto zw = [&](int q, int c, int which) -> T {
    if (!per && c == 2 && q == nz) return (T)0;
    if (!per && c < 2 && (q == 1 || q == nz)) return which == 1 ? (T)1 : (T)0;
    return which == 1 ? W1 : W0;
  };
  // x-y filter of velocity plane q at the thread's halo-1 points, folded into the z sums;
  // completes the filtered velocity of plane q - 1 (written to its ring slot when put != 0)
  auto filter_xy = [&](int q, bool put) {
    const int sl = q & 1, so = (q - 1) & 1;
    for (int r = 0; r < NH; ++r) {
      const int e = tid + r * NT;
      if (e < N1) {
        // the thread's halo-1 points for the velocity filter (R2 coordinates)
        const int hx = e % RX1 + 1, hy = e / RX1 + 1;
        const int jr = j0 - 2 + hy;   // global row of the point
        const bool yedge = YW && (jr == 0 || jr == g.ny - 1);
        for (int c = 0; c < 3; ++c) {
          T pl = (T)0;
          for (int dy = -1; dy <= 1; ++dy) {
            const T* rr = &vel[sl][c][(hy + dy) * RX2 + hx];
            const T row = W0 * rr[-1] + W1 * rr[0] + W0 * rr[1];
            const T wy = (yedge && c != 1) ? (dy == 0 ? (T)1 : (T)0) : (dy == 0 ? W1 : W0);
            pl = pl + wy * row;
          }
          if (YW && c == 1 && (jr >= g.ny - 1 || jr < 0)) pl = (T)0;   // v~ on and beyond the y walls
          if (put) ut[so][c][e] = G1[r][c] + zw(q - 1, c, 2) * pl;
          G1[r][c] = G2[r][c] + zw(q, c, 1) * pl;
          G2[r][c] = zw(q + 1, c, 0) * pl;
        }
      }
    }
  };
  // ducts: the y ghost rows of u~ and w~ of plane q by the strain ghost rule (extrapolated
  // with the wall model, odd with no-slip), from the completed rows next to them
  auto fix_rows = [&](int q) {
    const int sl = q & 1;
    for (int e = tid; e < N1; e += NT) {
      const int jr = j0 - 1 + e / RX1;
      if (jr != -1 && jr != g.ny) continue;
      const int d = jr < 0 ? RX1 : -RX1;   // one row inward
      for (int c = 0; c < 3; c += 2) {
        const T a0 = ut[sl][c][e + d];
        ut[sl][c][e] = wm ? a0 - (ut[sl][c][e + 2 * d] - a0) : -a0;
      }
    }
  };
  // the thread's stage points: its own cell and, on the first NHALO threads, one halo-1 point
  // (R2 coordinates); each carries the upper z-edge terms of the previous plane
  const int ox = tx + 2, oy = ty + 2;
  const bool has_halo = tid < NHALO;
  int bx = 1, by = 1;
  if (has_halo) {
    const int h = tid;
    if (h < 2 * RX1) {
      bx = h % RX1 + 1;
      by = h < RX1 ? 1 : RY1;
    } else {
      bx = (h - 2 * RX1) < TY ? 1 : RX1;
      by = (h - 2 * RX1) % TY + 2;
    }
  }
  ZEdges<T> P0, P1;   // velocity: own cell, halo point
  ZEdges<T> PT;       // filtered velocity: own cell
  auto vacc = [](int s0, int s1) {
    return [=](int c, int dz, int o) -> T { return vel[dz ? s1 : s0][c][o]; };
  };
  // running sums of the z pass of the test filter over the thread's cell: S1 holds plane p's
  // sum without its upper neighbour, S2 plane p + 1's lower-neighbour term
  T S1[NQ], S2[NQ], qx[NQ];
  auto zq = [&](int q, int which) -> T {
    if (!per && (q == 1 || q == nz)) return which == 1 ? (T)1 : (T)0;
    return which == 1 ? W1 : W0;
  };
  // ---- stage p: filter inputs of plane p at the tile + 1 halo, then their x-y filter at the
  // thread's cell (into qx)
  auto stage = [&](int p) {
    const int pq = phys(p);
    const int s0 = p & 1, s1 = (p + 1) & 1;
    const T rdzf = (T)ro_load(g.rdzf, pq), rdzc = (T)ro_load(g.rdzc, pq);
    const T rdzn = rdzc_above(p);
    const bool wrap = phys(p + 1) - 1 != pq;
    const bool own = p >= kb && p <= ke;
    const auto A = vacc(s0, s1);
    auto point = [&](int x, int y, ZEdges<T>& P, bool store) {
      const int o = y * RX2 + x;
      const ZEdges<T> E = zedges<T>(A, o, RX2, rdx, rdy, rdzc);
      T s[6];
      strain_zm<T>(A, o, RX2, rdx, rdy, rdzf, P, E, s);
      const T sm_ = strain_norm<T>(s);
      const int e = (y - 1) * RX1 + x - 1;
      const T uc = (T)0.5 * (A(0, 0, o) + A(0, 0, o - 1));
      const T vc = (T)0.5 * (A(1, 0, o) + A(1, 0, o - RX2));
      const T wc = (T)0.5 * (E.w + P.w);
      qb[0][e] = T2(uc, vc);
      qb[1][e] = T2(wc, uc * uc);
      qb[2][e] = T2(vc * vc, wc * wc);
      qb[3][e] = T2(uc * vc, uc * wc);
      qb[4][e] = T2(vc * wc, sm_ * s[0]);
      qb[5][e] = T2(sm_ * s[1], sm_ * s[2]);
      qb[6][e] = T2(sm_ * s[3], sm_ * s[4]);
      qb[7][e] = T2(sm_ * s[5], (T)0);
      if (store && nut != nullptr && own) {
        const int i = i0 + tx, j = j0 + ty;
        if (i < g.nx && j < g.ny) store_nut(g, nut, p, j, i, sm_);
      }
      if (wrap)
        P = zedges<T>(A, o, RX2, rdx, rdy, rdzn);
      else
        P = E;
    };
    point(ox, oy, P0, true);
    if (has_halo) point(bx, by, P1, false);
    lds_barrier();
    // x-y filter of the 15 inputs at the thread's own cell (R1 coords tx+1, ty+1)
    for (int a = 0; a < NQ; ++a) qx[a] = (T)0;
    const bool yedge = YW && (j0 + ty == 0 || j0 + ty == g.ny - 1);
#pragma unroll 1
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll 1
      for (int dx = -1; dx <= 1; ++dx) {
        const T wy = yedge ? (dy == 0 ? (T)1 : (T)0) : (dy == 0 ? W1 : W0);
        const T wxy = wy * (dx == 0 ? W1 : W0);
        const int e = (ty + 1 + dy) * RX1 + tx + 1 + dx;
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          const T2 pr = qb[a / 2][e];
          qx[a] = qx[a] + wxy * (a % 2 ? pr.y : pr.x);
        }
      }
  };
  // ---- output plane k: F holds the test-filtered inputs of its cell; the filtered velocity of
  // planes k and k + 1 is in the ring (the top ghost plane is formed on the fly), PT holds the
  // upper edge terms of plane k - 1
  auto output = [&](int k, const T* F) {
    const int pk = phys(k);
    double lm = 0.0, mm = 0.0;
    const int i = i0 + tx, j = j0 + ty;
    const int o = (ty + 1) * RX1 + tx + 1;   // own cell in R1
    const int sA = k & 1, sB = (k + 1) & 1;
    const bool top = !per && k == nz;
    const T rdzc = (T)ro_load(g.rdzc, pk), rdzf = (T)ro_load(g.rdzf, pk);
    T st[6];
    if (top) {
      // strain ghost rule above the top wall, from planes nz (slot sA) and nz - 1 (slot sB)
      const T ca = (T)ro_load(g.dzc, nz), cb = (T)ro_load(g.dzc, nz - 1);
      const auto A = [&](int c, int dz, int oo) -> T {
        const T a1 = ut[sA][c][oo];
        if (dz == 0) return a1;
        const T a2 = ut[sB][c][oo];
        return wm ? a1 + ca * ((a1 - a2) / cb) : -a1;
      };
      strain_zm<T>(A, o, RX1, rdx, rdy, rdzf, PT, zedges<T>(A, o, RX1, rdx, rdy, rdzc), st);
    } else {
      const auto A = [&](int c, int dz, int oo) -> T { return ut[dz ? sB : sA][c][oo]; };
      const ZEdges<T> E = zedges<T>(A, o, RX1, rdx, rdy, rdzc);
      strain_zm<T>(A, o, RX1, rdx, rdy, rdzf, PT, E, st);
      if (phys(k + 1) - 1 != pk)
        PT = zedges<T>(A, o, RX1, rdx, rdy, rdzc_above(k));
      else
        PT = E;
    }
    if (i < g.nx && j < g.ny) {
      const T stm = strain_norm<T>(st);
      const bool wall_layer = !per && (k == 1 || k == nz);
      const bool wall_row = YW && (j == 0 || j == g.ny - 1);
      // 3-D, 2-D or (duct corners) 1-D test filter: 4, 4^(2/3), 2^(2/3)
      const T alpha2 = (wall_layer && wall_row) ? (T)1.5874010519681994
                                                : ((wall_layer || wall_row) ? (T)2.5198420997897464 : (T)4);
      const T d2 = (T)ro_load(g.delta2, pk);
      const T Fa[6] = {F[0], F[1], F[2], F[0], F[0], F[1]}, Fb[6] = {F[0], F[1], F[2], F[1], F[2], F[2]};
      for (int c = 0; c < 6; ++c) {
        const T L = F[3 + c] - Fa[c] * Fb[c];
        const T M = (T)2 * d2 * (F[9 + c] - alpha2 * stm * st[c]);
        const double wgt2 = c < 3 ? 1.0 : 2.0;
        lm += wgt2 * (double)L * (double)M;
        mm += wgt2 * (double)M * (double)M;
      }
    }
    lm = row_sum(lm);
    mm = row_sum(mm);
    if (YW) {
      // x-line sums: a row of the tile is 32 lanes (two rows of 16) of one wave; partials
      // [k][j][tile x]
      const bool lo = (tid & 63) < 32;
      lm = lo ? lane_f64(lm, 0) + lane_f64(lm, 16) : lane_f64(lm, 32) + lane_f64(lm, 48);
      mm = lo ? lane_f64(mm, 0) + lane_f64(mm, 16) : lane_f64(mm, 32) + lane_f64(mm, 48);
      const int jrow = j0 + ty;
      if (tx == 0 && jrow < g.ny) {
        const int64_t oo = (((int64_t)(k - 1) * g.ny + jrow) * gdx + bid.x) * 2;
        part[oo] = lm;
        part[oo + 1] = mm;
      }
      return;
    }
    // wave sums in a fixed order (row trees, then the four rows in turn); the waves' partials
    // go out per plane and are summed over (tile, wave) in a fixed order by the plane reduction
    lm = ((lane_f64(lm, 0) + lane_f64(lm, 16)) + lane_f64(lm, 32)) + lane_f64(lm, 48);
    mm = ((lane_f64(mm, 0) + lane_f64(mm, 16)) + lane_f64(mm, 32)) + lane_f64(mm, 48);
    if (tid % 64 == 0) {
      const int64_t oo = ((int64_t)(k - 1) * ntile * WV + tile * WV + tid / 64) * 2;
      part[oo] = lm;
      part[oo + 1] = mm;
    }
  };
  // ---- prologue: planes pstart - 1 and pstart in the ring, pstart + 1 in flight
  const int pstart = per ? kb - 1 : max(kb - 1, 1);
  const int pend = per ? ke + 1 : min(ke + 1, nz);
  if (wm && pstart == 1) {
    // the bottom ghost plane: u, v extrapolated linearly in z from planes 1 (in the ring) and
    // 2 (held in registers), w and the duct's y-ghost u as stored
    fetch(1);
    commit(1);
    fetch(2);
    T xa[NL], xb[NL];
    for (int r = 0; r < NL; ++r) {
      xa[r] = ra[r];
      xb[r] = rb[r];
    }
    fetch(0);
    const T ca = (T)ro_load(g.dzc, 0), cb = (T)ro_load(g.dzc, 1);
    for (int r = 0; r < NL; ++r) {
      const int e = tid + r * NT;
      if (e < N2) {
        const T b1 = vel[1][1][e];
        rb[r] = b1 - ca * ((xb[r] - b1) / cb);
        if (!yghost(r)) {
          const T a1 = vel[1][0][e];
          ra[r] = a1 - ca * ((xa[r] - a1) / cb);
        }
      }
    }
    commit(0);
    fetch(2);
  } else {
    fetch(pstart - 1);
    commit(pstart - 1);
    fetch(pstart);
    commit(pstart);
    fetch(pstart + 1);
  }
  lds_barrier();
  for (int r = 0; r < NH; ++r)
    for (int c = 0; c < 3; ++c) G2[r][c] = (T)0;
  filter_xy(pstart - 1, false);
  filter_xy(pstart, false);
  {
    const auto A = vacc((pstart - 1) & 1, pstart & 1);
    const T rdzn = rdzc_above(pstart - 1);
    P0 = zedges<T>(A, oy * RX2 + ox, RX2, rdx, rdy, rdzn);
    if (has_halo) P1 = zedges<T>(A, by * RX2 + bx, RX2, rdx, rdy, rdzn);
  }
  for (int a = 0; a < NQ; ++a) S2[a] = (T)0;
  lds_barrier();   // the first commit replaces plane pstart - 1
  // ---- march: velocity plane p + 1 is committed to LDS at the top of iteration p, the loads
  // of plane p + 2 are issued right after and complete under the work on plane p.  Threads
  // exchange data through LDS only (the stored |S| and partial sums are read by later
  // launches): the barriers leave global loads in flight.
  for (int p = pstart; p <= pend; ++p) {
    commit(p + 1);
    lds_barrier();
    fetch(min(p + 2, pend + 1));   // the last one reloads plane pend + 1 and is not committed
    filter_xy(p + 1, true);
    stage(p);
    if (YW) {
      fix_rows(p);
      lds_barrier();
    }
    const int k = p - 1;
    if (k == kb - 1 && (per || kb > 1)) {
      // upper edge terms of the filtered velocity below the first output plane
      const auto A = [&](int c, int dz, int oo) -> T { return ut[dz ? (p & 1) : (k & 1)][c][oo]; };
      PT = zedges<T>(A, (ty + 1) * RX1 + tx + 1, RX1, rdx, rdy, rdzc_above(k));
    }
    if (k >= kb && k <= ke) {
      if (!per && k == 1) {
        // below the bottom wall: the strain ghost rule from planes 1 and 2, w~ = 0 on the wall
        const T ca = (T)ro_load(g.dzc, 0), cb = (T)ro_load(g.dzc, 1);
        const auto A = [&](int c, int dz, int oo) -> T {
          if (dz) return ut[1][c][oo];
          if (c == 2) return (T)0;
          const T a1 = ut[1][c][oo], a2 = ut[0][c][oo];
          return wm ? a1 - ca * ((a2 - a1) / cb) : -a1;
        };
        PT = zedges<T>(A, (ty + 1) * RX1 + tx + 1, RX1, rdx, rdy, (T)ro_load(g.rdzc, 0));
      }
      for (int a = 0; a < NQ; ++a) S1[a] = S1[a] + zq(k, 2) * qx[a];
      output(k, S1);
    }
    for (int a = 0; a < NQ; ++a) {
      S1[a] = S2[a] + zq(p, 1) * qx[a];
      S2[a] = zq(p + 1, 0) * qx[a];
    }
  }
  if (!per && ke == nz) output(nz, S1);   // the z pass is the identity on the top layer
}

template <typename T, bool YW = false, int ZBC = -1>
__global__ void __launch_bounds__((fused::Tile<T, YW>::NT), (fused::Tile<T, YW>::MINB)) k_dsm_fused(GridP g, const T* u, const T* v, const T* w, T* nut, double* part,
                                                   int kc, const int* gate) {
  dsm_fused_body<T, YW, ZBC>(xcd_tile(blockIdx, gridDim), gridDim.x, gridDim.y, g, u, v, w, nut, part, kc, gate);
}

// Ducts: c_s per x line (j, k) from the tile partials [k][j][tile x], summed in tile order,
// clipped at zero (0 where <M M> = 0); one thread per line.  gate: as in k_dsm_fused.
__global__ void __launch_bounds__(256) k_dsm_reduce_lines(GridP g, const double* part, int ntx, double* cs,
                                                          const int* gate) {
  if (gate != nullptr && gate[0] == 0) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.nz * g.ny) return;
  double a = 0.0, b = 0.0;
  for (int t = 0; t < ntx; ++t) {
    a += part[((int64_t)e * ntx + t) * 2];
    b += part[((int64_t)e * ntx + t) * 2 + 1];
  }
  cs[e] = b > 0.0 ? fmax(a / b, 0.0) : 0.0;
}

// Ducts: the stored field becomes c_s(j, k) |S| (the plane factor coef[k] = Delta_k^2), the
// ghost planes taking the coefficient of their neighbour plane; one thread per stored cell
// of the interior rows (the ghost rows are refilled afterwards).
template <typename T>
__global__ void __launch_bounds__(256) k_nut_lines(GridP g, T* nut, const double* cs) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nxy = (int64_t)g.nx * g.ny;
  if (e >= (int64_t)(g.nz + 2) * nxy) return;
  const int k = (int)(e / nxy);
  const int64_t r = e % nxy;
  const int j = (int)(r / g.nx);
  const int kk = k < 1 ? 1 : (k > g.nz ? g.nz : k);
  const int64_t c = (int64_t)k * g.sxy + r;
  nut[c] = (T)((double)nut[c] * cs[(int64_t)(kk - 1) * g.ny + j]);
}

// Batched dynamic model (and its plane / volume reduction) over all boxes of a batch.
template <typename T>
__global__ void __launch_bounds__(fused::Tile<T>::NT, fused::Tile<T>::MINB) kb_dsm_fused(BatchMap m) {
  int box;
  const dim3 bid = batch_bid(m, BK_DSM, blockIdx.x, box);
  const BoxDesc& d = m.desc[box];
  dsm_fused_body<T>(bid, d.gdim[BK_DSM][0], d.gdim[BK_DSM][1], d.g, (const T*)d.u, (const T*)d.v, (const T*)d.w,
                    (T*)d.nut, d.dsm_part, d.kc, nullptr);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_dsm_reduce(BatchMap m) {
  int box;
  const dim3 bid = batch_bid(m, BK_DSMRED, blockIdx.x, box);
  const BoxDesc& d = m.desc[box];
  dsm_reduce_body<T>(bid.x, d.g, d.dsm_part, d.gdim[BK_DSM][0] * d.gdim[BK_DSM][1] * fused::Tile<T>::WV, d.cs, d.coef,
                     nullptr, (T*)nullptr);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_strain_mag(BatchMap m) {
  int box;
  const dim3 bid = batch_bid(m, BK_POINT, blockIdx.x, box);
  const BoxDesc& d = m.desc[box];
  const int i = bid.x * blockDim.x + threadIdx.x;
  const int j = bid.y * blockDim.y + threadIdx.y;
  const int k = bid.z + 1;
  if (i >= d.g.nx || j >= d.g.ny) return;
  T s[6];
  centre_strain(d.g, (const T*)d.u, (const T*)d.v, (const T*)d.w, k, j, i, s);
  store_nut(d.g, (T*)d.nut, k, j, i, strain_mag(s));
}

// ============================================================================ learned closure
// Plane sums of the four wall-stress components (bottom x, bottom y, top x, top y) from the
// wall-model stresses or the no-slip viscous flux, WM_BLOCKS blocks over contiguous chunks of
// the plane, each a fixed-order tree; the last block to finish (a ticket counter, cleared
// again by that block) sums the partials by a fixed-order tree and stores the friction velocity of
// each wall, u_tau = sqrt(|(<tau_x>, <tau_y>)|), in dt[2] (bottom) and dt[3] (top).  cnt
// (learned closure, may be null): that block also clears the fallback counters, ahead of the
// inference kernel that adds to them.
constexpr int WM_BLOCKS = 64;

template <typename T>
__global__ void __launch_bounds__(256) k_wall_mean(GridP g, const T* u, const T* v, const double* tau, int wallmodel,
                                                   double* part, double* dtp, int* cnt, unsigned* ticket) {
  __shared__ double sm[4][256];
  __shared__ bool last;
  double a[4] = {0, 0, 0, 0};
  const int64_t s = g.sxy;
  const int n = g.nz;
  const int64_t chunk = (s + WM_BLOCKS - 1) / WM_BLOCKS;
  const int64_t c0 = blockIdx.x * chunk, c1 = c0 + chunk < s ? c0 + chunk : s;
  if (g.zbc != LES_ZBC_PERIODIC)
    for (int64_t c = c0 + threadIdx.x; c < c1; c += 256) {
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
  if (threadIdx.x < 4) {
    part[blockIdx.x * 4 + threadIdx.x] = sm[threadIdx.x][0];
    __threadfence();   // the partial is visible device-wide before the ticket is taken
  }
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(ticket, 1u) == WM_BLOCKS - 1;
  __syncthreads();
  if (!last || threadIdx.x >= 64) return;
  __threadfence();   // the other blocks' partials, published before their tickets
  static_assert(WM_BLOCKS <= 64, "one lane per block partial");
  double w[4];
  for (int q = 0; q < 4; ++q) {   // a fixed-order shuffle tree over the block partials
    double x = threadIdx.x < WM_BLOCKS ? part[threadIdx.x * 4 + q] : 0.0;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    w[q] = x;
  }
  if (threadIdx.x != 0) return;
  const double area = (double)s;
  dtp[2] = sqrt(hypot(w[0] / area, w[1] / area));
  dtp[3] = sqrt(hypot(w[2] / area, w[3] / area));
  if (cnt != nullptr) {
    cnt[0] = 0;
    cnt[1] = 0;
  }
  *ticket = 0u;
}

// Rotation tensor at the cell centre (edges, then the four-edge mean, like the strain),
// with the strain ghost rules (z, and y in a duct): o[0..2] = O12, O13, O23.
template <typename T>
__device__ inline void centre_rotation(const GridP& g, const T* u, const T* v, const T* w, int k, int j, int i,
                                       double o[3]) {
  const int ip = wrap_p(i, g.nx), im = wrap_m(i, g.nx), jp = wrap_p(j, g.nys), jm = wrap_m(j, g.nys);
  const double rdx = g.rdx, rdy = g.rdy, rdzc = 1.0 / g.dzc[k], rdzcm = 1.0 / g.dzc[k - 1];
  auto U = [&](int kk, int jj, int ii) { return (double)sval_y(g, u, kk, jj, ii, true); };
  auto V = [&](int kk, int jj, int ii) { return (double)sval(g, v, kk, jj, ii); };
  auto W = [&](int kk, int jj, int ii) { return (double)sval_y(g, w, kk, jj, ii, false); };
  auto r12 = [&](int jj, int ii) {
    return 0.5 * ((U(k, wrap_p(jj, g.nys), ii) - U(k, jj, ii)) * rdy - (V(k, jj, wrap_p(ii, g.nx)) - V(k, jj, ii)) * rdx);
  };
  o[0] = 0.25 * (r12(j, i) + r12(j, im) + r12(jm, i) + r12(jm, im));
  auto r13 = [&](int kk, int ii, double rz) {
    return 0.5 * ((U(kk + 1, j, ii) - U(kk, j, ii)) * rz - (W(kk, j, wrap_p(ii, g.nx)) - W(kk, j, ii)) * rdx);
  };
  o[1] = 0.25 * (r13(k, i, rdzc) + r13(k, im, rdzc) + r13(k - 1, i, rdzcm) + r13(k - 1, im, rdzcm));
  auto r23 = [&](int kk, int jj, double rz) {
    return 0.5 * ((V(kk + 1, jj, i) - V(kk, jj, i)) * rz - (W(kk, wrap_p(jj, g.nys), i) - W(kk, jj, i)) * rdy);
  };
  o[2] = 0.25 * (r23(k, j, rdzc) + r23(k, jm, rdzc) + r23(k - 1, j, rdzcm) + r23(k - 1, jm, rdzcm));
  (void)ip;
  (void)jp;
}

// The seven raw inputs of the network at a cell (see les.h): invariants of S/n and O/n,
// n = sqrt(S_ij S_ij + O_ij O_ij), then y+ and Delta/delta (delta = 1).
__device__ inline void raw_features(const double s[6], const double o[3], double yplus, double delta, double f[7]) {
  // closed forms for a symmetric S = (s11 s22 s33 s12 s13 s23) and an antisymmetric O with
  // upper entries (o12 o13 o23): P = O^2 (symmetric), Q = S^2 (symmetric)
  const double s11 = s[0], s22 = s[1], s33 = s[2], s12 = s[3], s13 = s[4], s23 = s[5];
  const double o1 = o[0], o2 = o[1], o3 = o[2];
  const double ss = s11 * s11 + s22 * s22 + s33 * s33 + 2.0 * (s12 * s12 + s13 * s13 + s23 * s23);
  const double oo = 2.0 * (o1 * o1 + o2 * o2 + o3 * o3);
  const double nrm = sqrt(ss + oo);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  const double i2 = inv * inv, i3 = i2 * inv, i4 = i2 * i2;
  const double p00 = -(o1 * o1 + o2 * o2), p11 = -(o1 * o1 + o3 * o3), p22 = -(o2 * o2 + o3 * o3);
  const double p01 = -o2 * o3, p02 = o1 * o3, p12 = -o1 * o2;
  const double q00 = s11 * s11 + s12 * s12 + s13 * s13, q11 = s12 * s12 + s22 * s22 + s23 * s23;
  const double q22 = s13 * s13 + s23 * s23 + s33 * s33;
  const double q01 = s11 * s12 + s12 * s22 + s13 * s23, q02 = s11 * s13 + s12 * s23 + s13 * s33;
  const double q12 = s12 * s13 + s22 * s23 + s23 * s33;
  const double s3 = q00 * s11 + q11 * s22 + q22 * s33 + 2.0 * (q01 * s12 + q02 * s13 + q12 * s23);   // tr S^3
  const double ps = p00 * s11 + p11 * s22 + p22 * s33 + 2.0 * (p01 * s12 + p02 * s13 + p12 * s23);   // tr O^2 S
  const double pq = p00 * q00 + p11 * q11 + p22 * q22 + 2.0 * (p01 * q01 + p02 * q02 + p12 * q12);   // tr O^2 S^2
  f[0] = ss * i2;
  f[1] = -oo * i2;
  f[2] = s3 * i3;
  f[3] = ps * i3;
  f[4] = pq * i4;
  f[5] = yplus;
  f[6] = delta;
}

struct MlpNorm {
  double lo[7], inv[7];   // scaled input = (raw - lo) * inv, inv = 1 / (hi - lo)
};

// y+ of cell (k, j): the distance to the nearer z wall in that wall's units (ut[0] bottom,
// ut[1] top); in a duct the smallest d_w u_tau,w over the four walls (ut[2] at y = 0, ut[3]
// at y = ly), the van Driest rule; 0 with periodic z.
__device__ inline double cell_yplus(const GridP& g, int k, int j, const double* ut, double ly) {
  if (g.zbc == LES_ZBC_PERIODIC) return 0.0;
  const double zc = g.zc[k];
  if (g.ywall) {
    const double yc = (j + 0.5) * g.dy;
    return fmin(fmin(zc * ut[0], (g.lz - zc) * ut[1]), fmin(yc * ut[2], (ly - yc) * ut[3])) / g.nu;
  }
  const bool lower = zc <= 0.5 * g.lz;
  return (lower ? zc : g.lz - zc) * (lower ? ut[0] : ut[1]) / g.nu;
}

template <typename T>
__device__ inline void cell_features(const GridP& g, const T* u, const T* v, const T* w, int k, int j, int i,
                                     const double* ut, double ly, double f[7], T s6[6]) {
  centre_strain(g, u, v, w, k, j, i, s6);
  double s[6];
  for (int a = 0; a < 6; ++a) s[a] = (double)s6[a];
  double o[3];
  centre_rotation(g, u, v, w, k, j, i, o);
  raw_features(s, o, cell_yplus(g, k, j, ut, ly), sqrt(g.delta2[k]), f);
}

// Fused inference, z-marching over a chunk of planes per 32 x 8 tile (like the dynamic
// model): the velocity ring of 3 planes on the tile + 1 halo sits in LDS (strain ghost rule
// applied on wall ghost planes).  Per plane each thread forms the velocity-gradient tensor
// of its cell (diagonal at the centre, off-diagonal terms as four-edge means, so S and O are
// its symmetric and antisymmetric parts), the seven scaled inputs, and each wave of 64 cells
// runs the network on the matrix cores.  Stores c |S| with c = max(0, MLP); a cell whose
// scaled inputs leave [-0.05, 1.05] is counted and stores -|S| instead, a mark that
// k_mlp_fallback replaces by the dynamic coefficient of its plane (of its x line in a duct,
// YW) times |S| once the dynamic model of the same state has run (c |S| >= 0 elsewhere).
namespace tiled {
constexpr int TX = 32, TY = 8, NT = TX * TY;
constexpr int RX = TX + 2, RY = TY + 2, N1 = RX * RY;
}  // namespace tiled

template <typename T, bool YW, int ZBC = -1>
__global__ void __launch_bounds__(256, 4) k_mlp_nut(GridP g, const T* __restrict__ u, const T* __restrict__ v,
                                                 const T* __restrict__ w, T* __restrict__ nut,
                                                 const float* __restrict__ P, MlpNorm nm,
                                                 const double* __restrict__ ut, double ly, int* __restrict__ cnt,
                                                 int kc) {
  using namespace mlp;
  using tiled::TX;
  using tiled::TY;
  using tiled::RX;
  using tiled::RY;
  using tiled::N1;
  __shared__ Weights Wt;
  constexpr int XS = 8;   // stored features per cell (7 and a zero): four blocks per CU in FP64
  __shared__ __align__(16) unsigned short xs[WAVES][64 * XS];
  __shared__ T vel[3][3][N1];
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int wave = tid / 64, lane = tid % 64;
  const dim3 bid = xcd_tile(blockIdx, gridDim);
  const int i0 = bid.x * TX, j0 = bid.y * TY;
  const int nz = g.nz;
  const int kb = 1 + bid.z * kc;
  const int ke = min(nz, kb + kc - 1);
  const int zbc = ZBC < 0 ? g.zbc : ZBC;
  const bool per = zbc == LES_ZBC_PERIODIC;
  const bool wm = zbc == LES_ZBC_WALLMODEL;
  load_weights(P, Wt, tid, tiled::NT);
  auto phys = [&](int q) {
    if (!per) return q;
    int m = (q - 1) % nz;
    if (m < 0) m += nz;
    return m + 1;
  };
  auto slot = [](int q) { return ((q % 3) + 3) % 3; };
  // in-plane offsets of the thread's halo points (tiles may exceed the grid: wrap), and the
  // velocity of one plane held in registers from its fetch to its commit to LDS, so that the
  // loads of plane k + 2 overlap the work on plane k (strain ghost rule applied at fetch)
  constexpr int NL = (N1 + tiled::NT - 1) / tiled::NT;
  int lofs[NL];
  int yg[NL];   // ducts: 0, or the offset to the first interior row next to a y ghost row (+-nx)
  for (int r = 0; r < NL; ++r) {
    const int e = tid + r * tiled::NT;
    const int lrow = j0 - 1 + e / RX;
    int ii = (i0 - 1 + e % RX) % g.nx, jj = lrow % g.nys;
    if (ii < 0) ii += g.nx;
    if (jj < 0) jj += g.nys;
    lofs[r] = e < N1 ? jj * g.nx + ii : 0;
    yg[r] = 0;
    if (YW && wm && e < N1 && (lrow == -1 || lrow == g.ny)) {
      // strain ghost of u and w on a y ghost row: 2 a0 - a1 from the two rows next to it
      lofs[r] = (lrow < 0 ? 0 : g.ny - 1) * g.nx + ii;
      yg[r] = lrow < 0 ? g.nx : -g.nx;
    }
  }
  const int64_t sxy = g.sxy;
  // raw unconditional loads (points past the halo read offset 0 and are not committed), so
  // that nothing waits for them before their commit one plane later; the wall model's strain
  // ghosts on the wall ghost planes are formed at the commit from the thread's own LDS entries
  // of the two planes next to the wall
  T ra[NL], rb[NL], rc[NL];
  auto fetch = [&](int q) {
    const int pq = phys(q);
    const PlaneLoader<T> lu(u, pq, sxy), lv(v, pq, sxy), lw(w, pq, sxy);
    for (int r = 0; r < NL; ++r) {
      ra[r] = lu(lofs[r]);
      rb[r] = lv(lofs[r]);
      rc[r] = lw(lofs[r]);
    }
    if (YW) {
      for (int r = 0; r < NL; ++r) {
        if (yg[r] != 0) {
          // lofs points at the interior row next to the ghost row: u and w extrapolated in y
          // (in the z ghost planes these corner values are not used); v is 0 on the wall face
          const T a1 = lu(lofs[r] + yg[r]), c1 = lw(lofs[r] + yg[r]);
          ra[r] = ra[r] - (a1 - ra[r]);
          rc[r] = rc[r] - (c1 - rc[r]);
          rb[r] = (T)0;
        }
      }
    }
  };
  auto commit = [&](int q) {
    const int sl = slot(q);
    const int pq = phys(q);
    if (wm && (pq == 0 || pq == nz + 1)) {
      const bool bot = pq == 0;
      const int s1 = slot(bot ? q + 1 : q - 1), s2 = slot(bot ? q + 2 : q - 2);
      const T ca = (T)ro_load(g.dzc, bot ? 0 : nz), cb = (T)ro_load(g.dzc, bot ? 1 : nz - 1);
      for (int r = 0; r < NL; ++r) {
        const int e = tid + r * tiled::NT;
        if (e < N1 && !(YW && yg[r] != 0)) {
          const T a1 = vel[s1][0][e], a2 = vel[s2][0][e];
          const T b1 = vel[s1][1][e], b2 = vel[s2][1][e];
          ra[r] = bot ? a1 - ca * ((a2 - a1) / cb) : a1 + ca * ((a1 - a2) / cb);
          rb[r] = bot ? b1 - ca * ((b2 - b1) / cb) : b1 + ca * ((b1 - b2) / cb);
        }
      }
    }
    for (int r = 0; r < NL; ++r) {
      const int e = tid + r * tiled::NT;
      if (e < N1) {
        vel[sl][0][e] = ra[r];
        vel[sl][1][e] = rb[r];
        vel[sl][2][e] = rc[r];
      }
    }
  };
  if (wm && kb == 1) {
    // the bottom ghost plane is formed from planes 1 and 2: those are committed first (plane 2
    // is fetched again for the loop's first commit)
    fetch(1);
    commit(1);
    fetch(2);
    commit(2);
    fetch(0);
    commit(0);
    fetch(2);
  } else {
    fetch(kb - 1);
    commit(kb - 1);
    fetch(kb);
    commit(kb);
    fetch(kb + 1);
  }
  int flagged = 0;
  const int i = i0 + tx, j = j0 + ty;
  const bool inside = i < g.nx && j < g.ny;
  // threads exchange data through LDS only: the barriers leave global loads in flight
  for (int k = kb; k <= ke; ++k) {
    commit(k + 1);
    lds_barrier();
    fetch(min(k + 2, ke + 1));   // the last one reloads plane ke + 1 and is not committed
    const int pk = phys(k);
    const int sm = slot(k - 1), s0 = slot(k), sp = slot(k + 1);
    const int x = tx + 1, y = ty + 1;
    auto A = [&](int c, int dz, int dy, int dx) -> T {
      const int sl = dz < 0 ? sm : (dz > 0 ? sp : s0);
      return vel[sl][c][(y + dy) * RX + x + dx];
    };
    const T rdx = (T)g.rdx, rdy = (T)g.rdy, rdzf = (T)ro_load(g.rdzf, pk);
    const T rdzc = (T)ro_load(g.rdzc, pk), rdzcm = (T)ro_load(g.rdzc, pk - 1);
    const T q4 = (T)0.25, h = (T)0.5;
    // velocity-gradient tensor at the centre
    const T a11 = (A(0, 0, 0, 0) - A(0, 0, 0, -1)) * rdx;
    const T a22 = (A(1, 0, 0, 0) - A(1, 0, -1, 0)) * rdy;
    const T a33 = (A(2, 0, 0, 0) - A(2, -1, 0, 0)) * rdzf;
    const T dudy = q4 * (((A(0, 0, 1, 0) - A(0, 0, 0, 0)) + (A(0, 0, 1, -1) - A(0, 0, 0, -1)) +
                          (A(0, 0, 0, 0) - A(0, 0, -1, 0)) + (A(0, 0, 0, -1) - A(0, 0, -1, -1))) * rdy);
    const T dvdx = q4 * (((A(1, 0, 0, 1) - A(1, 0, 0, 0)) + (A(1, 0, 0, 0) - A(1, 0, 0, -1)) +
                          (A(1, 0, -1, 1) - A(1, 0, -1, 0)) + (A(1, 0, -1, 0) - A(1, 0, -1, -1))) * rdx);
    const T dudz = q4 * ((A(0, 1, 0, 0) - A(0, 0, 0, 0)) * rdzc + (A(0, 1, 0, -1) - A(0, 0, 0, -1)) * rdzc +
                         (A(0, 0, 0, 0) - A(0, -1, 0, 0)) * rdzcm + (A(0, 0, 0, -1) - A(0, -1, 0, -1)) * rdzcm);
    const T dwdx = q4 * (((A(2, 0, 0, 1) - A(2, 0, 0, 0)) + (A(2, 0, 0, 0) - A(2, 0, 0, -1)) +
                          (A(2, -1, 0, 1) - A(2, -1, 0, 0)) + (A(2, -1, 0, 0) - A(2, -1, 0, -1))) * rdx);
    const T dvdz = q4 * ((A(1, 1, 0, 0) - A(1, 0, 0, 0)) * rdzc + (A(1, 1, -1, 0) - A(1, 0, -1, 0)) * rdzc +
                         (A(1, 0, 0, 0) - A(1, -1, 0, 0)) * rdzcm + (A(1, 0, -1, 0) - A(1, -1, -1, 0)) * rdzcm);
    const T dwdy = q4 * (((A(2, 0, 1, 0) - A(2, 0, 0, 0)) + (A(2, 0, 0, 0) - A(2, 0, -1, 0)) +
                          (A(2, -1, 1, 0) - A(2, -1, 0, 0)) + (A(2, -1, 0, 0) - A(2, -1, -1, 0))) * rdy);
    T s6[6] = {a11, a22, a33, h * (dudy + dvdx), h * (dudz + dwdx), h * (dvdz + dwdy)};
    const double s[6] = {(double)s6[0], (double)s6[1], (double)s6[2], (double)s6[3], (double)s6[4], (double)s6[5]};
    const double o[3] = {0.5 * ((double)dudy - (double)dvdx), 0.5 * ((double)dudz - (double)dwdx),
                         0.5 * ((double)dvdz - (double)dwdy)};
    double yplus = 0.0;
    if (!per) {
      const double zc = ro_load(g.zc, pk);
      if (YW) {
        const double yc = (j + 0.5) * g.dy;
        yplus = fmin(fmin(zc * ro_load(ut, 0), (g.lz - zc) * ro_load(ut, 1)),
                     fmin(yc * ro_load(ut, 2), (ly - yc) * ro_load(ut, 3))) / g.nu;
      } else {
        const bool lower = zc <= 0.5 * g.lz;
        yplus = (lower ? zc : g.lz - zc) * (lower ? ro_load(ut, 0) : ro_load(ut, 1)) / g.nu;
      }
    }
    double f[7];
    raw_features(s, o, yplus, sqrt(ro_load(g.delta2, pk)), f);
    bool flag = false;
    for (int a = 0; a < 7; ++a) {
      const double xn = (f[a] - nm.lo[a]) * nm.inv[a];
      flag = flag || xn < -0.05 || xn > 1.05;
      f[a] = xn;
    }
    {
      // seven bf16 inputs and a zero as one 16-byte LDS store
      auto pk = [&](int a) -> unsigned int {
        if (!inside) return 0u;
        const fl2 pr = {(float)f[a], a + 1 < F ? (float)f[a + 1] : 0.0f};
        return __builtin_bit_cast(unsigned int, __builtin_convertvector(pr, bf2));
      };
      uint4* dst = reinterpret_cast<uint4*>(&xs[wave][lane * XS]);
      dst[0] = make_uint4(pk(0), pk(2), pk(4), pk(6));
    }
    // each wave reads only its own inputs: LDS operations of a wave complete in order
    __builtin_amdgcn_wave_barrier();
    Fwd out;
    forward_wave<false, XS>(Wt, xs[wave], lane, out);
    const int qq = lane >> 4;
    const float yv = qq == 0 ? out.y[0] : (qq == 1 ? out.y[1] : (qq == 2 ? out.y[2] : out.y[3]));
    if (inside) {
      const T smag = strain_mag(s6);
      const T c = yv > 0.0f ? (T)yv : (T)0;
      if (flag) ++flagged;
      store_nut(g, nut, pk, j, i, flag ? -smag : c * smag);
    }
    lds_barrier();   // the ring slot of plane k - 1 is refilled next
  }
  if (cnt != nullptr) {
    for (int off = 32; off > 0; off >>= 1) flagged += __shfl_down(flagged, off, 64);
    if (lane == 0 && flagged) atomicAdd(&cnt[1], flagged);
  }
}

// Fallback of the learned closure: the cells k_mlp_nut marked (negative stored value -|S|)
// take the dynamic coefficient of their plane (of their x line in a duct) computed from the
// same velocity, c_s |S|, ghost planes included.  Runs only when the current evaluation
// flagged a cell (gate = its counter); one thread per interior cell.
template <typename T>
__global__ void __launch_bounds__(256) k_mlp_fallback(GridP g, T* __restrict__ nut, const double* __restrict__ cs,
                                                      const int* __restrict__ gate) {
  if (gate[0] == 0) return;
  const int64_t nxy = (int64_t)g.nx * g.ny;
  const int64_t ncell = (int64_t)g.nz * nxy;
  // grid-stride: the launch is small, so that it costs little when no cell fell back
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ncell; e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / nxy) + 1;
    const int64_t r = e % nxy;
    const int j = (int)(r / g.nx), i = (int)(r % g.nx);
    const T val = nut[idx3(g, k, j, i)];
    if (!(val < (T)0)) continue;
    const double c = g.ywall ? cs[(int64_t)(k - 1) * g.ny + j] : cs[k - 1];
    store_nut(g, nut, k, j, i, (T)c * -val);
  }
}

// Training pairs: sample s sits at the interior cell hashed from (seed, s) (SplitMix64); x
// gets its seven raw features, y the dynamic coefficient of its plane (of its x line in a
// duct).
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void k_mlp_sample(GridP g, const T* u, const T* v, const T* w, const double* cs, const double* ut,
                             double ly, uint64_t seed, int64_t n, float* x, float* y) {
  const int64_t sidx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (sidx >= n) return;
  const uint64_t nxy = (uint64_t)g.nx * (uint64_t)g.ny;
  const uint64_t ncell = (uint64_t)g.nz * nxy;
  const uint64_t e = splitmix64(seed ^ splitmix64((uint64_t)sidx)) % ncell;
  const int k = (int)(e / nxy) + 1;
  const int64_t r = (int64_t)(e % nxy);
  const int j = (int)(r / g.nx), i = (int)(r % g.nx);
  double f[7];
  T s6[6];
  cell_features(g, u, v, w, k, j, i, ut, ly, f, s6);
  for (int a = 0; a < 7; ++a) x[sidx * 7 + a] = (float)f[a];
  y[sidx] = (float)(g.ywall ? cs[(int64_t)(k - 1) * g.ny + j] : cs[k - 1]);
}

// ============================================================================ launcher
template <typename T>
void launch_eddy_viscosity(Ctx& c) {
  const GridP& g = c.g;
  Launch3 L = point_launch(g, g.nz);
  const int model = c.cfg.sgs;
  if (model == LES_SGS_NONE) return;
  const double pts = (double)g.nx * g.ny * g.nz;
  if (model == LES_SGS_SMAG || model == LES_SGS_SMAG_VD) {
    const bool duct_vd = g.ywall && model == LES_SGS_SMAG_VD;
    if (duct_vd) {
      static_assert(VD_BLOCKS * 8 <= 4096, "partials fit the reduction area");
      LES_LAUNCH(c, "vd_duct", 0, k_vd_duct_partial<T>, dim3(VD_BLOCKS), dim3(256), 0, g, (const T*)c.u,
                 (const T*)c.v, (const T*)c.w, c.t.tau, c.t.tauy, c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0, c.t.red);
      LES_LAUNCH(c, "vd_duct_final", 0, k_vd_duct_final, dim3(1), dim3(64), 0, g, c.t.red, c.t.vd4,
                 (int*)nullptr);
    }
    LES_LAUNCH(c, "strain_mag", 4 * pts * sizeof(T), k_strain_mag<T>, L.grid, L.block, 0, g, (const T*)c.u, (const T*)c.v,
                       (const T*)c.w, (T*)c.nut, duct_vd ? (const double*)c.t.vd4 : nullptr, c.cfg.ly);
    if (model == LES_SGS_SMAG_VD && c.cfg.zbc != LES_ZBC_PERIODIC && !g.ywall) {
      LES_LAUNCH(c, "vd_coef", 0, k_vd_coef_partial<T>, dim3(VD_BLOCKS), dim3(256), 0, g, (const T*)c.u,
                 (const T*)c.v, c.t.tau, c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0, c.t.red);
      LES_LAUNCH(c, "vd_coef_final", 0, k_vd_coef_final, dim3(1), dim3(256), 0, g, c.t.red, c.cfg.cs, c.t.coef);
    }
    return;
  }
  if (model == LES_SGS_DSM || model == LES_SGS_MLP) {
    const bool learned = model == LES_SGS_MLP && c.mlp_params != nullptr;
    // learned closure: the network runs first; the dynamic model of the same velocity runs
    // only if that evaluation flagged a cell (gate = its fallback counter), without storing
    // |S|, and k_mlp_fallback then fills the flagged cells from its coefficients
    const int* gate = learned ? c.mlp_cnt + 1 : nullptr;
    T* dsm_nut = learned ? nullptr : (T*)c.nut;
    const int kc = c.dsm_kc;
    using TL = fused::Tile<T>;
    using TLY = fused::Tile<T, true>;   // ducts
    const int dty = g.ywall ? TLY::TY : TL::TY;
    dim3 grid((g.nx + fused::TX - 1) / fused::TX, (g.ny + dty - 1) / dty, (g.nz + kc - 1) / kc);
    if (learned) {
      MlpNorm nm;
      for (int a = 0; a < 7; ++a) {
        nm.lo[a] = c.mlp_lo[a];
        nm.inv[a] = 1.0 / (c.mlp_hi[a] - c.mlp_lo[a]);
      }
      const int mkc = c.mlp_kc;
      const dim3 tgrid((g.nx + tiled::TX - 1) / tiled::TX, (g.ny + tiled::TY - 1) / tiled::TY, (g.nz + mkc - 1) / mkc);
      if (g.ywall) {
        // ducts: the four walls' friction velocities of the van Driest reduction
        LES_LAUNCH(c, "vd_duct", 0, k_vd_duct_partial<T>, dim3(VD_BLOCKS), dim3(256), 0, g, (const T*)c.u,
                   (const T*)c.v, (const T*)c.w, c.t.tau, c.t.tauy, c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0, c.t.red);
        LES_LAUNCH(c, "vd_duct_final", 0, k_vd_duct_final, dim3(1), dim3(64), 0, g, c.t.red, c.t.vd4, c.mlp_cnt);
        LES_LAUNCH(c, "mlp_nut", 4 * pts * sizeof(T), (k_mlp_nut<T, true>), tgrid, dim3(tiled::TX, tiled::TY), 0, g,
                   (const T*)c.u, (const T*)c.v, (const T*)c.w, (T*)c.nut, c.mlp_params, nm,
                   (const double*)c.t.vd4, c.cfg.ly, c.mlp_cnt, mkc);
      } else {
        LES_LAUNCH(c, "wall_mean", 0, k_wall_mean<T>, dim3(WM_BLOCKS), dim3(256), 0, g, (const T*)c.u,
                   (const T*)c.v, c.t.tau, c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0, c.t.red, c.t.dt, c.mlp_cnt,
                   (unsigned*)(c.mlp_cnt + 2));
        // FP64 with the wall model: the z boundary fixed at compile time (690 -> 677 us on
        // 512x256x128)
        auto km = k_mlp_nut<T, false>;
        if constexpr (sizeof(T) == 8)
          if (g.zbc == LES_ZBC_WALLMODEL) km = k_mlp_nut<T, false, LES_ZBC_WALLMODEL>;
        LES_LAUNCH(c, "mlp_nut", 4 * pts * sizeof(T), km, tgrid, dim3(tiled::TX, tiled::TY), 0, g,
                   (const T*)c.u, (const T*)c.v, (const T*)c.w, (T*)c.nut, c.mlp_params, nm,
                   (const double*)(c.t.dt + 2), c.cfg.ly, c.mlp_cnt, mkc);
      }
    }
    if (g.ywall) {
      // ducts: coefficients along x lines
      // FP64 with the wall model: the z boundary fixed at compile time (no spill; 225 -> 215 us
      // on the 512x80x80 duct)
      auto kfy = k_dsm_fused<T, true>;
      if constexpr (sizeof(T) == 8)
        if (g.zbc == LES_ZBC_WALLMODEL) kfy = k_dsm_fused<T, true, LES_ZBC_WALLMODEL>;
      LES_LAUNCH(c, "dsm_fused", 4 * pts * sizeof(T), kfy, grid, dim3(fused::TX, TLY::TY), 0, g,
                 (const T*)c.u, (const T*)c.v, (const T*)c.w, dsm_nut, c.t.dsm_part, kc, gate);
      const int nl = g.nz * g.ny;
      LES_LAUNCH(c, "dsm_reduce", 0, k_dsm_reduce_lines, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, g,
                 c.t.dsm_part, (int)grid.x, c.t.cs, gate);
      if (!learned) {
        const int64_t ns = (int64_t)(g.nz + 2) * g.nx * g.ny;
        LES_LAUNCH(c, "nut_lines", 2.0 * ns * sizeof(T), k_nut_lines<T>, dim3((unsigned)((ns + 255) / 256)), dim3(256),
                   0, g, (T*)c.nut, (const double*)c.t.cs);
      }
    } else {
      // FP64 channels with walls: the z boundary fixed at compile time (the wall-model build
      // needs 238 VGPRs instead of 255 and ran 674 -> 603 us on 512x256x128; in FP32, and
      // for periodic z, where the fixed builds measured slower, it stays a run-time value)
      auto kf = k_dsm_fused<T, false>;
      if constexpr (sizeof(T) == 8) {
        if (g.zbc == LES_ZBC_WALLMODEL) kf = k_dsm_fused<T, false, LES_ZBC_WALLMODEL>;
        if (g.zbc == LES_ZBC_NOSLIP) kf = k_dsm_fused<T, false, LES_ZBC_NOSLIP>;
      }
      LES_LAUNCH(c, "dsm_fused", 4 * pts * sizeof(T), kf, grid, dim3(fused::TX, TL::TY), 0, g,
                 (const T*)c.u, (const T*)c.v, (const T*)c.w, dsm_nut, c.t.dsm_part, kc, gate);
      const int ntile = (int)(grid.x * grid.y) * TL::WV;
      LES_LAUNCH(c, "dsm_reduce", 0, k_dsm_reduce<T>, dim3(g.nz), dim3(256), 0, g, c.t.dsm_part, ntile, c.t.cs,
                 learned ? nullptr : c.t.coef, gate, learned ? (T*)c.nut : (T*)nullptr);
    }
    if (learned && g.ywall) {   // channels: the fallback ran with the plane coefficients
      const int64_t ni = (int64_t)g.nz * g.nx * g.ny;
      LES_LAUNCH(c, "mlp_fallback", 0, k_mlp_fallback<T>, dim3((unsigned)std::min<int64_t>(1024, (ni + 255) / 256)),
                 dim3(256), 0, g,
                 (T*)c.nut, (const double*)c.t.cs, (const int*)gate);
    }
  }
}

template <typename T>
void batch_eddy_viscosity(hipStream_t st, const BatchMap& m, const int* totals, int any_dsm, int any_smag) {
  if (any_smag) hipLaunchKernelGGL(kb_strain_mag<T>, dim3(totals[BK_POINT]), dim3(32, 8), 0, st, m);
  if (any_dsm) {
    hipLaunchKernelGGL(kb_dsm_fused<T>, dim3(totals[BK_DSM]), dim3(fused::TX, fused::Tile<T>::TY), 0, st, m);
    hipLaunchKernelGGL(kb_dsm_reduce<T>, dim3(totals[BK_DSMRED]), dim3(256), 0, st, m);
  }
}
template void batch_eddy_viscosity<float>(hipStream_t, const BatchMap&, const int*, int, int);
template void batch_eddy_viscosity<double>(hipStream_t, const BatchMap&, const int*, int, int);

template <typename T>
void launch_mlp_sample(Ctx& c, uint64_t seed, int64_t n, float* x, float* y) {
  const GridP& g = c.g;
  const int wm = c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0;
  const double* ut = c.t.dt + 2;
  if (g.ywall) {
    LES_LAUNCH(c, "vd_duct", 0, k_vd_duct_partial<T>, dim3(VD_BLOCKS), dim3(256), 0, g, (const T*)c.u, (const T*)c.v,
               (const T*)c.w, c.t.tau, c.t.tauy, wm, c.t.red);
    LES_LAUNCH(c, "vd_duct_final", 0, k_vd_duct_final, dim3(1), dim3(64), 0, g, c.t.red, c.t.vd4,
                 (int*)nullptr);
    ut = c.t.vd4;
  } else {
    LES_LAUNCH(c, "wall_mean", 0, k_wall_mean<T>, dim3(WM_BLOCKS), dim3(256), 0, g, (const T*)c.u,
               (const T*)c.v, c.t.tau, wm, c.t.red, c.t.dt, (int*)nullptr, (unsigned*)(c.mlp_cnt + 2));
  }
  LES_LAUNCH(c, "mlp_sample", 0, k_mlp_sample<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, g, (const T*)c.u,
             (const T*)c.v, (const T*)c.w, c.t.cs, ut, c.cfg.ly, seed, n, x, y);
}
template void launch_mlp_sample<double>(Ctx&, uint64_t, int64_t, float*, float*);
template void launch_mlp_sample<float>(Ctx&, uint64_t, int64_t, float*, float*);

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
