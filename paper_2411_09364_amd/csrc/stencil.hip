// Momentum predictor, Crank-Nicolson z solves, projection, boundary planes, wall model
// and time step: the point-wise and column-wise parts of one RK3 substep
// (Alg. 1; Eqs. onestar_exp, twostar_imp1d, onestar_imp1d, correc, p_update_exp,
// p_update_imp1d; Eq. wm with the coupling of Sec. 2.2; Alg. 2).
#include "les_internal.h"

#include <type_traits>

namespace les {

constexpr int kMaxNz = 512;   // largest wall-bounded nz accepted by les_init

__device__ void helmholtz_factor_body(const GridP& g, double* hfac, const double* dtp, double gamma, int wallmodel,
                                      double* dzf, double* dzc, int tid, int nthr);

Launch3 point_launch(const GridP& g, int planes) {
  Launch3 L;
  int bx = g.nx >= 64 ? 64 : g.nx;
  int by = 256 / bx;
  if (by > g.ny) by = g.ny;
  L.block = dim3(bx, by, 1);
  L.grid = dim3((g.nx + bx - 1) / bx, (g.ny + by - 1) / by, planes);
  return L;
}

// 32 x 8 tiles for the stencil sweeps (a wave covers two 256-byte rows in FP64).
Launch3 tile_launch(const GridP& g, int planes) {
  Launch3 L;
  int bx, by;
  tile_shape(g.nx, g.ny, bx, by);
  L.block = dim3(bx, by, 1);
  L.grid = dim3((g.nx + bx - 1) / bx, (g.ny + by - 1) / by, planes);
  return L;
}

// nu_t at a cell centre: plane coefficient times the stored field.
template <typename T>
__device__ inline T nut_at(const T* nut, const double* coef, const GridP& g, int k, int j, int i) {
  return (T)coef[k] * nut[idx3(g, k, j, i)];
}

// ============================================================================ predictor
// Neighbourhood of one cell used by the momentum right-hand side.  Suffixes give the offset:
// ip/im = i +- 1, jp/jm = j +- 1, kp/km = k +- 1 (u, v, w at their faces; n = nu_t and p at
// centres).
template <typename T>
struct Nb {
  T u0, uip, uim, ujp, ujm, ukp, ukm, ujp_im, ukp_im;
  T v0, vip, vim, vjp, vjm, vkp, vkm, vjm_ip, vkp_jm;
  T w0, wip, wim, wjp, wjm, wkp, wkm, wkm_ip, wkm_jp;
  T n0, nip, nim, njp, njm, nkp, nkm, n_jp_ip, n_jm_ip, n_kp_ip, n_km_ip, n_jp_im, n_kp_jp, n_km_jp, n_kp_im, n_kp_jm;
  T p0, pip, pjp, pkp;
};

// Viscous treatment of the predictor: explicit (Eq. onestar_exp), Crank-Nicolson in z
// (Eq. twostar_imp1d) or in all directions (Eq. twostar_imp3d).
enum { VISC_EXPLICIT = LES_VISC_EXPLICIT, VISC_CN_Z = LES_VISC_CN_Z, VISC_CN_3D = LES_VISC_CN_3D };

// R_i = -d(u_i u_j)/dx_j + d(2 nu_t S_ij)/dx_j + nu L u_i (explicit), with L_xx + L_yy only
// (CN in z) or without viscous part (CN in all directions); u* = u + dt (alpha R^k +
// beta R^{k-1} - gamma G p), or the Helmholtz right-hand side u** - gamma nu dt/2 L' u^k with
// u** = u + dt (alpha R^k + beta R^{k-1} - gamma G p) + gamma nu dt L' u^k, L' = L_zz (CN in
// z) or the full Laplacian (CN in all directions).
// One cell (plane k) from its neighbourhood b and, when use_rprev, R^{k-1} (rup, rvp, rwp).
template <typename T, int MODE>
__device__ __forceinline__ void predictor_cell(const Nb<T>& b, const GridP& g, int k, T dt, double alpha,
                                               double beta, double gamma, bool use_rprev, T rup, T rvp, T rwp,
                                               T& Ru_out, T& Rv_out, T& Rw_out, T& uo, T& vo, T& wo) {
  // fused multiply-adds only where an expression asks for one, so that every kernel that
  // inlines this function rounds identically
#pragma clang fp contract(on)
  const int kp = k + 1, km = k - 1;
  const T rdx = (T)g.rdx, rdy = (T)g.rdy;
  const T rdzf = (T)ro_load(g.rdzf, k);
  const T rdzc = (T)ro_load(g.rdzc, k);
  const T rdzcm = (T)ro_load(g.rdzc, km);
  const T rdzfp = (T)ro_load(g.rdzf, kp);
  const T nu = (T)g.nu;
  const T h = (T)0.5, q = (T)0.25, two = (T)2;
  // ---------------- u-momentum at (i+1/2, j, k)
  T ax, ay, az, sx, sy, sz, lx, lz;
  {
    const T fxx_r = (h * (b.u0 + b.uip)) * (h * (b.u0 + b.uip));
    const T fxx_l = (h * (b.uim + b.u0)) * (h * (b.uim + b.u0));
    const T fxy_t = h * (b.u0 + b.ujp) * (h * (b.v0 + b.vip));
    const T fxy_b = h * (b.ujm + b.u0) * (h * (b.vjm + b.vjm_ip));
    const T fxz_t = h * (b.u0 + b.ukp) * (h * (b.w0 + b.wip));
    const T fxz_b = h * (b.ukm + b.u0) * (h * (b.wkm + b.wkm_ip));
    ax = (fxx_r - fxx_l) * rdx + (fxy_t - fxy_b) * rdy + (fxz_t - fxz_b) * rdzf;
    // SGS
    const T t11_r = two * b.nip * ((b.uip - b.u0) * rdx);
    const T t11_l = two * b.n0 * ((b.u0 - b.uim) * rdx);
    const T nu12_t = q * (b.n0 + b.nip + b.njp + b.n_jp_ip);
    const T e12_t = h * ((b.ujp - b.u0) * rdy + (b.vip - b.v0) * rdx);
    const T nu12_b = q * (b.njm + b.n_jm_ip + b.n0 + b.nip);
    const T e12_b = h * ((b.u0 - b.ujm) * rdy + (b.vjm_ip - b.vjm) * rdx);
    const T nu13_t = q * (b.n0 + b.nip + b.nkp + b.n_kp_ip);
    const T e13_t = h * ((b.ukp - b.u0) * rdzc + (b.wip - b.w0) * rdx);
    const T nu13_b = q * (b.nkm + b.n_km_ip + b.n0 + b.nip);
    const T e13_b = h * ((b.u0 - b.ukm) * rdzcm + (b.wkm_ip - b.wkm) * rdx);
    sx = (t11_r - t11_l) * rdx + (two * nu12_t * e12_t - two * nu12_b * e12_b) * rdy +
         (two * nu13_t * e13_t - two * nu13_b * e13_b) * rdzf;
    lx = (b.uip - two * b.u0 + b.uim) * (rdx * rdx) + (b.ujp - two * b.u0 + b.ujm) * (rdy * rdy);
    lz = ((b.ukp - b.u0) * rdzc - (b.u0 - b.ukm) * rdzcm) * rdzf;
  }
  const T lzu = lz;
  const T lxu = lx;
  T Ru = -ax + sx + nu * (MODE == VISC_EXPLICIT ? lx + lz : (MODE == VISC_CN_Z ? lx : (T)0));
  // ---------------- v-momentum at (i, j+1/2, k)
  {
    const T fyx_r = h * (b.v0 + b.vip) * (h * (b.u0 + b.ujp));
    const T fyx_l = h * (b.vim + b.v0) * (h * (b.uim + b.ujp_im));
    const T fyy_t = (h * (b.v0 + b.vjp)) * (h * (b.v0 + b.vjp));
    const T fyy_b = (h * (b.vjm + b.v0)) * (h * (b.vjm + b.v0));
    const T fyz_t = h * (b.v0 + b.vkp) * (h * (b.w0 + b.wjp));
    const T fyz_b = h * (b.vkm + b.v0) * (h * (b.wkm + b.wkm_jp));
    ay = (fyx_r - fyx_l) * rdx + (fyy_t - fyy_b) * rdy + (fyz_t - fyz_b) * rdzf;
    const T nu12_r = q * (b.n0 + b.nip + b.njp + b.n_jp_ip);
    const T e12_r = h * ((b.ujp - b.u0) * rdy + (b.vip - b.v0) * rdx);
    const T nu12_l = q * (b.nim + b.n0 + b.n_jp_im + b.njp);
    const T e12_l = h * ((b.ujp_im - b.uim) * rdy + (b.v0 - b.vim) * rdx);
    const T t22_t = two * b.njp * ((b.vjp - b.v0) * rdy);
    const T t22_b = two * b.n0 * ((b.v0 - b.vjm) * rdy);
    const T nu23_t = q * (b.n0 + b.njp + b.nkp + b.n_kp_jp);
    const T e23_t = h * ((b.vkp - b.v0) * rdzc + (b.wjp - b.w0) * rdy);
    const T nu23_b = q * (b.nkm + b.n_km_jp + b.n0 + b.njp);
    const T e23_b = h * ((b.v0 - b.vkm) * rdzcm + (b.wkm_jp - b.wkm) * rdy);
    sy = (two * nu12_r * e12_r - two * nu12_l * e12_l) * rdx + (t22_t - t22_b) * rdy +
         (two * nu23_t * e23_t - two * nu23_b * e23_b) * rdzf;
    lx = (b.vip - two * b.v0 + b.vim) * (rdx * rdx) + (b.vjp - two * b.v0 + b.vjm) * (rdy * rdy);
    lz = ((b.vkp - b.v0) * rdzc - (b.v0 - b.vkm) * rdzcm) * rdzf;
  }
  const T lzv = lz;
  const T lxv = lx;
  T Rv = -ay + sy + nu * (MODE == VISC_EXPLICIT ? lx + lz : (MODE == VISC_CN_Z ? lx : (T)0));
  // ---------------- w-momentum at (i, j, k+1/2)
  {
    const T fzx_r = h * (b.w0 + b.wip) * (h * (b.u0 + b.ukp));
    const T fzx_l = h * (b.wim + b.w0) * (h * (b.uim + b.ukp_im));
    const T fzy_t = h * (b.w0 + b.wjp) * (h * (b.v0 + b.vkp));
    const T fzy_b = h * (b.wjm + b.w0) * (h * (b.vjm + b.vkp_jm));
    const T fzz_t = (h * (b.w0 + b.wkp)) * (h * (b.w0 + b.wkp));
    const T fzz_b = (h * (b.wkm + b.w0)) * (h * (b.wkm + b.w0));
    az = (fzx_r - fzx_l) * rdx + (fzy_t - fzy_b) * rdy + (fzz_t - fzz_b) * rdzc;
    const T nu13_r = q * (b.n0 + b.nip + b.nkp + b.n_kp_ip);
    const T e13_r = h * ((b.ukp - b.u0) * rdzc + (b.wip - b.w0) * rdx);
    const T nu13_l = q * (b.nim + b.n0 + b.n_kp_im + b.nkp);
    const T e13_l = h * ((b.ukp_im - b.uim) * rdzc + (b.w0 - b.wim) * rdx);
    const T nu23_r = q * (b.n0 + b.njp + b.nkp + b.n_kp_jp);
    const T e23_r = h * ((b.vkp - b.v0) * rdzc + (b.wjp - b.w0) * rdy);
    const T nu23_l = q * (b.njm + b.n0 + b.n_kp_jm + b.nkp);
    const T e23_l = h * ((b.vkp_jm - b.vjm) * rdzc + (b.w0 - b.wjm) * rdy);
    const T t33_t = two * b.nkp * ((b.wkp - b.w0) * rdzfp);
    const T t33_b = two * b.n0 * ((b.w0 - b.wkm) * rdzf);
    sz = (two * nu13_r * e13_r - two * nu13_l * e13_l) * rdx + (two * nu23_r * e23_r - two * nu23_l * e23_l) * rdy +
         (t33_t - t33_b) * rdzc;
    lx = (b.wip - two * b.w0 + b.wim) * (rdx * rdx) + (b.wjp - two * b.w0 + b.wjm) * (rdy * rdy);
    lz = ((b.wkp - b.w0) * rdzfp - (b.w0 - b.wkm) * rdzf) * rdzc;
  }
  const T lzw = lz;
  const T lxw = lx;
  T Rw = -az + sz + nu * (MODE == VISC_EXPLICIT ? lx + lz : (MODE == VISC_CN_Z ? lx : (T)0));
  const T ta = (T)alpha, tb = (T)beta, tg = (T)gamma;
  T iu = ta * Ru, iv = ta * Rv, iw = ta * Rw;
  if (use_rprev) {
    iu = iu + tb * rup;
    iv = iv + tb * rvp;
    iw = iw + tb * rwp;
  }
  iu = iu - tg * ((b.pip - b.p0) * rdx);
  iv = iv - tg * ((b.pjp - b.p0) * rdy);
  iw = iw - tg * ((b.pkp - b.p0) * rdzc);
  Ru_out = Ru;
  Rv_out = Rv;
  Rw_out = Rw;
  const bool wall_face = (g.zbc != LES_ZBC_PERIODIC) && (k == g.nz);
  if (MODE == VISC_CN_Z) {
    const T cg = tg * nu, ch = tg * nu * dt / two;
    uo = (b.u0 + dt * (iu + cg * lzu)) - ch * lzu;
    vo = (b.v0 + dt * (iv + cg * lzv)) - ch * lzv;
    wo = wall_face ? (T)0 : (b.w0 + dt * (iw + cg * lzw)) - ch * lzw;
  } else if (MODE == VISC_CN_3D) {
    const T cg = tg * nu, ch = tg * nu * dt / two;
    const T lu = lxu + lzu, lv = lxv + lzv, lw = lxw + lzw;
    uo = (b.u0 + dt * (iu + cg * lu)) - ch * lu;
    vo = (b.v0 + dt * (iv + cg * lv)) - ch * lv;
    wo = wall_face ? (T)0 : (b.w0 + dt * (iw + cg * lw)) - ch * lw;
  } else {
    uo = b.u0 + dt * iu;
    vo = b.v0 + dt * iv;
    wo = wall_face ? (T)0 : b.w0 + dt * iw;
  }
}

// z-marching predictor: a 32 x TY tile walks a chunk of kc planes.  A ring of three planes of
// u, v, w, nu_t (coefficient applied) and p on the tile + 1 halo sits in LDS; the loads of
// plane k + 2 are issued right after plane k + 1 is committed and complete under the work
// on plane k.  With CN in z the first z slice of blocks holds the block that factorises the
// substep's Helmholtz matrices (the others of that slice return at once), unless a launch of
// its own has done so.  TY = 16 (FP64): one 512-thread block per CU, the halo a smaller share
// of the loads (18 / 16 rows against 10 / 8); TY = 8: three (FP64) or four (FP32) blocks per CU.
namespace zmarch {
constexpr int TX = 32;
template <int TY_>
struct Tile {
  static constexpr int TY = TY_, NT = TX * TY;
  static constexpr int RX = TX + 2, RY = TY + 2, N1 = RX * RY, NL = (N1 + NT - 1) / NT;
};
}  // namespace zmarch

// RW: bit 0 reads R^{k-1} (substeps 1, 2), bit 1 writes R^k (substeps 0, 1); compile-time so
// that the loop holds no branch around a global load or store.
template <typename T, int MODE, int RW, int TY>
__device__ __forceinline__ void predictor_zm_body(dim3 bid, const GridP& g, const T* __restrict__ u,
                                                  const T* __restrict__ v, const T* __restrict__ w,
                                                  const T* __restrict__ p, const T* __restrict__ nut,
                                                  const double* __restrict__ coef, T* __restrict__ ru,
                                                  T* __restrict__ rv, T* __restrict__ rw, T* __restrict__ us,
                                                  T* __restrict__ vs, T* __restrict__ ws,
                                                  const double* __restrict__ dtp, double alpha, double beta,
                                                  double gamma, int kc, int chunk,
                                                  const double* __restrict__ tau, int wallmodel,
                                                  const double* __restrict__ hfw,
                                                  T (&ring)[3][5][zmarch::Tile<TY>::N1]) {
  // ring: [plane slot][u v w nu p][tile + 1 halo]
  using ZT = zmarch::Tile<TY>;
  constexpr int TX = zmarch::TX, NT = ZT::NT, RX = ZT::RX, N1 = ZT::N1, NL = ZT::NL;
  constexpr bool use_rprev = (RW & 1) != 0, write_r = (RW & 2) != 0;
  // CN in z: the thread's running elimination values of u, v, w, kept in LDS
  __shared__ double ecar[MODE == VISC_CN_Z ? 3 : 1][NT];
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int i0 = bid.x * TX, j0 = bid.y * TY;
  const int kb = 1 + chunk * kc;
  const int ke = min(g.nz, kb + kc - 1);
  const int64_t sxy = g.sxy;
  int lofs[NL];
  for (int r = 0; r < NL; ++r) {
    const int e = tid + r * NT;
    // rows wrap over the stored rows: a duct's ghost rows sit where j = -1 and j = ny land
    int ii = (i0 - 1 + e % RX) % g.nx, jj = (j0 - 1 + e / RX) % g.nys;
    if (ii < 0) ii += g.nx;
    if (jj < 0) jj += g.nys;
    lofs[r] = e < N1 ? jj * g.nx + ii : 0;
  }
  // Raw loads only, issued unconditionally (points beyond the halo read the plane's first
  // value and are not committed), so that nothing waits for them before the commit one plane
  // later; the plane coefficient of nu_t is applied at the commit.
  T rg[NL][5];
  auto fetch = [&](int q) {   // planes 0 .. nz+1 are stored (ghosts included)
    const PlaneLoader<T> lu(u, q, sxy), lv(v, q, sxy), lw(w, q, sxy), ln(nut, q, sxy), lp(p, q, sxy);
    for (int r = 0; r < NL; ++r) {
      rg[r][0] = lu(lofs[r]);
      rg[r][1] = lv(lofs[r]);
      rg[r][2] = lw(lofs[r]);
      rg[r][3] = ln(lofs[r]);
      rg[r][4] = lp(lofs[r]);
    }
  };
  auto commit = [&](int q) {
    const int sl = q % 3;
    const T cq = (T)ro_load(coef, q);
    for (int r = 0; r < NL; ++r) {
      const int e = tid + r * NT;
      if (e < N1) {
        ring[sl][0][e] = rg[r][0];
        ring[sl][1][e] = rg[r][1];
        ring[sl][2][e] = rg[r][2];
        ring[sl][3][e] = cq * rg[r][3];
        ring[sl][4][e] = rg[r][4];
      }
    }
  };
  fetch(kb - 1);
  commit(kb - 1);
  fetch(kb);
  commit(kb);
  fetch(kb + 1);
  const int i = i0 + tx, j = j0 + ty;
  const bool inside = i < g.nx && j < g.ny;
  const T dt = (T)ro_load(dtp, 0);
  // R_prev of the own cell, loaded one plane ahead and unconditionally within the substep:
  // the plane after the chunk reads the chunk's last plane (not used), threads outside the
  // grid read the ghost plane 0, which no thread writes
  T rpn[3] = {(T)0, (T)0, (T)0};
  const int64_t rcell = inside ? (int64_t)j * g.nx + i : -1;
  auto fetch_r = [&](int k) {
    if constexpr (use_rprev) {
      const int64_t c = rcell < 0 ? 0 : (int64_t)min(k, ke) * sxy + rcell;
      rpn[0] = ru[c];
      rpn[1] = rv[c];
      rpn[2] = rw[c];
    }
  };
  fetch_r(kb);
  // CN in z with walls (FP64): the forward elimination of the z systems runs here, along the
  // march, from a zero start at the chunk's first row (the back substitution adds the
  // contribution of the rows below the chunk)
  if constexpr (MODE == VISC_CN_Z) {
    ecar[0][tid] = 0.0;
    ecar[1][tid] = 0.0;
    ecar[2][tid] = 0.0;
  }
  for (int k = kb; k <= ke; ++k) {
    commit(k + 1);
    // the ring is the only data threads exchange: global loads in flight stay in flight
    lds_barrier();
    fetch(min(k + 2, ke + 1));   // past the chunk: a plane that exists, not committed
    const T rup = rpn[0], rvp = rpn[1], rwp = rpn[2];
    if (inside) {
      const int sm = (k - 1) % 3, s0 = k % 3, sp = (k + 1) % 3;
      const int x = tx + 1, y = ty + 1;
      auto A = [&](int f, int sl, int dy, int dx) -> T { return ring[sl][f][(y + dy) * RX + x + dx]; };
      Nb<T> b;
      b.u0 = A(0, s0, 0, 0), b.uip = A(0, s0, 0, 1), b.uim = A(0, s0, 0, -1), b.ujp = A(0, s0, 1, 0);
      b.ujm = A(0, s0, -1, 0), b.ukp = A(0, sp, 0, 0), b.ukm = A(0, sm, 0, 0), b.ujp_im = A(0, s0, 1, -1);
      b.ukp_im = A(0, sp, 0, -1);
      b.v0 = A(1, s0, 0, 0), b.vip = A(1, s0, 0, 1), b.vim = A(1, s0, 0, -1), b.vjp = A(1, s0, 1, 0);
      b.vjm = A(1, s0, -1, 0), b.vkp = A(1, sp, 0, 0), b.vkm = A(1, sm, 0, 0), b.vjm_ip = A(1, s0, -1, 1);
      b.vkp_jm = A(1, sp, -1, 0);
      b.w0 = A(2, s0, 0, 0), b.wip = A(2, s0, 0, 1), b.wim = A(2, s0, 0, -1), b.wjp = A(2, s0, 1, 0);
      b.wjm = A(2, s0, -1, 0), b.wkp = A(2, sp, 0, 0), b.wkm = A(2, sm, 0, 0), b.wkm_ip = A(2, sm, 0, 1);
      b.wkm_jp = A(2, sm, 1, 0);
      b.n0 = A(3, s0, 0, 0), b.nip = A(3, s0, 0, 1), b.nim = A(3, s0, 0, -1), b.njp = A(3, s0, 1, 0);
      b.njm = A(3, s0, -1, 0), b.nkp = A(3, sp, 0, 0), b.nkm = A(3, sm, 0, 0);
      b.n_jp_ip = A(3, s0, 1, 1), b.n_jm_ip = A(3, s0, -1, 1), b.n_kp_ip = A(3, sp, 0, 1), b.n_km_ip = A(3, sm, 0, 1);
      b.n_jp_im = A(3, s0, 1, -1), b.n_kp_jp = A(3, sp, 1, 0), b.n_km_jp = A(3, sm, 1, 0), b.n_kp_im = A(3, sp, 0, -1);
      b.n_kp_jm = A(3, sp, -1, 0);
      b.p0 = A(4, s0, 0, 0), b.pip = A(4, s0, 0, 1), b.pjp = A(4, s0, 1, 0), b.pkp = A(4, sp, 0, 0);
      const int64_t c0 = idx3(g, k, j, i);
      T Ru, Rv, Rw, uo, vo, wo;
      predictor_cell<T, MODE>(b, g, k, dt, alpha, beta, gamma, use_rprev, rup, rvp, rwp, Ru, Rv, Rw, uo, vo,
                              wo);
      if (MODE == VISC_CN_3D && wallmodel && (k == 1 || k == g.nz)) {
        // wall-model rows: the lagged wall stress enters as a known flux (as in CN in z)
        const double ch = gamma * g.nu * ro_load(dtp, 0) / 2.0;
        const int64_t cj = (int64_t)j * g.nx + i;
        const int b0 = k == 1 ? 0 : 2;
        const double rz = 1.0 / g.dzf[k];
        uo = (T)((double)uo + ch * (-(tau[b0 * sxy + cj] / g.nu) * rz));
        vo = (T)((double)vo + ch * (-(tau[(b0 + 1) * sxy + cj] / g.nu) * rz));
      }
      if constexpr (MODE == VISC_CN_Z) {
        if (hfw != nullptr) {
          double fu = (double)uo, fv = (double)vo;
          if (wallmodel && (k == 1 || k == g.nz)) {
            // wall-model rows: the lagged wall stress enters as a known flux
            const double ch = gamma * g.nu * ro_load(dtp, 0) / 2.0;
            const int64_t cj = (int64_t)j * g.nx + i;
            const int b0 = k == 1 ? 0 : 2;
            const double dz = ro_load(g.dzf, k);
            fu += ch * (-(tau[b0 * sxy + cj] / g.nu) / dz);
            fv += ch * (-(tau[(b0 + 1) * sxy + cj] / g.nu) / dz);
          }
          const int n = g.nz, r = k - 1;
          const double eu = (fu - ro_load(hfw, 6 * n + r) * ecar[0][tid]) * ro_load(hfw, n + r);
          const double ev = (fv - ro_load(hfw, 6 * n + r) * ecar[1][tid]) * ro_load(hfw, n + r);
          ecar[0][tid] = eu;
          ecar[1][tid] = ev;
          uo = (T)eu;
          vo = (T)ev;
          if (k < n) {   // w rows: the faces 1 .. nz - 1
            const double ew = ((double)wo - ro_load(hfw, 7 * n + r) * ecar[2][tid]) * ro_load(hfw, 3 * n + r);
            ecar[2][tid] = ew;
            wo = (T)ew;
          }
        }
      }
      if constexpr (write_r) {
        ru[c0] = Ru;
        rv[c0] = Rv;
        rw[c0] = Rw;
      }
      us[c0] = uo;
      vs[c0] = (g.ywall && j == g.ny - 1) ? (T)0 : vo;   // v on the duct's wall face y = ly
      ws[c0] = wo;
    }
    fetch_r(k + 1);   // after this plane's use of rpn: no copy waits for the loads
    lds_barrier();    // the ring slot of plane k - 1 is refilled next
  }
}

template <typename T, int MODE, int RW, int TY>
__global__ void __launch_bounds__(32 * TY, TY == 16 ? (sizeof(T) == 8 ? 1 : 2) : (sizeof(T) == 8 ? 3 : 4)) k_predictor(GridP g, const T* __restrict__ u,
                                                                        const T* __restrict__ v,
                                                                        const T* __restrict__ w,
                                                                        const T* __restrict__ p,
                                                                        const T* __restrict__ nut,
                                                                        const double* __restrict__ coef,
                                                                        T* __restrict__ ru, T* __restrict__ rv,
                                                                        T* __restrict__ rw, T* __restrict__ us,
                                                                        T* __restrict__ vs, T* __restrict__ ws,
                                                                        const double* __restrict__ dtp,
                                                                        double alpha, double beta, double gamma,
                                                                        double* hfac,
                                                                        int wallmodel, int kc,
                                                                        const double* __restrict__ tau, int fslice,
                                                                        const double* __restrict__ hfw) {
  const dim3 bid = xcd_tile(blockIdx, gridDim);
  __shared__ T ring[3][5][zmarch::Tile<TY>::N1];
  static_assert(sizeof(ring) >= 2 * (kMaxNz + 2) * sizeof(double), "factorisation scratch");
  if (MODE != VISC_EXPLICIT && fslice && bid.z == 0) {
    // metric copies of the factorisation in the ring's memory
    double* fz = reinterpret_cast<double*>(&ring[0][0][0]);
    if (bid.x == 0 && bid.y == 0)
      helmholtz_factor_body(g, hfac, dtp, gamma, wallmodel, fz, fz + kMaxNz + 2,
                            threadIdx.y * blockDim.x + threadIdx.x, blockDim.x * blockDim.y);
    return;
  }
  predictor_zm_body<T, MODE, RW, TY>(bid, g, u, v, w, p, nut, coef, ru, rv, rw, us, vs, ws, dtp, alpha, beta,
                                     gamma, kc, (int)bid.z - fslice, tau, wallmodel, hfw, ring);
}

// Batched predictor (explicit viscous terms): one launch over all boxes of a batch, the same
// z-marching body per box.
template <typename T, int RW>
__global__ void __launch_bounds__(256, sizeof(T) == 8 ? 2 : 4) kb_predictor(BatchMap m, double alpha, double beta,
                                                                         double gamma) {
  int box;
  const dim3 bid = batch_bid(m, BK_PRED, blockIdx.x, box);
  const BoxDesc& d = m.desc[box];
  __shared__ T ring[3][5][zmarch::Tile<8>::N1];
  predictor_zm_body<T, VISC_EXPLICIT, RW, 8>(bid, d.g, (const T*)d.u, (const T*)d.v, (const T*)d.w,
                                          (const T*)d.p, (const T*)d.nut, d.coef, (T*)d.ru, (T*)d.rv, (T*)d.rw,
                                          (T*)d.us, (T*)d.vs, (T*)d.wsf, d.dt, alpha, beta, gamma, d.pkc, (int)bid.z,
                                          nullptr, 0, nullptr, ring);
}

// CN in z with walls, FP64: the predictor eliminates along its z march and a streaming
// kernel substitutes back (the z chunks of the march fixed up through the products of the
// elimination's row multipliers); the chunk corrections are held per thread for at most
// HZ_MAXCH chunks.  Otherwise the staged solve below runs after the predictor.
constexpr int HZ_MAXCH = 8;
template <typename T>
bool hz_fused(const Ctx& c) {
  return sizeof(T) == 8 && c.cfg.implicit_z == VISC_CN_Z && c.cfg.zbc != LES_ZBC_PERIODIC &&
         (c.g.nz + c.pred_kc - 1) / c.pred_kc <= HZ_MAXCH;
}

// Factorisation of the substep's z systems in one block of 1024 threads, ahead of the
// predictor: one thread per row (u/v rows on threads 0..511, w rows on 512..1023), with the
// recurrences of the Thomas factorisation taken as prefix scans (Hillis-Steele, log2 nz
// levels):
//   pivots p_k = b_k - a_k c_{k-1} / p_{k-1}: the ratio x_k / y_k of the first column of the
//     product M_k ... M_0, M_k = [[b_k, -a_k c_{k-1}], [1, 0]] (each partial product rescaled
//     by a power of two, which leaves the ratio unchanged);
//   products pp_k of the elimination's row multipliers -a_j r_j from the first row of each
//     chunk of kc rows (the weight of the value below a chunk in each eliminated row);
//   flow-rate profile q = H^-1 1 of the u rows (no-slip walls; 1 otherwise): forward
//     d_k = r_k - a_k r_k d_{k-1}, back q_k = d_k - c'_k q_{k+1}, both affine recurrences.
// Rows, layout and the row arithmetic as helmholtz_factor_body; the pivots, products and q
// agree with its sequential sweeps up to rounding.
constexpr int HZF_T = 512;   // threads per system (>= kMaxNz)
__global__ void __launch_bounds__(1024) k_hz_factor(GridP g, double* __restrict__ hfac,
                                                    const double* __restrict__ dtp, double gamma, int wallmodel,
                                                    int kc) {
  static_assert(HZF_T >= kMaxNz, "one thread per row");
  __shared__ double sc[2][4][HZF_T];   // per system: scan values (up to a 2 x 2 matrix per row)
  const int n = g.nz;
  const int sys = (int)threadIdx.x / HZF_T, k = (int)threadIdx.x % HZF_T;   // 0: u/v, 1: w
  const int rows = sys == 0 ? n : n - 1;
  const bool row = k < rows;
  const double c = gamma * g.nu * dtp[0] / 2.0;
  // the row (a, b, cc) and the super-diagonal of the row below
  auto coeffs = [&](int kk, double& a, double& b, double& cc) {   // kk = 1 .. rows
    if (sys == 0) {
      double lo = 1.0 / (g.dzc[kk - 1] * g.dzf[kk]);
      double up = 1.0 / (g.dzc[kk] * g.dzf[kk]);
      double dg = -(lo + up);
      if (kk == 1) dg += wallmodel ? lo : -lo;
      if (kk == n) dg += wallmodel ? up : -up;
      if (kk == 1) lo = 0.0;
      if (kk == n) up = 0.0;
      a = -c * lo, b = 1.0 - c * dg, cc = -c * up;
    } else {
      const int m = n - 1;
      double lo = 1.0 / (g.dzf[kk] * g.dzc[kk]);
      double up = 1.0 / (g.dzf[kk + 1] * g.dzc[kk]);
      const double dg = -(lo + up);
      if (kk == 1) lo = 0.0;
      if (kk == m) up = 0.0;
      a = -c * lo, b = 1.0 - c * dg, cc = -c * up;
    }
  };
  double a = 0.0, b = 1.0, cc = 0.0, cbelow = 0.0;
  if (row) {
    coeffs(k + 1, a, b, cc);
    if (k > 0) {
      double a1, b1;
      coeffs(k, a1, b1, cbelow);
    }
    hfac[(sys == 0 ? 6 : 7) * n + k] = a;
    hfac[(sys == 0 ? 8 : 10) * n + k] = b;
    hfac[(sys == 0 ? 9 : 11) * n + k] = cc;
  }
  double (*S)[HZF_T] = sc[sys];
  // ---- pivots: inclusive scan of 2 x 2 matrix products (window product on the left)
  double m00 = b, m01 = -a * cbelow, m10 = 1.0, m11 = 0.0;
  for (int d = 1; d < n; d <<= 1) {   // levels: uniform across the block
    S[0][k] = m00, S[1][k] = m01, S[2][k] = m10, S[3][k] = m11;
    __syncthreads();
    if (k >= d && row) {
      const double q00 = S[0][k - d], q01 = S[1][k - d], q10 = S[2][k - d], q11 = S[3][k - d];
      double r00 = m00 * q00 + m01 * q10, r01 = m00 * q01 + m01 * q11;
      double r10 = m10 * q00 + m11 * q10, r11 = m10 * q01 + m11 * q11;
      const double big = fmax(fmax(fabs(r00), fabs(r01)), fmax(fabs(r10), fabs(r11)));
      int e;
      (void)frexp(big, &e);
      m00 = ldexp(r00, -e), m01 = ldexp(r01, -e), m10 = ldexp(r10, -e), m11 = ldexp(r11, -e);
    }
    __syncthreads();
  }
  const double r = m10 / m00;   // 1 / pivot
  const double cpk = cc * r;
  if (row) {
    hfac[(sys == 0 ? 1 : 3) * n + k] = r;
    hfac[(sys == 0 ? 0 : 2) * n + k] = cpk;
  }
  // ---- chunk products of -a r (segmented inclusive product scan)
  double pp = -a * r;
  const int seg0 = (k / kc) * kc;
  for (int d = 1; d < kc; d <<= 1) {
    S[0][k] = pp;
    __syncthreads();
    if (k - d >= seg0 && row) pp = pp * S[0][k - d];
    __syncthreads();
  }
  if (row) hfac[(sys == 0 ? 12 : 13) * n + k] = pp;
  // ---- flow-rate profile of the u/v system: 1 unless both walls are no-slip
  if (g.zbc != LES_ZBC_NOSLIP) {   // uniform across the block
    if (sys == 0 && row) hfac[4 * n + k] = 1.0;
    return;
  }
  // every thread takes part in the scans' barriers; the w system's values are not stored
  // forward affine scan x -> al + be x, a window's map applied after the one below it
  double al = r, be = -a * r;
  for (int d = 1; d < n; d <<= 1) {
    S[0][k] = al, S[1][k] = be;
    __syncthreads();
    if (k >= d && row) {
      const double al2 = S[0][k - d], be2 = S[1][k - d];
      al = al + be * al2;
      be = be * be2;
    }
    __syncthreads();
  }
  // back affine scan from the top row: q_k = d_k - c'_k q_{k+1}
  double bl = al, bb = k == rows - 1 ? 0.0 : -cpk;
  for (int d = 1; d < n; d <<= 1) {
    S[0][k] = bl, S[1][k] = bb;
    __syncthreads();
    if (k + d < rows && row) {
      const double bl2 = S[0][k + d], bb2 = S[1][k + d];
      bl = bl + bb * bl2;
      bb = bb * bb2;
    }
    __syncthreads();
  }
  if (sys == 0 && row) hfac[4 * n + k] = bl;
}

template <typename T>
void launch_predictor(Ctx& c, int stage) {
  static const double A[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
  static const double B[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
  const double G = A[stage] + B[stage];
  const int kc = c.pred_kc;
  const unsigned nch = (unsigned)((c.g.nz + kc - 1) / kc);
  const int mode = c.cfg.implicit_z;   // VISC_* (validated at init)
  const bool fused = hz_fused<T>(c);
  // the Helmholtz rows are needed with walls only (periodic z solves by FFT): a launch of its
  // own factorises them ahead of a predictor that eliminates along its march, else the extra
  // z slice of the predictor's launch does
  const int fslice = !fused && mode != VISC_EXPLICIT && c.cfg.zbc != LES_ZBC_PERIODIC ? 1 : 0;
  if (fused)
    LES_LAUNCH(c, "hz_factor", 0, k_hz_factor, dim3(1), dim3(2 * HZF_T), 0, c.g, c.t.hfac, c.t.dt, G,
               c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0, kc);
  const int TX = zmarch::TX, TY = c.pred_ty;
  const dim3 grid((c.g.nx + TX - 1) / TX, (c.g.ny + TY - 1) / TY, nch + fslice);
  const int use_rprev = stage > 0;
  const int write_r = stage < 2;
  // R^k written by substeps 0 and 1, R^{k-1} read by substeps 1 and 2
  auto pick = [&](auto m, auto ty) {
    constexpr int M = decltype(m)::value, Y = decltype(ty)::value;
    return stage == 0 ? k_predictor<T, M, 2, Y> : (stage == 1 ? k_predictor<T, M, 3, Y> : k_predictor<T, M, 1, Y>);
  };
  auto pick_ty = [&](auto m) {
    return TY == 16 ? pick(m, std::integral_constant<int, 16>()) : pick(m, std::integral_constant<int, 8>());
  };
  auto f = mode == VISC_CN_3D ? pick_ty(std::integral_constant<int, VISC_CN_3D>())
                              : (mode == VISC_CN_Z ? pick_ty(std::integral_constant<int, VISC_CN_Z>())
                                                   : pick_ty(std::integral_constant<int, VISC_EXPLICIT>()));
  const double pts = (double)c.g.sxy * c.g.nz;
  const double words = 8 + 3 * use_rprev + 3 * write_r;
  LES_LAUNCH(c, "predictor", words * pts * sizeof(T), f, grid, dim3(TX, TY), 0, c.g, (const T*)c.u, (const T*)c.v,
             (const T*)c.w, (const T*)c.p, (const T*)c.nut, c.t.coef, (T*)c.ru, (T*)c.rv, (T*)c.rw, (T*)c.us,
             (T*)c.vs, (T*)c.wsf, c.t.dt, A[stage], B[stage], G, c.t.hfac,
             c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0, kc, c.t.tau, fslice,
             fused ? (const double*)c.t.hfac : nullptr);
}

// ============================================================================ CN in z
// The matrix (1 - c L_zz), c = gamma nu dt / 2, is the same for every (i, j) column, so
// its Thomas factorisation (pivots and normalised super-diagonal) is computed once per
// substep by three threads: u/v rows, w rows, and the flow-rate profile q = H^-1 1 of
// the u rows (no-slip walls; 1 otherwise).  Layout of hfac: [cp_uv | rp_uv | cp_w | rp_w
// | q | - | a_uv | a_w | b_uv | c_uv | b_w | c_w | pp_uv | pp_w] each nz long (pp: see
// k_hz_factor).
// Runs in one block of nthr threads; dzf/dzc are LDS copies of the metrics.  Thread 0 runs
// the u/v chain (and the flow-rate profile), thread 64 (thread 0 in small blocks) the w chain.
__device__ void helmholtz_factor_body(const GridP& g, double* hfac, const double* dtp, double gamma, int wallmodel,
                                      double* dzf, double* dzc, int tid, int nthr) {
  const int n = g.nz;
  const int wthread = nthr > 64 ? 64 : 0;
  for (int k = tid; k < n + 2; k += nthr) {
    dzf[k] = g.dzf[k];
    dzc[k] = g.dzc[k];
  }
  __syncthreads();
  const double c = gamma * g.nu * dtp[0] / 2.0;
  double* cp_uv = hfac;
  double* rp_uv = hfac + n;
  double* cp_w = hfac + 2 * n;
  double* rp_w = hfac + 3 * n;
  double* qv = hfac + 4 * n;
  double* a_uv = hfac + 6 * n;
  double* a_w = hfac + 7 * n;
  double* b_uv = hfac + 8 * n;    // diagonal and super-diagonal of the rows (CN in all
  double* c_uv = hfac + 9 * n;    // directions shifts the diagonal per wavenumber pair)
  double* b_w = hfac + 10 * n;
  double* c_w = hfac + 11 * n;
  if (tid == 0) {
    double cprev = 0.0, dp = 0.0;
    for (int kk = 1; kk <= n; ++kk) {
      double lo = 1.0 / (dzc[kk - 1] * dzf[kk]);
      double up = 1.0 / (dzc[kk] * dzf[kk]);
      double dg = -(lo + up);
      if (kk == 1) dg += wallmodel ? lo : -lo;
      if (kk == n) dg += wallmodel ? up : -up;
      if (kk == 1) lo = 0.0;
      if (kk == n) up = 0.0;
      const double a = -c * lo, b = 1.0 - c * dg, cc = -c * up;
      const double r = 1.0 / (b - a * cprev);
      rp_uv[kk - 1] = r;
      a_uv[kk - 1] = a;
      b_uv[kk - 1] = b;
      c_uv[kk - 1] = cc;
      cprev = cc * r;
      cp_uv[kk - 1] = cprev;
      // forward sweep of q = H^-1 1 (bulk-forcing profile, no-slip rows) alongside
      dp = (1.0 - a * dp) * r;
      qv[kk - 1] = dp;
    }
    if (g.zbc == LES_ZBC_NOSLIP) {
      for (int kk = n - 1; kk >= 1; --kk) qv[kk - 1] = qv[kk - 1] - cp_uv[kk - 1] * qv[kk];
    } else {
      for (int kk = 0; kk < n; ++kk) qv[kk] = 1.0;
    }
  }
  if (tid == wthread) {
    const int m = n - 1;
    double cprev = 0.0;
    for (int kk = 1; kk <= m; ++kk) {
      double lo = 1.0 / (dzf[kk] * dzc[kk]);
      double up = 1.0 / (dzf[kk + 1] * dzc[kk]);
      const double dg = -(lo + up);
      if (kk == 1) lo = 0.0;
      if (kk == m) up = 0.0;
      const double a = -c * lo, b = 1.0 - c * dg, cc = -c * up;
      const double r = 1.0 / (b - a * cprev);
      rp_w[kk - 1] = r;
      a_w[kk - 1] = a;
      b_w[kk - 1] = b;
      c_w[kk - 1] = cc;
      cprev = cc * r;
      cp_w[kk - 1] = cprev;
    }
  }
}

// CN-z Helmholtz solves (Eq. onestar_imp1d), staged through LDS: a block takes hc
// consecutive (j, i) columns of one component, all threads load the m x hc right-hand sides
// produced by the predictor (coalesced along i, held in double), hc threads run the FP64
// elimination with the shared factors, all threads store.  The wall-model rows take the
// lagged wall stress (from u^k) as a known flux.
template <typename T>
__global__ void __launch_bounds__(256) k_helmholtz(GridP g, T* __restrict__ us, T* __restrict__ vs,
                                                   T* __restrict__ ws, const double* __restrict__ hfac,
                                                   const double* __restrict__ tau, const double* __restrict__ dtp,
                                                   double gamma, int wallmodel, int hc) {
  extern __shared__ double hsm[];   // [m][hc]
  const int comp = blockIdx.y;
  const int n = g.nz;
  const int m = comp < 2 ? n : n - 1;
  const int64_t s = g.sxy;
  const int64_t col0 = (int64_t)blockIdx.x * hc;
  const int cw = (int)(s - col0 < hc ? s - col0 : hc);
  T* x = (comp == 0 ? us : (comp == 1 ? vs : ws)) + s + col0;   // plane 1
  double* fac = hsm + (size_t)m * hc;   // c', 1/pivot, sub-diagonal of this component's rows
  for (int e = threadIdx.x; e < m; e += blockDim.x) {
    fac[e] = hfac[(comp < 2 ? 0 : 2 * n) + e];
    fac[m + e] = hfac[(comp < 2 ? n : 3 * n) + e];
    fac[2 * m + e] = hfac[(comp < 2 ? 6 * n : 7 * n) + e];
  }
  // loads in batches of HB per thread, all issued before their LDS stores
  constexpr int HB = 8;
  const int total = m * hc;
  for (int e0 = 0; e0 < total; e0 += HB * (int)blockDim.x) {
    T v[HB];
#pragma unroll
    for (int b = 0; b < HB; ++b) {
      const int e = e0 + b * (int)blockDim.x + (int)threadIdx.x;
      const int k = e / hc, q = e % hc;
      v[b] = (e < total && q < cw) ? x[(int64_t)k * s + q] : (T)0;
    }
#pragma unroll
    for (int b = 0; b < HB; ++b) {
      const int e = e0 + b * (int)blockDim.x + (int)threadIdx.x;
      if (e < total) hsm[e] = (double)v[b];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cw) {
    const int q = threadIdx.x;
    const double* cp = fac;
    const double* rp = fac + m;
    const double* av = fac + 2 * m;
    double* col = hsm + q;   // row k at col[k hc]
    if (comp < 2 && wallmodel) {
      const double c = gamma * g.nu * dtp[0] / 2.0;
      col[0] += c * (-(tau[(comp == 0 ? 0 : 1) * s + col0 + q] / g.nu) / g.dzf[1]);
      col[(n - 1) * hc] += c * (-(tau[(comp == 0 ? 2 : 3) * s + col0 + q] / g.nu) / g.dzf[n]);
    }
    // rows in chunks of CH, every LDS read of a chunk issued before its chain
    constexpr int CH = 8;
    double dp = 0.0;
    for (int k0 = 0; k0 < m; k0 += CH) {
      double fv[CH], a8[CH], r8[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int k = k0 + j < m ? k0 + j : m - 1;
        fv[j] = col[k * hc];
        a8[j] = av[k];
        r8[j] = rp[k];
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        if (k0 + j < m) {
          dp = (fv[j] - a8[j] * dp) * r8[j];
          col[(k0 + j) * hc] = dp;
        }
      }
    }
    double xn = dp;
    for (int k1 = m - 2; k1 >= 0; k1 -= CH) {
      double fv[CH], c8[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int k = k1 - j >= 0 ? k1 - j : 0;
        fv[j] = col[k * hc];
        c8[j] = cp[k];
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        if (k1 - j >= 0) {
          xn = fv[j] - c8[j] * xn;
          col[(k1 - j) * hc] = xn;
        }
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * hc; e += blockDim.x) {
    const int k = e / hc, q = e % hc;
    if (q < cw) x[(int64_t)k * s + q] = (T)hsm[e];
  }
}

// Back substitution of the CN-z systems eliminated by the predictor (Eq. onestar_imp1d): one
// thread per interior (j, i) column and component, marching down the rows.  The predictor's
// chunk c left e_r = d_r - pp_r D_c in its rows, D_c the elimination value of the row below
// the chunk; the D_c are rebuilt from the chunk tops upwards, then x_r = d_r - c'_r x_{r+1}.
template <typename T>
__global__ void __launch_bounds__(256) k_hz_back(GridP g, T* __restrict__ us, T* __restrict__ vs,
                                                 T* __restrict__ ws, const double* __restrict__ hfac, int kc) {
  __shared__ double dl[HZ_MAXCH][256];   // each thread's own chunk corrections
  const int comp = blockIdx.y;
  const int n = g.nz;
  const int m = comp < 2 ? n : n - 1;
  const int64_t s = g.sxy;
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= (int64_t)g.ny * g.nx) return;
  T* x = (comp == 0 ? us : (comp == 1 ? vs : ws)) + s + col;   // row r at x[r s]
  const double* cp = hfac + (comp < 2 ? 0 : 2 * n);
  const double* pp = hfac + (comp < 2 ? 12 * n : 13 * n);
  const int nch = (m + kc - 1) / kc;
  double D = 0.0;
  dl[0][threadIdx.x] = 0.0;
  for (int ch = 1; ch < nch; ++ch) {
    const int e = ch * kc - 1;
    D = (double)x[(int64_t)e * s] + ro_load(pp, e) * D;
    dl[ch][threadIdx.x] = D;
  }
  constexpr int B = 8;
  double xn = 0.0;
  for (int ch = nch - 1; ch >= 0; --ch) {
    const int lo = ch * kc, hi = min(m, lo + kc) - 1;
    const double Dc = dl[ch][threadIdx.x];
    for (int r0 = hi; r0 >= lo; r0 -= B) {
      double v[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int r = r0 - j >= lo ? r0 - j : lo;
        v[j] = (double)x[(int64_t)r * s];
      }
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int r = r0 - j;
        if (r >= lo) {
          const double d = ch > 0 ? v[j] + ro_load(pp, r) * Dc : v[j];
          xn = r == m - 1 ? d : d - ro_load(cp, r) * xn;
          x[(int64_t)r * s] = (T)xn;
        }
      }
    }
  }
}

template <typename T>
void launch_helmholtz(Ctx& c, int stage) {
  static const double G[3] = {8.0 / 15.0, 2.0 / 15.0, 1.0 / 3.0};
  if (hz_fused<T>(c)) {
    const dim3 grid((unsigned)(((int64_t)c.g.ny * c.g.nx + 255) / 256), 3);
    LES_LAUNCH(c, "helmholtz_z", 6.0 * c.g.ny * c.g.nx * c.g.nz * sizeof(T), k_hz_back<T>, grid, dim3(256), 0, c.g,
               (T*)c.us, (T*)c.vs, (T*)c.wsf, c.t.hfac, c.pred_kc);
    return;
  }
  // columns per block: the largest power of two <= 64 whose rows fit 64 KB of LDS
  int hc = 64;
  while (hc > 8 && (size_t)c.g.nz * (hc + 3) * sizeof(double) > 65536) hc /= 2;
  const size_t sh = (size_t)c.g.nz * (hc + 3) * sizeof(double);
  dim3 block(256), grid((unsigned)((c.g.sxy + hc - 1) / hc), 3);
  LES_LAUNCH(c, "helmholtz_z", 6.0 * c.g.sxy * c.g.nz * sizeof(T), k_helmholtz<T>, grid, block, sh, c.g, (T*)c.us,
             (T*)c.vs, (T*)c.wsf, c.t.hfac, c.t.tau, c.t.dt, G[stage], c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0, hc);
}

// ============================================================================ boundary planes
// Ghost planes after an update (Alg. 2 without the wall model): periodic copies, or
// w = 0 on wall faces, p Neumann, u and v odd (no-slip).  One thread per (j, i).
template <typename T>
__global__ void k_bc_fill(GridP g, T* u, T* v, T* w, T* p) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= g.sxy) return;
  const int64_t s = g.sxy, n = g.nz;
  if (g.zbc == LES_ZBC_PERIODIC) {
    T* f[4] = {u, v, w, p};
    for (int a = 0; a < 4; ++a) {
      f[a][c] = f[a][n * s + c];
      f[a][(n + 1) * s + c] = f[a][s + c];
    }
    return;
  }
  u[c] = -u[s + c];
  v[c] = -v[s + c];
  u[(n + 1) * s + c] = -u[n * s + c];
  v[(n + 1) * s + c] = -v[n * s + c];
  w[c] = (T)0;
  w[n * s + c] = (T)0;
  w[(n + 1) * s + c] = (T)0;
  p[c] = p[s + c];
  p[(n + 1) * s + c] = p[n * s + c];
}

template <typename T>
void launch_bc_fill(Ctx& c, T* u, T* v, T* w, T* p) {
  LES_LAUNCH(c, "bc_fill", 14.0 * c.g.sxy * sizeof(T), k_bc_fill<T>, dim3((unsigned)((c.g.sxy + 255) / 256)),
             dim3(256), 0, c.g, u, v, w, p);
}

// ============================================================================ correction
// u = u* - gamma dt G phi (Eq. correc), p += phi (Eq. p_update_exp) or
// p += phi - gamma nu dt/2 L_zz phi (Eq. p_update_imp1d), flow-rate shift s q(z) on u,
// then the non-wall-model ghost planes.  phi ghosts follow the Poisson boundary
// condition (zero flux at walls, periodic copy otherwise) and are read on the fly.
// Maximum over a whole wave of 64 lanes: DPP steps within each row of 16 lanes (quad
// permutations, half-row and row mirrors), then the four rows' values by readlane.
template <int CTRL>
__device__ inline double dpp_move_f64(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false));
}
__device__ inline double readlane_f64(double x, int L) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), L),
                          __builtin_amdgcn_readlane(__double2loint(x), L));
}
__device__ inline double whole_wave_max(double x) {
  x = fmax(x, dpp_move_f64<0xB1>(x));
  x = fmax(x, dpp_move_f64<0x4E>(x));
  x = fmax(x, dpp_move_f64<0x141>(x));
  x = fmax(x, dpp_move_f64<0x140>(x));
  return fmax(fmax(readlane_f64(x, 0), readlane_f64(x, 16)), fmax(readlane_f64(x, 32), readlane_f64(x, 48)));
}

template <typename T, bool ADV = false>
__device__ __forceinline__ void correct_body(dim3 bid, GridP g, const T* __restrict__ us, const T* __restrict__ vs,
                                                 const T* __restrict__ ws, const T* __restrict__ phi, T* __restrict__ u,
                                                 T* __restrict__ v, T* __restrict__ w, T* __restrict__ p,
                                                 const double* __restrict__ dtp, const double* __restrict__ qprof,
                                                 double gamma, int implicit, double* __restrict__ advp = nullptr) {
  const int i = bid.x * blockDim.x + threadIdx.x;
  const int j = bid.y * blockDim.y + threadIdx.y;
  const int k = bid.z + 1;
  // ADV: the maxima of the time step's advective measure of the new velocity, four slots per
  // block of the launch (by hardware block index), so every thread stays: one per wave when the
  // block is whole waves (no barrier; unused slots 0), else (narrow grids) the block's maximum
  // by LDS atomics on the bits (non-negative doubles order as their bit patterns) in slot 0
  const int nthr = (int)(blockDim.x * blockDim.y), tid = (int)(threadIdx.y * blockDim.x + threadIdx.x);
  __shared__ unsigned long long bmax;
  double adv = 0.0;
  if constexpr (ADV) {
    if (nthr % 64 != 0) {
      if (tid == 0) bmax = 0;
      __syncthreads();
    }
  }
  if (i < g.nx && j < g.ny) {
  const int n = g.nz;
  const bool per = g.zbc == LES_ZBC_PERIODIC;
  const int kp = (k == n) ? (per ? 1 : n) : k + 1;   // phi ghost plane by BC
  const int km = (k == 1) ? (per ? n : 1) : k - 1;
  const int64_t c0 = idx3(g, k, j, i);
  const T gdt = (T)(gamma * dtp[0]);
  const T ph = phi[c0];
  const T phx = phi[idx3(g, k, j, wrap_p(i, g.nx))];
  const T phy = phi[idx3(g, k, wrap_p(j, g.nys), i)];
  const T phz = phi[idx3(g, kp, j, i)];
  T un = us[c0] - gdt * ((phx - ph) * (T)g.rdx);
  if (qprof != nullptr) un = un + (T)(dtp[1] * qprof[k - 1]);
  const T vn = (g.ywall && j == g.ny - 1) ? (T)0 : vs[c0] - gdt * ((phy - ph) * (T)g.rdy);
  T wn;
  if (!per && k == n) wn = (T)0;
  else wn = ws[c0] - gdt * ((phz - ph) * (T)g.rdzc[k]);
  T pn = p[c0] + ph;
  if (implicit) {
    // Eq. p_update_imp1d (L_zz) or Eq. p_update_imp3d (full Laplacian)
    const T phm = phi[idx3(g, km, j, i)];
    T lap = ((phz - ph) * (T)g.rdzc[k] - (ph - phm) * (T)g.rdzc[k - 1]) * (T)g.rdzf[k];
    if (implicit == 2) {
      const T phxm = phi[idx3(g, k, j, wrap_m(i, g.nx))], phym = phi[idx3(g, k, wrap_m(j, g.nys), i)];
      lap = (phx - (T)2 * ph + phxm) * (T)(g.rdx * g.rdx) + (phy - (T)2 * ph + phym) * (T)(g.rdy * g.rdy) + lap;
    }
    pn = pn - (T)(gamma * g.nu * dtp[0] / 2.0) * lap;
  }
  u[c0] = un;
  v[c0] = vn;
  w[c0] = wn;
  p[c0] = pn;
  if constexpr (ADV) {
    adv = cfl_adv((double)un, (double)vn, (double)wn, g.rdx, g.rdy, g.rdzf[k]);
    if (!(adv == adv)) adv = 0.0;   // a NaN counts as 0, as fmax has it
  }
  // ghost planes
  const int64_t s = g.sxy;
  const int64_t c2 = (int64_t)j * g.nx + i;
  if (per) {
    if (k == n) { u[c2] = un; v[c2] = vn; w[c2] = wn; p[c2] = pn; }
    if (k == 1) { u[(n + 1) * s + c2] = un; v[(n + 1) * s + c2] = vn; w[(n + 1) * s + c2] = wn; p[(n + 1) * s + c2] = pn; }
  } else {
    if (k == 1) { u[c2] = -un; v[c2] = -vn; w[c2] = (T)0; p[c2] = pn; }
    if (k == n) { u[(n + 1) * s + c2] = -un; v[(n + 1) * s + c2] = -vn; w[(n + 1) * s + c2] = (T)0; p[(n + 1) * s + c2] = pn; }
  }
  }
  if constexpr (ADV) {
    double* slot = advp + 4 * (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
    if (nthr % 64 == 0) {
      adv = whole_wave_max(adv);
      if (tid % 64 == 0) slot[tid / 64] = adv;
      if (tid == 0)
        for (int q = nthr / 64; q < 4; ++q) slot[q] = 0.0;
    } else {
      if (i < g.nx && j < g.ny) atomicMax(&bmax, (unsigned long long)__double_as_longlong(adv));
      __syncthreads();
      if (tid == 0) {
        slot[0] = __longlong_as_double((long long)bmax);
        slot[1] = slot[2] = slot[3] = 0.0;
      }
    }
  }
}

template <typename T, bool ADV>
__global__ void __launch_bounds__(256) k_correct(GridP g, const T* us, const T* vs, const T* ws, const T* phi, T* u,
                                                 T* v, T* w, T* p, const double* dtp, const double* qprof,
                                                 double gamma, int implicit, double* advp) {
  correct_body<T, ADV>(xcd_tile(blockIdx, gridDim), g, us, vs, ws, phi, u, v, w, p, dtp, qprof, gamma, implicit,
                       advp);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_correct(BatchMap m, double gamma) {
  int box;
  const dim3 bid = batch_bid(m, BK_POINT, blockIdx.x, box);
  const BoxDesc& d = m.desc[box];
  correct_body<T>(bid, d.g, (const T*)d.us, (const T*)d.vs, (const T*)d.wsf, (const T*)d.phi, (T*)d.u, (T*)d.v,
                  (T*)d.w, (T*)d.p, d.dt, nullptr, gamma, 0);
}

template <typename T>
void launch_correct(Ctx& c, int stage) {
  static const double G[3] = {8.0 / 15.0, 2.0 / 15.0, 1.0 / 3.0};
  Launch3 L = tile_launch(c.g, c.g.nz);
  const double* q = c.cfg.ubulk > 0.0 ? c.t.hfac + 4 * c.g.nz : nullptr;
  // FP64: the advective maxima of the new velocity for the next time step, unless
  // LES_CFL_PASS=1 (in FP32 the extra work cost the correction more than the pass it saves)
  const bool adv = c.cfl_fold && sizeof(T) == 8;
  c.cfl_adv_ready = adv;
  LES_LAUNCH(c, "correct", 9.0 * c.g.sxy * c.g.nz * sizeof(T), (adv ? k_correct<T, true> : k_correct<T, false>),
             L.grid, L.block, 0, c.g, (const T*)c.us, (const T*)c.vs,
                     (const T*)c.wsf, (const T*)c.phi, (T*)c.u, (T*)c.v, (T*)c.w, (T*)c.p, c.t.dt, q, G[stage],
                     c.cfg.implicit_z, c.t.cflc);
}

// ============================================================================ wall model
// Newton-Raphson for u_tau in u_tau [ln(u_tau h/nu)/kappa + B] = U (Eq. wm, Sec. 2.2),
// kept on the increasing branch of the convex left-hand side, to |du| <= 1e-14 u_tau.
__device__ inline double wm_newton(double U, double h, double nu, double kappa, double bconst, double guess) {
  if (!(U > 0.0)) return 0.0;
  const double xmin = nu / h * exp(-kappa * bconst - 1.0);
  double x = guess > xmin ? guess : fmax(sqrt(nu * U / h), 2.0 * xmin);
  for (int it = 0; it < 100; ++it) {
    const double lg = log(x * h / nu);
    const double f = x * (lg / kappa + bconst) - U;
    const double fp = lg / kappa + bconst + 1.0 / kappa;
    double xn = x - f / fp;
    if (xn <= xmin) xn = 0.5 * (x + xmin);
    if (fabs(xn - x) <= 1e-14 * xn) return xn;
    x = xn;
  }
  return x;
}

// One thread per (wall, component, j, i): interpolate to h_wm, bring the other component
// to the same face by its four-face mean, solve for u_tau, store tau and the ghost value
// that makes the viscous wall flux equal to tau.
template <typename T>
__global__ void k_wallmodel(GridP g, T* u, T* v, double* tau, double* utau, int kb0, int kb1, double tb, double hb,
                            int kt0, int kt1, double tt, double ht, double kappa, double bconst) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int which = blockIdx.y;  // 0 bot-x, 1 bot-y, 2 top-x, 3 top-y
  if (c >= (int64_t)g.nx * g.ny) return;   // interior rows (a duct's ghost rows carry no stress)
  const int i = (int)(c % g.nx), j = (int)(c / g.nx);
  const bool top = which >= 2;
  const bool isx = (which & 1) == 0;
  const int k0 = top ? kt0 : kb0, k1 = top ? kt1 : kb1;
  const double t = top ? tt : tb, h = top ? ht : hb;
  auto at = [&](const T* f, int jj, int ii) {
    return (1.0 - t) * (double)f[idx3(g, k0, jj, ii)] + t * (double)f[idx3(g, k1, jj, ii)];
  };
  double a, b;
  if (isx) {
    a = at(u, j, i);
    const int ip = wrap_p(i, g.nx), jm = wrap_m(j, g.nys);
    b = 0.25 * (at(v, j, i) + at(v, j, ip) + at(v, jm, i) + at(v, jm, ip));
  } else {
    a = at(v, j, i);
    const int im = wrap_m(i, g.nx), jp = wrap_p(j, g.nys);
    b = 0.25 * (at(u, j, i) + at(u, j, im) + at(u, jp, i) + at(u, jp, im));
  }
  const double U = sqrt(a * a + b * b);
  const int64_t o = (int64_t)which * g.sxy + c;
  const double x = wm_newton(U, h, g.nu, kappa, bconst, utau[o]);
  utau[o] = x;
  // the v row on a duct's wall face y = ly has no wall-parallel velocity
  const double tw = (U > 0.0 && !(g.ywall && !isx && j == g.ny - 1)) ? x * x * a / U : 0.0;
  tau[o] = tw;
  T* f = isx ? u : v;
  const int n = g.nz;
  if (!top) f[c] = (T)((double)f[g.sxy + c] - g.dzc[0] * tw / g.nu);
  else f[(int64_t)(n + 1) * g.sxy + c] = (T)((double)f[(int64_t)n * g.sxy + c] - g.dzc[n] * tw / g.nu);
}

template <typename T>
void launch_wallmodel(Ctx& c) {
  const int n = c.g.nz;
  int kb0 = 1, kb1 = 2, kt0 = n, kt1 = n - 1;
  double tb = 0.0, tt = 0.0, hb = c.zc[1], ht = c.cfg.lz - c.zc[n];
  if (c.cfg.h_wm > 0.0) {
    const double h = c.cfg.h_wm;
    for (int k = 1; k < n; ++k)
      if (c.zc[k] <= h) kb0 = k;
    kb1 = kb0 + 1;
    tb = (h - c.zc[kb0]) / (c.zc[kb1] - c.zc[kb0]);
    for (int k = n; k >= 2; --k)
      if (c.cfg.lz - c.zc[k] <= h) kt0 = k;
    kt1 = kt0 - 1;
    const double lo = c.cfg.lz - c.zc[kt0], hi = c.cfg.lz - c.zc[kt1];
    tt = (h - lo) / (hi - lo);
    hb = ht = h;
  }
  dim3 grid((unsigned)((c.g.sxy + 255) / 256), 4);
  LES_LAUNCH(c, "wallmodel", c.g.sxy * (8.0 * sizeof(T) + 4 * 3 * 8.0), k_wallmodel<T>, grid, dim3(256), 0, c.g, (T*)c.u, (T*)c.v, c.t.tau, c.t.utau, kb0,
                     kb1, tb, hb, kt0, kt1, tt, ht, c.cfg.kappa, c.cfg.bconst);
}

// ============================================================================ duct: y walls
// The square duct (Sec. 4.4) keeps two ghost rows per plane after the interior rows: row ny
// above y = ly and row ny + 1 below y = 0, where the wrapped index j - 1 of row 0 lands, so
// the y-periodic stencils read the boundary values there.  Rules (Alg. 2 with the z walls'
// treatment in y): v = 0 on both wall faces (row ny - 1 and ghost row ny + 1; row ny is
// never read and is set to 0), u and w odd (no-slip) or from the y-wall stresses (the
// viscous flux nu (u_0 - u_ghost)/dy equals the stress), p even.  One thread per (k, i),
// every stored plane k = 0..nz+1, run after the z ghost planes so that the corners follow
// the y rule.
template <typename T>
__global__ void k_bc_fill_y(GridP g, T* u, T* v, T* w, T* p, const double* tauy, int wallmodel) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= g.nx) return;
  const int ny = g.ny;
  const int64_t lo = idx3(g, k, ny + 1, i), hi = idx3(g, k, ny, i);
  const int64_t j0 = idx3(g, k, 0, i), j1 = idx3(g, k, ny - 1, i);
  v[j1] = (T)0;
  v[hi] = (T)0;
  v[lo] = (T)0;
  if (wallmodel) {
    const int64_t s = (int64_t)(g.nz + 2) * g.nx, o = (int64_t)k * g.nx + i;
    u[lo] = (T)((double)u[j0] - g.dy * tauy[o] / g.nu);
    w[lo] = (T)((double)w[j0] - g.dy * tauy[s + o] / g.nu);
    u[hi] = (T)((double)u[j1] - g.dy * tauy[2 * s + o] / g.nu);
    w[hi] = (T)((double)w[j1] - g.dy * tauy[3 * s + o] / g.nu);
  } else {
    u[lo] = -u[j0];
    w[lo] = -w[j0];
    u[hi] = -u[j1];
    w[hi] = -w[j1];
  }
  p[lo] = p[j0];
  p[hi] = p[j1];
}

template <typename T>
void launch_bc_fill_y(Ctx& c, T* u, T* v, T* w, T* p) {
  LES_LAUNCH(c, "bc_fill_y", 14.0 * c.g.nx * (c.g.nz + 2) * sizeof(T), k_bc_fill_y<T>,
             dim3((unsigned)((c.g.nx + 63) / 64), (unsigned)(c.g.nz + 2)), dim3(64), 0, c.g, u, v, w, p, c.t.tauy,
             c.cfg.zbc == LES_ZBC_WALLMODEL ? 1 : 0);
}

// y ghost rows of a cell-centred scalar: even (sign 1: pressure, pressure correction) or odd
// (sign -1: the eddy-viscosity field, R12 in y), every stored plane.
template <typename T>
__global__ void k_fill_y_scalar(GridP g, T* f, T sign) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= g.nx) return;
  f[idx3(g, k, g.ny + 1, i)] = sign * f[idx3(g, k, 0, i)];
  f[idx3(g, k, g.ny, i)] = sign * f[idx3(g, k, g.ny - 1, i)];
}

template <typename T>
void launch_fill_y_scalar(Ctx& c, T* f, double sign) {
  LES_LAUNCH(c, "fill_y", 4.0 * c.g.nx * (c.g.nz + 2) * sizeof(T), k_fill_y_scalar<T>,
             dim3((unsigned)((c.g.nx + 63) / 64), (unsigned)(c.g.nz + 2)), dim3(64), 0, c.g, f, (T)sign);
}

// Wall model on the y walls: the z-wall rule with y and z exchanged.  One thread per (wall,
// component, k, i): u (at (i+1/2, k)) and w (at (i, k+1/2)) interpolated in y to h_wm, the
// other component brought to the point by its four-face mean (x and z neighbours), Newton for
// u_tau, tau = u_tau^2 (component)/U.  w on the z wall face k = nz carries no stress; the
// ghost rows are written afterwards from tau (k_bc_fill_y).  tauy: [4][nz+2][nx] (tau_x at
// y = 0, tau_z at y = 0, tau_x at y = ly, tau_z at y = ly), ghost planes left at zero.
template <typename T>
__global__ void k_wallmodel_y(GridP g, const T* u, const T* w, double* tauy, double* utauy, int jb0, int jb1,
                              double tb, double hb, int jt0, int jt1, double tt, double ht, double kappa,
                              double bconst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y + 1;
  const int which = blockIdx.z;   // 0 lo-x, 1 lo-z, 2 hi-x, 3 hi-z
  if (i >= g.nx) return;
  const bool top = which >= 2;
  const bool isx = (which & 1) == 0;
  const int j0 = top ? jt0 : jb0, j1 = top ? jt1 : jb1;
  const double t = top ? tt : tb, h = top ? ht : hb;
  auto at = [&](const T* f, int kk, int ii) {
    return (1.0 - t) * (double)f[idx3(g, kk, j0, ii)] + t * (double)f[idx3(g, kk, j1, ii)];
  };
  const int64_t o = (int64_t)which * (g.nz + 2) * g.nx + (int64_t)k * g.nx + i;
  if (!isx && k == g.nz) {
    tauy[o] = 0.0;
    return;
  }
  double a, b;
  if (isx) {
    a = at(u, k, i);
    const int ip = wrap_p(i, g.nx);
    b = 0.25 * (at(w, k, i) + at(w, k, ip) + at(w, k - 1, i) + at(w, k - 1, ip));
  } else {
    a = at(w, k, i);
    const int im = wrap_m(i, g.nx);
    b = 0.25 * (at(u, k, i) + at(u, k, im) + at(u, k + 1, i) + at(u, k + 1, im));
  }
  const double U = sqrt(a * a + b * b);
  const double x = wm_newton(U, h, g.nu, kappa, bconst, utauy[o]);
  utauy[o] = x;
  tauy[o] = U > 0.0 ? x * x * a / U : 0.0;
}

template <typename T>
void launch_wallmodel_y(Ctx& c) {
  const int ny = c.g.ny;
  const double dy = c.g.dy;
  auto yc = [&](int j) { return (j + 0.5) * dy; };
  int jb0 = 0, jb1 = 1, jt0 = ny - 1, jt1 = ny - 2;
  double tb = 0.0, tt = 0.0, hb = yc(0), ht = c.cfg.ly - yc(ny - 1);
  if (c.cfg.h_wm > 0.0) {
    const double h = c.cfg.h_wm;
    for (int j = 0; j < ny - 1; ++j)
      if (yc(j) <= h) jb0 = j;
    jb1 = jb0 + 1;
    tb = (h - yc(jb0)) / (yc(jb1) - yc(jb0));
    for (int j = ny - 1; j >= 1; --j)
      if (c.cfg.ly - yc(j) <= h) jt0 = j;
    jt1 = jt0 - 1;
    const double lo = c.cfg.ly - yc(jt0), hi = c.cfg.ly - yc(jt1);
    tt = (h - lo) / (hi - lo);
    hb = ht = h;
  }
  LES_LAUNCH(c, "wallmodel_y", (double)c.g.nx * c.g.nz * (8.0 * sizeof(T) + 4 * 3 * 8.0), k_wallmodel_y<T>,
             dim3((unsigned)((c.g.nx + 63) / 64), (unsigned)c.g.nz, 4), dim3(64), 0, c.g, (const T*)c.u, (const T*)c.w,
             c.t.tauy, c.t.utauy, jb0, jb1, tb, hb, jt0, jt1, tt, ht, c.cfg.kappa, c.cfg.bconst);
}

// ============================================================================ time step
// Block maxima of |u|/dx + |v|/dy + |w|/dzf and of nu_t, reduced in a fixed order by a
// single block which then writes dt (R22 reading of the paper's time-step rule).
// VISC_ONLY: the maxima of nu_t alone (the advective ones come from the correction's blocks)
template <typename T, bool VISC_ONLY = false>
__device__ __forceinline__ void cfl_partial_body(int b, int nb, GridP g, const T* u, const T* v, const T* w,
                                                 const T* nut, const double* coef, double* part,
                                                 const double* adv = nullptr, int64_t nadv = 0) {
  __shared__ double sm[2][256];
  double mc = 0.0, mn = 0.0;
  if constexpr (VISC_ONLY) {
    // the advective maxima: this block's share of the correction's block maxima
    const int64_t per = (nadv + nb - 1) / nb, e0 = (int64_t)b * per, e1 = min(e0 + per, nadv);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) mc = fmax(mc, adv[e]);
  }
  // interior cells: the first nxy of every plane (a duct's ghost rows follow them)
  const int64_t nxy = (int64_t)g.nx * g.ny;
  const int64_t total = (int64_t)g.nz * nxy;
  // the flattened interior index advances by a fixed stride: its plane and in-plane offset
  // are stepped along instead of divided out per element
  const int64_t step = (int64_t)nb * blockDim.x;
  int64_t e = b * (int64_t)blockDim.x + threadIdx.x;
  int k = (int)(e / nxy) + 1;
  int64_t r = e % nxy;
  const int64_t dk = step / nxy, dr = step % nxy;
  for (; e < total; e += step) {
    const int64_t c = (int64_t)k * g.sxy + r;
    if constexpr (!VISC_ONLY) mc = fmax(mc, cfl_adv((double)u[c], (double)v[c], (double)w[c], g.rdx, g.rdy, g.rdzf[k]));
    mn = fmax(mn, coef[k] * (double)nut[c]);
    k += (int)dk;
    r += dr;
    if (r >= nxy) {
      r -= nxy;
      ++k;
    }
  }
  sm[0][threadIdx.x] = mc;
  sm[1][threadIdx.x] = mn;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sm[0][threadIdx.x] = fmax(sm[0][threadIdx.x], sm[0][threadIdx.x + s]);
      sm[1][threadIdx.x] = fmax(sm[1][threadIdx.x], sm[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * b] = sm[0][0];
    part[2 * b + 1] = sm[1][0];
  }
}

template <typename T, bool VISC_ONLY>
__global__ void __launch_bounds__(256) k_cfl_partial(GridP g, const T* u, const T* v, const T* w, const T* nut,
                                                     const double* coef, double* part, const double* adv,
                                                     int64_t nadv) {
  cfl_partial_body<T, VISC_ONLY>(blockIdx.x, gridDim.x, g, u, v, w, nut, coef, part, adv, nadv);
}

__device__ __forceinline__ void cfl_final_body(const double* part, int nblk, double* dtp, double cfl, double nu,
                                               double sinv) {
  __shared__ double sm[2][256];
  double mc = 0.0, mn = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    mc = fmax(mc, part[2 * b]);
    mn = fmax(mn, part[2 * b + 1]);
  }
  sm[0][threadIdx.x] = mc;
  sm[1][threadIdx.x] = mn;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sm[0][threadIdx.x] = fmax(sm[0][threadIdx.x], sm[0][threadIdx.x + s]);
      sm[1][threadIdx.x] = fmax(sm[1][threadIdx.x], sm[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double dtv = 0.95 * 2.51 / (4.0 * (nu + sm[1][0]) * sinv);
    const double dtc = sm[0][0] > 0.0 ? cfl / sm[0][0] : INFINITY;
    dtp[0] = fmin(dtc, dtv);
  }
}

__global__ void __launch_bounds__(256) k_cfl_final(const double* part, int nblk, double* dtp, double cfl, double nu,
                                                   double sinv) {
  cfl_final_body(part, nblk, dtp, cfl, nu, sinv);
}

// Batched time step: BK_CFL blocks per box write partials into the box's reduction area,
// then one block per box forms that box's dt (explicit viscous terms in all directions).
template <typename T>
__global__ void __launch_bounds__(256) kb_cfl_partial(BatchMap m) {
  int box;
  const dim3 bid = batch_bid(m, BK_CFL, blockIdx.x, box);
  const BoxDesc& d = m.desc[box];
  cfl_partial_body<T>(bid.x, d.gdim[BK_CFL][0], d.g, (const T*)d.u, (const T*)d.v, (const T*)d.w, (const T*)d.nut,
                      d.coef, d.red);
}

__global__ void __launch_bounds__(256) kb_cfl_final(BatchMap m, double cfl) {
  const BoxDesc& d = m.desc[blockIdx.x];
  double dmin = 1e300;
  for (int k = 1; k <= d.g.nz; ++k) dmin = fmin(dmin, d.g.dzf[k]);
  const double sinv = d.g.rdx * d.g.rdx + d.g.rdy * d.g.rdy + 1.0 / (dmin * dmin);
  cfl_final_body(d.red, d.gdim[BK_CFL][0], d.dt, cfl, d.g.nu, sinv);
}

// Batched dt from the host: dt for every box.
__global__ void kb_set_dt(BatchMap m, double dt) {
  if (threadIdx.x == 0) m.desc[blockIdx.x].dt[0] = dt;
}

template <typename T>
void launch_dt(Ctx& c, double cfl) {
  // the advective maxima from the last correction's blocks while the fields are those it wrote
  // (les_nut, les_bind and les_project drop them), else from a pass of their own; the nu_t-only
  // pass takes more blocks (one load per cell)
  const bool fold = c.cfl_fold && c.cfl_adv_ready;
  const int nblk = fold ? 2048 : 512;
  static_assert(2 * 2048 <= 4096, "partials fit the reduction area");
  const Launch3 L = tile_launch(c.g, c.g.nz);
  const int64_t nadv = fold ? 4 * (int64_t)L.grid.x * L.grid.y * L.grid.z : 0;
  if (fold)
    LES_LAUNCH(c, "cfl_visc", 1.0 * c.g.sxy * c.g.nz * sizeof(T), (k_cfl_partial<T, true>), dim3(nblk), dim3(256), 0,
               c.g, (const T*)c.u, (const T*)c.v, (const T*)c.w, (const T*)c.nut, c.t.coef, c.t.red,
               (const double*)c.t.cflc, nadv);
  else
    LES_LAUNCH(c, "cfl_partial", 4.0 * c.g.sxy * c.g.nz * sizeof(T), (k_cfl_partial<T, false>), dim3(nblk), dim3(256),
               0, c.g, (const T*)c.u, (const T*)c.v, (const T*)c.w, (const T*)c.nut, c.t.coef, c.t.red,
               (const double*)nullptr, (int64_t)0);
  // viscous limit: z term dropped with CN in z; with CN in all directions only the explicit
  // SGS viscosity limits (molecular viscosity passed as 0)
  double sinv = 1.0 / (c.g.dx * c.g.dx) + 1.0 / (c.g.dy * c.g.dy);
  if (c.cfg.implicit_z != VISC_CN_Z) {
    double dmin = 1e300;
    for (int k = 1; k <= c.g.nz; ++k) dmin = std::min(dmin, c.dzf[k]);
    sinv += 1.0 / (dmin * dmin);
  }
  const double nuv = c.cfg.implicit_z == VISC_CN_3D ? 0.0 : c.cfg.nu;
  LES_LAUNCH(c, "cfl_final", 0, k_cfl_final, dim3(1), dim3(256), 0, c.t.red, nblk, c.t.dt, cfl, nuv, sinv);
}

__global__ void k_set_dt(double* dtp, double dt) {
  if (threadIdx.x == 0) dtp[0] = dt;
}
void launch_set_dt(Ctx& c, double dt) { LES_LAUNCH(c, "set_dt", 0, k_set_dt, dim3(1), dim3(64), 0, c.t.dt, dt); }

// ============================================================================ diagnostics
// out: [0] max|div|, [1] sum(u dzf), [2] max |vel|, [3] nonfinite count, [4] sum tau_x bot,
// [5] sum tau_x top.  Stage 1: DIAG_BLOCKS blocks over contiguous chunks of the cells, each a
// fixed-order tree into 6 partials; stage 2: one block combines them in order (used
// synchronously by les_diag).
constexpr int DIAG_BLOCKS = 512;

template <typename T>
__global__ void __launch_bounds__(256) k_diag_partial(GridP g, const T* u, const T* v, const T* w, const T* p,
                                                      const double* tau, double* part) {
  __shared__ double sm[6][256];
  double md = 0.0, su = 0.0, mv = 0.0, nf = 0.0, tb = 0.0, tt = 0.0;
  const bool per = g.zbc == LES_ZBC_PERIODIC;
  const int64_t nxy = (int64_t)g.nx * g.ny;   // interior cells of a plane (stored first)
  const int64_t total = (int64_t)g.nz * nxy;
  const int64_t chunk = (total + DIAG_BLOCKS - 1) / DIAG_BLOCKS;
  const int64_t e0 = blockIdx.x * chunk, e1 = e0 + chunk < total ? e0 + chunk : total;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int k = (int)(e / nxy) + 1;
    const int64_t r = e % nxy;
    const int i = (int)(r % g.nx), j = (int)(r / g.nx);
    const int64_t c = (int64_t)k * g.sxy + r;
    const double d = ((double)u[c] - (double)u[idx3(g, k, j, wrap_m(i, g.nx))]) * g.rdx +
                     ((double)v[c] - (double)v[idx3(g, k, wrap_m(j, g.nys), i)]) * g.rdy +
                     ((double)w[c] - (double)w[c - g.sxy]) / g.dzf[k];
    md = fmax(md, fabs(d));
    su += (double)u[c] * g.dzf[k];
    mv = fmax(mv, fmax(fabs((double)u[c]), fmax(fabs((double)v[c]), fabs((double)w[c]))));
    if (!isfinite((double)u[c]) || !isfinite((double)v[c]) || !isfinite((double)w[c]) || !isfinite((double)p[c]))
      nf += 1.0;
  }
  if (!per && tau != nullptr) {
    const int64_t pc = (nxy + DIAG_BLOCKS - 1) / DIAG_BLOCKS;
    const int64_t r0 = blockIdx.x * pc, r1 = r0 + pc < nxy ? r0 + pc : nxy;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      tb += tau[r];
      tt += tau[2 * g.sxy + r];
    }
  }
  double vals[6] = {md, su, mv, nf, tb, tt};
  for (int a = 0; a < 6; ++a) sm[a][threadIdx.x] = vals[a];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sm[0][threadIdx.x] = fmax(sm[0][threadIdx.x], sm[0][threadIdx.x + s]);
      sm[1][threadIdx.x] += sm[1][threadIdx.x + s];
      sm[2][threadIdx.x] = fmax(sm[2][threadIdx.x], sm[2][threadIdx.x + s]);
      sm[3][threadIdx.x] += sm[3][threadIdx.x + s];
      sm[4][threadIdx.x] += sm[4][threadIdx.x + s];
      sm[5][threadIdx.x] += sm[5][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_diag_final(const double* part, double* out) {
  if (threadIdx.x != 0) return;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int b = 0; b < DIAG_BLOCKS; ++b) {
    v[0] = fmax(v[0], part[b * 6]);
    v[1] += part[b * 6 + 1];
    v[2] = fmax(v[2], part[b * 6 + 2]);
    v[3] += part[b * 6 + 3];
    v[4] += part[b * 6 + 4];
    v[5] += part[b * 6 + 5];
  }
  for (int a = 0; a < 6; ++a) out[a] = v[a];
}

template <typename T>
void launch_diag(Ctx& c, double* out_dev) {
  static_assert(DIAG_BLOCKS * 6 <= 4096, "partials fit the reduction area");
  LES_LAUNCH(c, "diag", 0, k_diag_partial<T>, dim3(DIAG_BLOCKS), dim3(256), 0, c.g, (const T*)c.u, (const T*)c.v,
             (const T*)c.w, (const T*)c.p, c.cfg.zbc == LES_ZBC_WALLMODEL ? c.t.tau : nullptr, c.t.red);
  LES_LAUNCH(c, "diag_final", 0, k_diag_final, dim3(1), dim3(64), 0, c.t.red, out_dev);
}

// ============================================================================ batch launchers
template <typename T>
void batch_predictor(hipStream_t st, const BatchMap& m, int total, int stage) {
  static const double A[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
  static const double B[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
  auto f = stage == 0 ? kb_predictor<T, 2> : (stage == 1 ? kb_predictor<T, 3> : kb_predictor<T, 1>);
  hipLaunchKernelGGL(f, dim3(total), dim3(32, 8), 0, st, m, A[stage], B[stage], A[stage] + B[stage]);
}
template <typename T>
void batch_correct(hipStream_t st, const BatchMap& m, int total, int stage) {
  static const double G[3] = {8.0 / 15.0, 2.0 / 15.0, 1.0 / 3.0};
  hipLaunchKernelGGL(kb_correct<T>, dim3(total), dim3(32, 8), 0, st, m, G[stage]);
}
template <typename T>
void batch_dt(hipStream_t st, const BatchMap& m, int total_cfl, int nbox, double cfl) {
  hipLaunchKernelGGL(kb_cfl_partial<T>, dim3(total_cfl), dim3(256), 0, st, m);
  hipLaunchKernelGGL(kb_cfl_final, dim3(nbox), dim3(256), 0, st, m, cfl);
}
void batch_set_dt(hipStream_t st, const BatchMap& m, int nbox, double dt) {
  hipLaunchKernelGGL(kb_set_dt, dim3(nbox), dim3(64), 0, st, m, dt);
}
template void batch_predictor<float>(hipStream_t, const BatchMap&, int, int);
template void batch_predictor<double>(hipStream_t, const BatchMap&, int, int);
template void batch_correct<float>(hipStream_t, const BatchMap&, int, int);
template void batch_correct<double>(hipStream_t, const BatchMap&, int, int);
template void batch_dt<float>(hipStream_t, const BatchMap&, int, int, double);
template void batch_dt<double>(hipStream_t, const BatchMap&, int, int, double);

// ============================================================================ instantiations
#define INST(T)                                                  \
  template void launch_predictor<T>(Ctx&, int);                  \
  template void launch_helmholtz<T>(Ctx&, int);                  \
  template void launch_correct<T>(Ctx&, int);                    \
  template void launch_bc_fill<T>(Ctx&, T*, T*, T*, T*);         \
  template void launch_wallmodel<T>(Ctx&);                       \
  template void launch_wallmodel_y<T>(Ctx&);                     \
  template void launch_bc_fill_y<T>(Ctx&, T*, T*, T*, T*);       \
  template void launch_fill_y_scalar<T>(Ctx&, T*, double);       \
  template void launch_dt<T>(Ctx&, double);                      \
  template void launch_diag<T>(Ctx&, double*);
INST(double)
INST(float)

}  // namespace les
