// Eigenfunction-expansion Poisson solver (Sec. 2.2: Fourier transforms in the periodic
// directions and the Thomas algorithm along the non-uniform one; Eq. poi).
//
//   k_rfftx      f = D u* / (gamma dt) (or a given field) on two neighbouring x-rows,
//                packed as one complex row, Stockham FFT in LDS, split into the two
//                half spectra l = 0..nx/2; also the flow-rate partial sums of u*.
//   k_fft_lines  complex FFT along y (or z) for tiles of consecutive l, in LDS.
//   k_thomas     FP64 Thomas solve along z for every (l, m) column, staged through LDS;
//                the singular (0, 0) column is pinned and mean-corrected.
//   k_fftz_solve periodic z: forward FFT along z, division by the eigenvalue sum, inverse.
//   k_irfftx     Hermitian reconstruction of two rows, inverse FFT, real and imaginary
//                parts back to the two rows of phi.
//
// Spectrum layout: complex [nz][ny][nx/2+1] (l fastest), interior planes only.
// Normalisation: forward transforms unscaled; the solve multiplies by 1/(nx ny [nz]) so
// the inverse transforms are plain sums.
#include "les_internal.h"

#include <algorithm>

namespace les {

template <typename R>
struct cpx {
  R x, y;
};

FftPlan make_plan(int n) {
  FftPlan p{};
  p.n = n;
  int m = n;
  int s = 0;
  if (m % 5 == 0) {
    p.rad[s++] = 5;
    m /= 5;
  }
  if (m % 3 == 0) {
    p.rad[s++] = 3;
    m /= 3;
  }
  while (m % 4 == 0) {
    p.rad[s++] = 4;
    m /= 4;
  }
  while (m % 2 == 0) {
    p.rad[s++] = 2;
    m /= 2;
  }
  p.nst = s;
  return p;
}

// Stockham autosort FFT (sub-transform size Ns grows by the radix each stage).  src and
// dst are ping-pong LDS buffers of one transform; `lane` and `team` split the butterflies
// of a stage among the team's threads.  DIR = -1 forward (exp(-2 pi i q/N)), +1 inverse.
// tw holds (cos, sin)(2 pi q/N), q = 0..N-1.  Each radix has its own body so that the
// butterfly operands stay in registers.
template <typename R, int DIR>
__device__ inline cpx<R> twiddle(cpx<R> a, const R* __restrict__ tw, int qq) {
  const R c = tw[2 * qq], sn = (R)DIR * tw[2 * qq + 1];
  return {a.x * c - a.y * sn, a.x * sn + a.y * c};
}

template <typename R, int DIR>
__device__ inline void stage2(const cpx<R>* src, cpx<R>* dst, int N, int Ns, const R* tw, int lane, int team) {
  const int nb = N / 2, ts = N / (Ns * 2);
  for (int b = lane; b < nb; b += team) {
    const int k = b % Ns;
    const cpx<R> v0 = src[b];
    const cpx<R> v1 = twiddle<R, DIR>(src[b + nb], tw, k * ts);
    const int o = (b / Ns) * Ns * 2 + k;
    dst[o] = {v0.x + v1.x, v0.y + v1.y};
    dst[o + Ns] = {v0.x - v1.x, v0.y - v1.y};
  }
}

template <typename R, int DIR>
__device__ inline void stage4(const cpx<R>* src, cpx<R>* dst, int N, int Ns, const R* tw, int lane, int team) {
  const int nb = N / 4, ts = N / (Ns * 4);
  for (int b = lane; b < nb; b += team) {
    const int k = b % Ns;
    const cpx<R> v0 = src[b];
    const cpx<R> v1 = twiddle<R, DIR>(src[b + nb], tw, k * ts);
    const cpx<R> v2 = twiddle<R, DIR>(src[b + 2 * nb], tw, 2 * k * ts);
    const cpx<R> v3 = twiddle<R, DIR>(src[b + 3 * nb], tw, 3 * k * ts);
    const cpx<R> s02 = {v0.x + v2.x, v0.y + v2.y}, d02 = {v0.x - v2.x, v0.y - v2.y};
    const cpx<R> s13 = {v1.x + v3.x, v1.y + v3.y}, d13 = {v1.x - v3.x, v1.y - v3.y};
    const cpx<R> jd = {-(R)DIR * d13.y, (R)DIR * d13.x};   // DIR * i * d13
    const int o = (b / Ns) * Ns * 4 + k;
    dst[o] = {s02.x + s13.x, s02.y + s13.y};
    dst[o + Ns] = {d02.x + jd.x, d02.y + jd.y};
    dst[o + 2 * Ns] = {s02.x - s13.x, s02.y - s13.y};
    dst[o + 3 * Ns] = {d02.x - jd.x, d02.y - jd.y};
  }
}

template <typename R, int DIR>
__device__ inline void stage3(const cpx<R>* src, cpx<R>* dst, int N, int Ns, const R* tw, int lane, int team) {
  const int nb = N / 3, ts = N / (Ns * 3);
  const R h3 = (R)0.86602540378443864676;
  for (int b = lane; b < nb; b += team) {
    const int k = b % Ns;
    const cpx<R> v0 = src[b];
    const cpx<R> v1 = twiddle<R, DIR>(src[b + nb], tw, k * ts);
    const cpx<R> v2 = twiddle<R, DIR>(src[b + 2 * nb], tw, 2 * k * ts);
    const cpx<R> s12 = {v1.x + v2.x, v1.y + v2.y}, d12 = {v1.x - v2.x, v1.y - v2.y};
    const cpx<R> m = {v0.x - (R)0.5 * s12.x, v0.y - (R)0.5 * s12.y};
    const cpx<R> jd = {-(R)DIR * h3 * d12.y, (R)DIR * h3 * d12.x};
    const int o = (b / Ns) * Ns * 3 + k;
    dst[o] = {v0.x + s12.x, v0.y + s12.y};
    dst[o + Ns] = {m.x + jd.x, m.y + jd.y};
    dst[o + 2 * Ns] = {m.x - jd.x, m.y - jd.y};
  }
}

// radix 5: with t1 = v1 + v4, t2 = v2 + v3, t3 = v1 - v4, t4 = v2 - v3 (c_q, s_q the cosine
// and sine of 2 pi q / 5): X1,4 = v0 + c1 t1 + c2 t2 +- DIR i (s1 t3 + s2 t4),
// X2,3 = v0 + c2 t1 + c1 t2 +- DIR i (s2 t3 - s1 t4), X0 = v0 + t1 + t2
template <typename R, int DIR>
__device__ inline void bfly5(const cpx<R> v[5], cpx<R> out[5]) {
  const R c1 = (R)0.30901699437494742410, c2 = (R)-0.80901699437494742410;
  const R s1 = (R)0.95105651629515357212, s2 = (R)0.58778525229247312917;
  const cpx<R> t1 = {v[1].x + v[4].x, v[1].y + v[4].y}, t2 = {v[2].x + v[3].x, v[2].y + v[3].y};
  const cpx<R> t3 = {v[1].x - v[4].x, v[1].y - v[4].y}, t4 = {v[2].x - v[3].x, v[2].y - v[3].y};
  const cpx<R> a1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
  const cpx<R> a2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
  const cpx<R> b1 = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
  const cpx<R> b2 = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
  const cpx<R> j1 = {-(R)DIR * b1.y, (R)DIR * b1.x}, j2 = {-(R)DIR * b2.y, (R)DIR * b2.x};   // DIR i b
  out[0] = {v[0].x + t1.x + t2.x, v[0].y + t1.y + t2.y};
  out[1] = {a1.x + j1.x, a1.y + j1.y};
  out[4] = {a1.x - j1.x, a1.y - j1.y};
  out[2] = {a2.x + j2.x, a2.y + j2.y};
  out[3] = {a2.x - j2.x, a2.y - j2.y};
}

template <typename R, int DIR>
__device__ inline void stage5(const cpx<R>* src, cpx<R>* dst, int N, int Ns, const R* tw, int lane, int team) {
  const int nb = N / 5, ts = N / (Ns * 5);
  for (int b = lane; b < nb; b += team) {
    const int k = b % Ns;
    cpx<R> v[5], o5[5];
    v[0] = src[b];
#pragma unroll
    for (int q = 1; q < 5; ++q) v[q] = twiddle<R, DIR>(src[b + q * nb], tw, q * k * ts);
    bfly5<R, DIR>(v, o5);
    const int o = (b / Ns) * Ns * 5 + k;
#pragma unroll
    for (int q = 0; q < 5; ++q) dst[o + q * Ns] = o5[q];
  }
}

template <typename R, int DIR>
__device__ cpx<R>* stockham(cpx<R>* src, cpx<R>* dst, const FftPlan& P, const R* __restrict__ tw, int lane, int team) {
  const int N = P.n;
  int Ns = 1;
  for (int s = 0; s < P.nst; ++s) {
    const int r = P.rad[s];
    if (r == 4) stage4<R, DIR>(src, dst, N, Ns, tw, lane, team);
    else if (r == 2) stage2<R, DIR>(src, dst, N, Ns, tw, lane, team);
    else if (r == 3) stage3<R, DIR>(src, dst, N, Ns, tw, lane, team);
    else stage5<R, DIR>(src, dst, N, Ns, tw, lane, team);
    __syncthreads();
    cpx<R>* t = src;
    src = dst;
    dst = t;
    Ns *= r;
  }
  return src;
}

// In-place Stockham for long strided lines, where the line groups of the ping-pong form are
// too narrow to fill a cache line: one LDS buffer holds twice the lines.  Each stage first
// reads every butterfly of the thread into registers (at most PPT / RAD of them, PPT = the
// points per thread that the launch guarantees), then, after a barrier, writes the outputs
// over the same buffer.
template <typename R, int DIR, int RAD, int BPT>
__device__ inline void stage_ip(cpx<R>* buf, int N, int Ns, const R* tw, int lane, int team) {
  const int nb = N / RAD, ts = N / (Ns * RAD);
  cpx<R> v[BPT][RAD];
#pragma unroll
  for (int t = 0; t < BPT; ++t) {
    const int b = lane + t * team;
    if (b < nb) {
      const int k = b % Ns;
      v[t][0] = buf[b];
#pragma unroll
      for (int q = 1; q < RAD; ++q) v[t][q] = twiddle<R, DIR>(buf[b + q * nb], tw, q * k * ts);
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < BPT; ++t) {
    const int b = lane + t * team;
    if (b < nb) {
      const int k = b % Ns;
      const int o = (b / Ns) * Ns * RAD + k;
      if (RAD == 2) {
        const cpx<R> v0 = v[t][0], v1 = v[t][1];
        buf[o] = {v0.x + v1.x, v0.y + v1.y};
        buf[o + Ns] = {v0.x - v1.x, v0.y - v1.y};
      } else if (RAD == 4) {
        const cpx<R> v0 = v[t][0], v1 = v[t][1], v2 = v[t][2], v3 = v[t][3];
        const cpx<R> s02 = {v0.x + v2.x, v0.y + v2.y}, d02 = {v0.x - v2.x, v0.y - v2.y};
        const cpx<R> s13 = {v1.x + v3.x, v1.y + v3.y}, d13 = {v1.x - v3.x, v1.y - v3.y};
        const cpx<R> jd = {-(R)DIR * d13.y, (R)DIR * d13.x};   // DIR * i * d13
        buf[o] = {s02.x + s13.x, s02.y + s13.y};
        buf[o + Ns] = {d02.x + jd.x, d02.y + jd.y};
        buf[o + 2 * Ns] = {s02.x - s13.x, s02.y - s13.y};
        buf[o + 3 * Ns] = {d02.x - jd.x, d02.y - jd.y};
      } else if (RAD == 5) {
        cpx<R> o5[5];
        bfly5<R, DIR>(v[t], o5);
#pragma unroll
        for (int q = 0; q < 5; ++q) buf[o + q * Ns] = o5[q];
      } else {
        const R h3 = (R)0.86602540378443864676;
        const cpx<R> v0 = v[t][0], v1 = v[t][1], v2 = v[t][RAD - 1];
        const cpx<R> s12 = {v1.x + v2.x, v1.y + v2.y}, d12 = {v1.x - v2.x, v1.y - v2.y};
        const cpx<R> m = {v0.x - (R)0.5 * s12.x, v0.y - (R)0.5 * s12.y};
        const cpx<R> jd = {-(R)DIR * h3 * d12.y, (R)DIR * h3 * d12.x};
        buf[o] = {v0.x + s12.x, v0.y + s12.y};
        buf[o + Ns] = {m.x + jd.x, m.y + jd.y};
        buf[o + 2 * Ns] = {m.x - jd.x, m.y - jd.y};
      }
    }
  }
  __syncthreads();
}

template <typename R, int DIR, int PPT>
__device__ cpx<R>* stockham_ip(cpx<R>* buf, const FftPlan& P, const R* __restrict__ tw, int lane, int team) {
  const int N = P.n;
  int Ns = 1;
  for (int s = 0; s < P.nst; ++s) {
    const int r = P.rad[s];
    if (r == 4) stage_ip<R, DIR, 4, (PPT + 3) / 4>(buf, N, Ns, tw, lane, team);
    else if (r == 2) stage_ip<R, DIR, 2, (PPT + 1) / 2>(buf, N, Ns, tw, lane, team);
    else if (r == 3) stage_ip<R, DIR, 3, (PPT + 2) / 3>(buf, N, Ns, tw, lane, team);
    else stage_ip<R, DIR, 5, (PPT + 4) / 5>(buf, N, Ns, tw, lane, team);
    Ns *= r;
  }
  return buf;
}

template <typename T>
__device__ inline const T* twsel(const double* d, const float* f);
template <>
__device__ inline const double* twsel<double>(const double* d, const float*) { return d; }
template <>
__device__ inline const float* twsel<float>(const double*, const float* f) { return f; }

// ============================================================================ forward x
// MODE 0: f = D u* scaled; MODE 1: f given (les_poisson).
template <typename T, int MODE>
__device__ __forceinline__ void rfftx_body(dim3 bid, GridP g, const FftPlan& P, const T* __restrict__ us, const T* __restrict__ vs,
                                               const T* __restrict__ ws, const T* __restrict__ fin,
                                               cpx<T>* __restrict__ spec, const double* __restrict__ twd,
                                               const float* __restrict__ twf, const double* __restrict__ dtp,
                                               double gamma, int npair_blk, double* __restrict__ bulk_part) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  const int nx = g.nx, nxh = nx / 2 + 1, nyh = g.ny / 2;
  cpx<T>* B = A + npair_blk * nx;
  const int64_t npairs = (int64_t)g.nz * nyh;
  // gamma = 0: the plain divergence (initial projection), no time factor
  const T scale = (MODE == 0 && gamma > 0.0) ? (T)(1.0 / (gamma * dtp[0])) : (T)1;
  double bsum = 0.0;
  for (int e = threadIdx.x; e < npair_blk * nx; e += blockDim.x) {
    const int p = e / nx, i = e % nx;
    const int64_t gp = (int64_t)bid.x * npair_blk + p;
    cpx<T> z = {(T)0, (T)0};
    if (gp < npairs) {
      const int k = (int)gp / nyh + 1;
      const int j0 = 2 * ((int)gp % nyh);
      T fv[2];
      for (int r = 0; r < 2; ++r) {
        const int j = j0 + r;
        const int64_t c = idx3(g, k, j, i);
        if (MODE == 0) {
          const T d = (us[c] - us[idx3(g, k, j, wrap_m(i, nx))]) * (T)g.rdx +
                      (vs[c] - ((g.ywall && j == 0) ? (T)0 : vs[idx3(g, k, wrap_m(j, g.ny), i)])) * (T)g.rdy +
                      (ws[c] - ((k == 1 && g.zbc == LES_ZBC_PERIODIC) ? ws[idx3(g, g.nz, j, i)] : ws[c - g.sxy])) *
                          (T)g.rdzf[k];
          fv[r] = d * scale;
          if (bulk_part) bsum += (double)us[c] * g.dzf[k];
        } else {
          fv[r] = fin[c];
        }
      }
      z = {fv[0], fv[1]};
    }
    A[e] = z;
  }
  if (bulk_part) {
    __shared__ double red[256];
    red[threadIdx.x] = bsum;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) bulk_part[bid.x] = red[0];
  }
  __syncthreads();
  const int team = blockDim.x / npair_blk;
  const int p = threadIdx.x / team, lane = threadIdx.x % team;
  cpx<T>* res = nullptr;
  {
    const T* tw = twsel<T>(twd, twf);
    res = stockham<T, -1>(A + p * nx, B + p * nx, P, tw, lane, team);
  }
  // res points into A or B for team p (same parity for all teams)
  const int64_t gp = (int64_t)bid.x * npair_blk + p;
  if (gp >= npairs) return;
  const int k = (int)gp / nyh;
  const int j0 = 2 * ((int)gp % nyh);
  cpx<T>* s0 = spec + ((int64_t)k * g.ny + j0) * g.nxp;
  cpx<T>* s1 = s0 + g.nxp;
  for (int l = lane; l < nxh; l += team) {
    const cpx<T> a = res[l];
    const cpx<T> b = res[(nx - l) % nx];
    // A_l = (Z_l + conj Z_{N-l})/2, B_l = (Z_l - conj Z_{N-l})/(2i)
    s0[l] = {(T)0.5 * (a.x + b.x), (T)0.5 * (a.y - b.y)};
    s1[l] = {(T)0.5 * (a.y + b.y), (T)0.5 * (b.x - a.x)};
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_rfftx(GridP g, FftPlan P, const T* us, const T* vs, const T* ws, const T* fin,
                                               cpx<T>* spec, const double* twd, const float* twf, const double* dtp,
                                               double gamma, int npair_blk, double* bulk_part) {
  rfftx_body<T, MODE>(blockIdx, g, P, us, vs, ws, fin, spec, twd, twf, dtp, gamma, npair_blk, bulk_part);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_rfftx(BatchMap m, double gamma) {
  int box;
  const dim3 bid = batch_bid(m, BK_RFFTX, blockIdx.x, box);
  const BoxDesc& d = m.desc[box];
  rfftx_body<T, 0>(bid, d.g, d.px, (const T*)d.us, (const T*)d.vs, (const T*)d.wsf, nullptr, (cpx<T>*)d.spec, d.twx,
                   d.twx_f, d.dt, gamma, d.pbx, nullptr);
}

// ============================================================================ inverse x
template <typename T>
__device__ __forceinline__ void irfftx_body(dim3 bid, GridP g, const FftPlan& P, const cpx<T>* __restrict__ spec,
                                                T* __restrict__ out, const double* __restrict__ twd,
                                                const float* __restrict__ twf, int npair_blk) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  const int nx = g.nx, nxh = nx / 2 + 1, nyh = g.ny / 2;
  cpx<T>* B = A + npair_blk * nx;
  const int64_t npairs = (int64_t)g.nz * nyh;
  // Hermitian reconstruction of two rows' spectra; loads in batches of four per thread,
  // all issued before their LDS stores
  const int total = npair_blk * nx;
  for (int e0 = 0; e0 < total; e0 += 4 * (int)blockDim.x) {
    cpx<T> va[4], vb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int e = e0 + b * (int)blockDim.x + (int)threadIdx.x;
      const int p = e / nx, l = e % nx;
      const int64_t gp = (int64_t)bid.x * npair_blk + p;
      const bool ok = e < total && gp < npairs;
      const int64_t k = ok ? (int)gp / nyh : 0;   // pair indices fit 32 bits
      const int j0 = ok ? 2 * ((int)gp % nyh) : 0;
      const int ls = l < nxh ? l : nx - l;
      const cpx<T>* s0 = spec + (k * g.ny + j0) * g.nxp;
      va[b] = s0[ls];
      vb[b] = s0[g.nxp + ls];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int e = e0 + b * (int)blockDim.x + (int)threadIdx.x;
      if (e >= total) continue;
      const int p = e / nx, l = e % nx;
      const int64_t gp = (int64_t)bid.x * npair_blk + p;
      cpx<T> z = {(T)0, (T)0};
      if (gp < npairs) {
        const cpx<T> a = va[b], bb = vb[b];
        z = l < nxh ? cpx<T>{a.x - bb.y, a.y + bb.x} : cpx<T>{a.x + bb.y, -a.y + bb.x};
      }
      A[e] = z;
    }
  }
  __syncthreads();
  const int team = blockDim.x / npair_blk;
  const int p = threadIdx.x / team, lane = threadIdx.x % team;
  const T* tw = twsel<T>(twd, twf);
  cpx<T>* res = stockham<T, 1>(A + p * nx, B + p * nx, P, tw, lane, team);
  const int64_t gp = (int64_t)bid.x * npair_blk + p;
  if (gp >= npairs) return;
  const int k = (int)gp / nyh + 1;
  const int j0 = 2 * ((int)gp % nyh);
  for (int i = lane; i < nx; i += team) {
    out[idx3(g, k, j0, i)] = res[i].x;
    out[idx3(g, k, j0 + 1, i)] = res[i].y;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_irfftx(GridP g, FftPlan P, const cpx<T>* spec, T* out, const double* twd,
                                                const float* twf, int npair_blk) {
  irfftx_body<T>(blockIdx, g, P, spec, out, twd, twf, npair_blk);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_irfftx(BatchMap m) {
  int box;
  const dim3 bid = batch_bid(m, BK_RFFTX, blockIdx.x, box);
  const BoxDesc& d = m.desc[box];
  irfftx_body<T>(bid, d.g, d.px, (const cpx<T>*)d.spec, (T*)d.phi, d.twx, d.twx_f, d.pbx);
}

// ============================================================================ strided lines
// Complex FFT of length P.n along a strided dimension for L consecutive l values:
// element t of line (l, o) is at base + o*ostride + t*lstride + l.  grid.x covers l tiles,
// grid.y covers o.  SOLVE (periodic z only): forward FFT, multiply by the normalisation
// over the eigenvalue lam = lamx + lamy + lamz of the operator, inverse FFT.  The operator
// is the Laplacian when hg = 0 (Poisson; the zero mode is set to 0), else the Helmholtz
// operator 1 - hg dt lam of Crank-Nicolson in all directions (hg = gamma nu / 2, dt from
// the device slot).
//
// DCT = 1 (ducts, walls in y): the lines are transformed by the cosine expansion of the
// zero-flux second difference instead, X_m = sum_t x_t cos(pi m (t + 1/2) / N) (DIR = -1)
// and its unnormalised inverse y_t = X_0 + 2 sum_{m >= 1} X_m cos(pi m (t + 1/2) / N) (DIR =
// +1, so that a forward-inverse pair multiplies by N, like the FFT pair), each through one
// complex FFT of length N of the same line (the lines are complex, and the transforms are
// linear, so real and imaginary parts go through together): forward, the line is loaded
// in the order x_0, x_2, .., x_{N-2}, x_{N-1}, .., x_3, x_1 and X_m = (W_m V_m + conj(W_m)
// V_{N-m}) / 2 with W_m = exp(-i pi m / (2N)) and V its FFT; inverse, V_m = conj(W_m) (X_m -
// i X_{N-m}) (X_N = 0) before the inverse FFT, whose output is stored back in the permuted
// order.  twc holds (cos, sin)(pi m / (2N)).
template <typename T, int DIR, bool SOLVE, int PPT = 0, int DCT = 0>
__device__ __forceinline__ void fft_lines_body(dim3 bid, const FftPlan& P, cpx<T>* __restrict__ data, int nl, int64_t lstride,
                                                   int64_t ostride, int L, const double* __restrict__ twd,
                                                   const float* __restrict__ twf, const double* __restrict__ lamx,
                                                   const double* __restrict__ lamy, const double* __restrict__ lamz,
                                                   double norm, const double* __restrict__ dtp = nullptr,
                                                   double hg = 0.0, const double* __restrict__ twcd = nullptr,
                                                   const float* __restrict__ twcf = nullptr) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  const int N = P.n;
  const int NP = N + 1;   // padded line stride in LDS (spreads the l-interleaved stores over banks)
  cpx<T>* B = A + L * NP;
  const int l0 = bid.x * L;
  const int o = bid.y;
  cpx<T>* base = data + (int64_t)o * ostride;
  // loads in batches of LB per thread, all issued before their LDS stores (out-of-range lanes
  // read element 0 and store zero): four, or in FP32 with the in-place form all PPT points of
  // the thread at once (measured faster there; slower in FP64)
  constexpr int LB = (sizeof(T) == 4 && PPT > 0) ? PPT : 4;
  const int total = L * N;
  for (int e0 = 0; e0 < total; e0 += LB * (int)blockDim.x) {
    cpx<T> v[LB];
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int e = e0 + b * (int)blockDim.x + (int)threadIdx.x;
      const int t = e / L, l = l0 + e % L;
      const bool ok = e < total && l < nl;
      v[b] = base[ok ? (int64_t)t * lstride + l : 0];
      if (!ok) v[b] = cpx<T>{(T)0, (T)0};
    }
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int e = e0 + b * (int)blockDim.x + (int)threadIdx.x;
      if (e < total) {
        const int t = e / L;
        // forward cosine transform: even points first, then odd points in reverse
        const int pos = (DCT && DIR < 0) ? ((t & 1) ? N - 1 - (t >> 1) : (t >> 1)) : t;
        A[(e % L) * NP + pos] = v[b];
      }
    }
  }
  __syncthreads();
  const int team = blockDim.x / L;
  const int ll = threadIdx.x / team, lane = threadIdx.x % team;
  const T* tw = twsel<T>(twd, twf);
  const T* twc = DCT ? twsel<T>(twcd, twcf) : nullptr;
  if (DCT && DIR > 0) {
    // inverse cosine transform: V_m = conj(W_m) (X_m - i X_{N-m}), pairs (m, N - m) in place
    cpx<T>* X = A + ll * NP;
    for (int m = lane; m <= N / 2; m += team) {
      const cpx<T> a = X[m];
      const cpx<T> b = m == 0 ? cpx<T>{(T)0, (T)0} : X[N - m];
      {
        const T c = twc[2 * m], sn = twc[2 * m + 1];
        const T zx = a.x + b.y, zy = a.y - b.x;
        X[m] = {c * zx - sn * zy, sn * zx + c * zy};
      }
      if (m > 0 && 2 * m != N) {
        const T c = twc[2 * (N - m)], sn = twc[2 * (N - m) + 1];
        const T zx = b.x + a.y, zy = b.y - a.x;
        X[N - m] = {c * zx - sn * zy, sn * zx + c * zy};
      }
    }
    __syncthreads();
  }
  cpx<T>* res;
  if constexpr (PPT > 0) res = stockham_ip<T, DIR, PPT>(A + ll * NP, P, tw, lane, team);
  else res = stockham<T, DIR>(A + ll * NP, B + ll * NP, P, tw, lane, team);
  if (SOLVE) {
    // res holds the z spectrum of column (l, m = o); o indexes y modes here
    const int l = l0 + ll;
    const double hc = hg != 0.0 ? hg * dtp[0] : 0.0;
    for (int t = lane; t < N; t += team) {
      double lam = (l < nl ? lamx[l] : 0.0) + lamy[o] + lamz[t];
      double f = hg != 0.0 ? norm / (1.0 - hc * lam) : ((lam != 0.0) ? norm / lam : 0.0);
      res[t].x = (T)((double)res[t].x * f);
      res[t].y = (T)((double)res[t].y * f);
    }
    __syncthreads();
    if constexpr (PPT > 0) {
      res = stockham_ip<T, 1, PPT>(res, P, tw, lane, team);
    } else {
      cpx<T>* other = (res == A + ll * NP) ? B + ll * NP : A + ll * NP;
      res = stockham<T, 1>(res, other, P, tw, lane, team);
    }
  }
  // every team's result lies in the same buffer (A or B)
  cpx<T>* R = (res == A + ll * NP) ? A : B;
  __syncthreads();
  for (int e = threadIdx.x; e < L * N; e += blockDim.x) {
    const int t = e / L, l2 = e % L;
    const int l = l0 + l2;
    if (l >= nl) continue;
    if (DCT && DIR < 0) {
      // X_t = (W_t V_t + conj(W_t) V_{N-t}) / 2
      const cpx<T> a = R[l2 * NP + t], b = R[l2 * NP + (t == 0 ? 0 : N - t)];
      const T c = twc[2 * t], sn = twc[2 * t + 1];
      const T xr = (c * a.x + sn * a.y) + (c * b.x - sn * b.y);
      const T xi = (c * a.y - sn * a.x) + (c * b.y + sn * b.x);
      base[(int64_t)t * lstride + l] = {(T)0.5 * xr, (T)0.5 * xi};
    } else if (DCT) {
      base[(int64_t)t * lstride + l] = R[l2 * NP + ((t & 1) ? N - 1 - (t >> 1) : (t >> 1))];
    } else {
      base[(int64_t)t * lstride + l] = R[l2 * NP + t];
    }
  }
}

template <typename T, int DIR, bool SOLVE, int PPT = 0, int DCT = 0>
__global__ void __launch_bounds__(256) k_fft_lines(FftPlan P, cpx<T>* data, int nl, int64_t lstride, int64_t ostride,
                                                   int L, const double* twd, const float* twf, const double* lamx,
                                                   const double* lamy, const double* lamz, double norm,
                                                   const double* dtp, double hg, const double* twcd,
                                                   const float* twcf) {
  fft_lines_body<T, DIR, SOLVE, PPT, DCT>(blockIdx, P, data, nl, lstride, ostride, L, twd, twf, lamx, lamy, lamz, norm,
                                          dtp, hg, twcd, twcf);
}

// Batched y transforms (SOLVE = false) or periodic-z spectral solve (SOLVE = true).
template <typename T, int DIR, bool SOLVE>
__global__ void __launch_bounds__(256) kb_fft_lines(BatchMap m) {
  int box;
  const dim3 bid = batch_bid(m, SOLVE ? BK_FFTZ : BK_FFTY, blockIdx.x, box);
  const BoxDesc& d = m.desc[box];
  const int nxh = d.g.nx / 2 + 1;
  if (SOLVE)
    fft_lines_body<T, DIR, true>(bid, d.pz, (cpx<T>*)d.spec, nxh, (int64_t)d.g.nxp * d.g.ny, (int64_t)d.g.nxp, d.lz, d.twz,
                                 d.twz_f, d.lamx, d.lamy, d.lamz, 1.0 / ((double)d.g.nx * d.g.ny * d.g.nz));
  else
    fft_lines_body<T, DIR, false>(bid, d.py, (cpx<T>*)d.spec, nxh, (int64_t)d.g.nxp, (int64_t)d.g.nxp * d.g.ny, d.ly,
                                  d.twy, d.twy_f, d.lamx, d.lamy, d.lamz, 1.0);
}

// Factorisation of the z systems of every (l, m) column (Sec. 2.2: one tridiagonal system
// per wavenumber pair), once per grid: the Poisson matrix depends on the geometry only, so
// c'_k = c_k / p_k and 1/p_k, p_k = b_k + lambda_x(l) + lambda_y(m) - a_k c'_{k-1}, are kept
// in the workspace ([k][m][l] pairs, FP64) for m <= ny/2; mode ny - m has the same
// eigenvalue and reads the pairs of m.
__global__ void __launch_bounds__(256) k_thomas_factor(GridP g, const double* __restrict__ pa,
                                                       const double* __restrict__ pb, const double* __restrict__ pc,
                                                       const double* __restrict__ lamx,
                                                       const double* __restrict__ lamy, double2* __restrict__ pfac) {
  const int nxh = g.nx / 2 + 1;
  const int64_t ncol = (int64_t)g.nxp * factor_modes(g);   // l >= nx/2+1 are padding
  const int64_t col = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  const int l = (int)(col % g.nxp), m = (int)(col / g.nxp);
  if (l >= nxh) return;
  const double lam = lamx[l] + lamy[m];
  // the singular (0, 0) column pins its last unknown: rows 0..nz-2 factorised, the last row
  // stored as (0, 0) so that the solve returns x = 0 there
  const int nr = col == 0 ? g.nz - 1 : g.nz;
  double cprev = 0.0;
  for (int k = 0; k < nr; ++k) {
    const double a = pa[k];
    const double rr = 1.0 / ((pb[k] + lam) - a * cprev);
    const double cc = pc[k] * rr;
    pfac[(int64_t)k * ncol + col] = make_double2(cc, rr);
    cprev = cc;
  }
  if (nr < g.nz) pfac[(int64_t)nr * ncol + col] = make_double2(0.0, 0.0);
}

void launch_thomas_factor(Ctx& c) {
  const int64_t ncol = (int64_t)c.g.nxp * factor_modes(c.g);
  hipLaunchKernelGGL(k_thomas_factor, dim3((unsigned)((ncol + 255) / 256)), dim3(256), 0, c.stream, c.g, c.t.pa,
                     c.t.pb, c.t.pc, c.t.lamx, c.t.lamy, (double2*)c.t.pfac);
}

// Launch shape of the chain solves of n rows (nchain chains over all components): segments of
// S rows (8 up to s8 rows, else 16), P segments per block, CG chains per segment: 64 (a wave
// per segment, 512 contiguous bytes of each FP64 row) while P <= 16 and the launch still has
// four blocks per CU, else 32 (nz <= 512).
struct ThomasShape {
  int S, CG, P;
};
inline ThomasShape thomas_shape(int n, int s8, int64_t nchain) {
  const int S = n <= s8 ? 8 : 16, P = (n + S - 1) / S;
  return {S, P <= 16 && nchain / 64 >= 4 * 256 ? 64 : 32, P};
}

// FP64 z solves of every (l, m) column with the stored factors, by segmented scans
// (seg_scan_solve).  A column gives two chains (real and imaginary parts), and there are only
// a few tens of thousands of chains of nz rows: a plain Thomas sweep per chain leaves most of
// the chip idle behind its dependent chain.  Threads: CG consecutive chains (adjacent in
// memory, so each row load of a segment group is contiguous) times the segments of S rows.
// Rows are held in registers, loaded once and stored once.  ZERO (Poisson): the pinned (0, 0) column
// has its own factor pairs (last row zero); its dzf-weighted mean is removed here and its
// imaginary part set to zero.  Rows nrow..nz-1 are left as they are (the wall face of w in
// the Helmholtz solves).
template <typename T, int S, int CG, bool ZERO>
__device__ __forceinline__ void thomas_scan_body(unsigned bx, GridP g, cpx<T>* __restrict__ spec,
                                                 const double* __restrict__ pa, const double2* __restrict__ pfac,
                                                 double norm, int nrow) {
  __shared__ double E[1024 / CG][CG], G[1024 / CG][CG];
  // with CG a multiple of the wave size a wave holds one segment, whose a_k are then
  // wave-uniform (scalar loads)
  const int cl = (int)threadIdx.x % CG, P = (int)blockDim.x / CG;
  const int p = CG % 64 == 0 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / CG) : (int)threadIdx.x / CG;
  const int n = nrow, nxh = g.nx / 2 + 1;
  const int64_t ncol = (int64_t)g.nxp * g.ny, ncol2 = 2 * ncol;
  const int64_t c2 = (int64_t)bx * CG + cl;
  const int64_t col = c2 >> 1;
  const int l = (int)(col % g.nxp), m = (int)(col / g.nxp);
  const bool ok = c2 < ncol2 && l < nxh;
  // periodic y: mode ny - m uses the pairs of m; ducts: every m has its own
  const int mm = (g.ywall || m <= g.ny / 2) ? m : g.ny - m;
  const int64_t nfac = (int64_t)g.nxp * factor_modes(g);
  const double2* fp = pfac + (ok ? (int64_t)mm * g.nxp + l : 0);
  T* x = reinterpret_cast<T*>(spec) + (ok ? c2 : 0);
  const int k0 = p * S;
  double v[S];
  double2 fc[S];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int k = k0 + j;
    const bool in = ok && k < n;
    v[j] = in ? (double)x[(int64_t)k * ncol2] * norm : 0.0;
    fc[j] = in ? fp[(int64_t)k * nfac] : make_double2(0.0, 0.0);
  }
  // a_k: scalar loads when a wave holds one segment; else (two segments per wave) from a copy
  // in LDS, read where used rather than held in registers (the 16-row variant spilled)
  __shared__ double sa[CG % 64 == 0 ? 1 : 512];
  if constexpr (CG % 64 != 0) {
    for (int k = (int)threadIdx.x; k < n; k += (int)blockDim.x) sa[k] = pa[k];
    __syncthreads();
  }
  auto AF = [&](int j) -> double {
    if constexpr (CG % 64 == 0) return pa[k0 + j];
    else return sa[k0 + j];
  };
  seg_scan_solve<S, CG>(v, k0, n, p, P, cl, E, G, [&](int j) { return fc[j].y; }, AF, [&](int j) { return fc[j].x; });
  if (ZERO && bx == 0) {
    // zero mode: chains 0 (real part) and 1 (imaginary part) of this block
    double sw = 0.0, sd = 0.0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int k = k0 + j;
      if (k < n) {
        sw += v[j] * g.dzf[k + 1];
        sd += g.dzf[k + 1];
      }
    }
    __syncthreads();
    if (cl == 0) {
      E[p][0] = sw;
      G[p][0] = sd;
    }
    __syncthreads();
    if (cl == 0) {
      double tw = 0.0, td = 0.0;
      for (int q = 0; q < P; ++q) {
        tw += E[q][0];
        td += G[q][0];
      }
      const double mean = tw / td;
#pragma unroll
      for (int j = 0; j < S; ++j) v[j] -= mean;
    } else if (cl == 1) {
#pragma unroll
      for (int j = 0; j < S; ++j) v[j] = 0.0;
    }
  }
  if (ok) {
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int k = k0 + j;
      if (k < n) x[(int64_t)k * ncol2] = (T)v[j];
    }
  }
}

template <typename T, int S, int CG, bool ZERO>
__global__ void __launch_bounds__(1024) k_thomas_scan(GridP g, cpx<T>* __restrict__ spec, const double* __restrict__ pa,
                                                      const double2* __restrict__ pfac, double norm, int nrow) {
  thomas_scan_body<T, S, CG, ZERO>(blockIdx.x, g, spec, pa, pfac, norm, nrow);
}

// ---------------------------------------------------------------- three components at once
// The Helmholtz solves of CN in all directions transform u*, v* and w* through three spectrum
// buffers (cstride apart), so each stage is one launch over all components (blockIdx.y or z).
template <typename T>
__global__ void __launch_bounds__(256) k_rfftx3(GridP g, FftPlan P, const T* us, const T* vs, const T* ws,
                                                cpx<T>* spec, int64_t cstride, const double* twd, const float* twf,
                                                int npair_blk) {
  const int comp = blockIdx.y;
  const T* f = comp == 0 ? us : (comp == 1 ? vs : ws);
  rfftx_body<T, 1>(dim3(blockIdx.x), g, P, nullptr, nullptr, nullptr, f, spec + comp * cstride, twd, twf, nullptr,
                   1.0, npair_blk, nullptr);
}

template <typename T>
__global__ void __launch_bounds__(256) k_irfftx3(GridP g, FftPlan P, const cpx<T>* spec, int64_t cstride, T* us,
                                                 T* vs, T* ws, const double* twd, const float* twf, int npair_blk) {
  const int comp = blockIdx.y;
  T* f = comp == 0 ? us : (comp == 1 ? vs : ws);
  irfftx_body<T>(dim3(blockIdx.x), g, P, spec + comp * cstride, f, twd, twf, npair_blk);
}

template <typename T, int DIR, bool SOLVE, int PPT = 0>
__global__ void __launch_bounds__(256) k_fft_lines3(FftPlan P, cpx<T>* data, int64_t cstride, int nl, int64_t lstride,
                                                    int64_t ostride, int L, const double* twd, const float* twf,
                                                    const double* lamx, const double* lamy, const double* lamz,
                                                    double norm, const double* dtp, double hg) {
  fft_lines_body<T, DIR, SOLVE, PPT>(dim3(blockIdx.x, blockIdx.y), P, data + blockIdx.z * cstride, nl, lstride, ostride,
                                     L, twd, twf, lamx, lamy, lamz, norm, dtp, hg);
}

// component blockIdx.y: u and v take the u/v rows and factors, w the w rows (nz - 1 unknowns)
template <typename T, int S, int CG>
__global__ void __launch_bounds__(1024) k_thomas_scan3(GridP g, cpx<T>* __restrict__ spec, int64_t cstride,
                                                       const double* __restrict__ a_uv, const double* __restrict__ a_w,
                                                       const double2* __restrict__ fac_uv,
                                                       const double2* __restrict__ fac_w, double norm) {
  const int comp = blockIdx.y;
  thomas_scan_body<T, S, CG, false>(blockIdx.x, g, spec + comp * cstride, comp < 2 ? a_uv : a_w,
                                comp < 2 ? fac_uv : fac_w, norm, comp < 2 ? g.nz : g.nz - 1);
}

// Crank-Nicolson in all directions, wall-bounded z (Eq. onestar_imp3d): after FFTs in x and
// y, every (l, m) column holds the tridiagonal system with rows a_k, b_k - c (lamx(l) +
// lamy(m)), c_k (c = gamma nu dt / 2; a, b, c the CN-z rows of the component, wall folds
// included), solved in FP64.  The pivots depend on dt, so the factor pairs (c', 1/pivot) of
// this substep are formed here, once for the u/v rows and once for the w rows, for m <=
// ny/2 (mode ny - m has the same eigenvalue); the solves are k_thomas_scan.  One thread per
// (column, row set).
__global__ void __launch_bounds__(256) k_helm3d_factor(GridP g, const double* __restrict__ hfac,
                                                       const double* __restrict__ lamx,
                                                       const double* __restrict__ lamy,
                                                       const double* __restrict__ dtp, double hg,
                                                       double2* __restrict__ fac) {
  const int nxh = g.nx / 2 + 1, n = g.nz;
  const int64_t nfac = (int64_t)g.nxp * (g.ny / 2 + 1);
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 2 * nfac) return;
  const int w = t >= nfac;
  const int64_t col = w ? t - nfac : t;
  const int l = (int)(col % g.nxp), m = (int)(col / g.nxp);
  if (l >= nxh) return;
  const double shift = hg * dtp[0] * (lamx[l] + lamy[m]);
  const double* ra = hfac + (w ? 7 : 6) * n;
  const double* rb = hfac + (w ? 10 : 8) * n;
  const double* rc = hfac + (w ? 11 : 9) * n;
  double2* f = fac + (w ? (int64_t)n * nfac : 0) + col;
  const int nr = w ? n - 1 : n;
  double cprev = 0.0;
  for (int k = 0; k < nr; ++k) {
    const double r = 1.0 / ((rb[k] - shift) - ra[k] * cprev);
    cprev = rc[k] * r;
    f[(int64_t)k * nfac] = make_double2(cprev, r);
  }
}

// ============================================================================ bulk
// s = (U_b - <u*>) / <q>, <.> the dzf-weighted volume mean; stored in dt[1].  One block:
// strided partial sums per thread, then a fixed-order tree (deterministic).
struct BulkArgs {
  const double* part;
  int nblk;
  double* dtp;
  const double* q;
  const double* dzf;
  int nz;
  double ubulk, cells_xy, lz;
};

// sm: 3 x 256 doubles of LDS (the dynamic buffer of the transform it runs beside)
__device__ __forceinline__ void bulk_final_body(const BulkArgs& a_, double (*sm)[256]) {
  const double* part = a_.part;
  const int nblk = a_.nblk, nz = a_.nz;
  const double* q = a_.q;
  const double* dzf = a_.dzf;
  double a = 0.0, b = 0.0, d = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) a += part[i];
  for (int k = threadIdx.x; k < nz; k += 256) {
    b += q[k] * dzf[k + 1];
    d += dzf[k + 1];
  }
  sm[0][threadIdx.x] = a;
  sm[1][threadIdx.x] = b;
  sm[2][threadIdx.x] = d;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int r = 0; r < 3; ++r) sm[r][threadIdx.x] += sm[r][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = sm[0][0] / (a_.cells_xy * a_.lz);
    a_.dtp[1] = (a_.ubulk - mean) / (sm[1][0] / sm[2][0]);
  }
}

// Forward y transform with the flow-rate shift folded in: block (0, 0), dispatched first,
// forms s from the forward-x partials while the others transform (plane = blockIdx.y - 1).
template <typename T, int PPT = 0, int DCT = 0>
__global__ void __launch_bounds__(256) k_ffty_bulk(FftPlan P, cpx<T>* data, int nl, int64_t lstride, int64_t ostride,
                                                   int L, const double* twd, const float* twf, const double* lamx,
                                                   const double* lamy, const double* lamz, BulkArgs ba,
                                                   const double* twcd, const float* twcf) {
  if (blockIdx.y == 0) {
    extern __shared__ unsigned char smem_raw[];
    if (blockIdx.x == 0) bulk_final_body(ba, reinterpret_cast<double(*)[256]>(smem_raw));
    return;
  }
  fft_lines_body<T, -1, false, PPT, DCT>(dim3(blockIdx.x, blockIdx.y - 1), P, data, nl, lstride, ostride, L, twd, twf,
                                         lamx, lamy, lamz, 1.0, nullptr, 0.0, twcd, twcf);
}

// ghost planes of a cell-centred scalar (Neumann walls or periodic copies)
template <typename T>
__global__ void k_scalar_ghosts(GridP g, T* f) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= g.sxy) return;
  const int64_t s = g.sxy, n = g.nz;
  if (g.zbc == LES_ZBC_PERIODIC) {
    f[c] = f[n * s + c];
    f[(n + 1) * s + c] = f[s + c];
  } else {
    f[c] = f[s + c];
    f[(n + 1) * s + c] = f[n * s + c];
  }
}

// ============================================================================ launchers
// Transforms per 256-thread block: a power of two (so the block splits into equal teams)
// with at most 1024 complex points per buffer (two buffers: <= 32 KiB in double; larger
// tiles measured slower on the channel workload).
static int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
static int pairs_per_block(int nx) {
  // rows of 256 points and more: two row pairs per block (measured faster than four on the
  // 256 x 128 x 96 channel; shorter rows keep up to eight)
  int p = pow2_floor(std::max(1, (nx >= 256 ? 512 : 1024) / nx));
  return std::min(p, 8);
}
static int lines_per_block(int n) {
  int L = pow2_floor(std::max(1, 1024 / n));
  return std::min(L, 32);
}

// Line groups of the single-field strided transforms: the ping-pong form (two buffers of
// L <= 1024 / n lines), unless its row segments of L consecutive l stay under 128 bytes (one
// cache line; long lines); then the in-place form with up to four times the lines (L n <=
// 4096, one buffer within 64 KB), ppt = L n / 256 points per thread rounded up to 8 or 16.
struct LineShape {
  int L, ppt;      // ppt 0: ping-pong
  size_t sh;       // dynamic LDS bytes
};
static LineShape line_shape(int n, size_t esz) {
  const int Lpp = lines_per_block(n);
  if ((size_t)Lpp * esz >= 128 || n > 4096) return {Lpp, 0, 2 * (size_t)Lpp * (n + 1) * esz};
  int L = Lpp;
  while (L < 32 && (size_t)(2 * L) * n <= 4096 && (size_t)(2 * L) * (n + 1) * esz <= 65536) L *= 2;
  const int ppt = L * n / 256 <= 8 ? 8 : 16;
  return {L, ppt, (size_t)L * (n + 1) * esz};
}

template <typename T>
static void fwd_x(Ctx& c, int mode, const T* us, const T* vs, const T* ws, const T* fin, double gamma, bool bulk) {
  const FftPlan P = make_plan(c.g.nx);
  const int pb = pairs_per_block(c.g.nx);
  const int64_t npairs = (int64_t)c.g.nz * (c.g.ny / 2);
  const unsigned nblk = (unsigned)((npairs + pb - 1) / pb);
  const size_t sh = 2 * (size_t)pb * c.g.nx * sizeof(cpx<T>);
  double* bp = bulk ? c.t.bulk : nullptr;
  const double spec_bytes = (double)(c.g.nx / 2 + 1) * c.g.ny * c.g.nz * 2 * sizeof(T);
  const double in_bytes = (mode == 0 ? 3.0 : 1.0) * c.g.sxy * c.g.nz * sizeof(T);
  if (mode == 0)
    LES_LAUNCH(c, "rfftx_div", in_bytes + spec_bytes, (k_rfftx<T, 0>), dim3(nblk), dim3(256), sh, c.g, P, us, vs, ws, fin,
                       (cpx<T>*)c.spec, c.t.twx, c.t.twx_f, c.t.dt, gamma, pb, bp);
  else
    LES_LAUNCH(c, "rfftx", in_bytes + spec_bytes, (k_rfftx<T, 1>), dim3(nblk), dim3(256), sh, c.g, P, us, vs, ws, fin,
                       (cpx<T>*)c.spec, c.t.twx, c.t.twx_f, c.t.dt, gamma, pb, bp);
  // the flow-rate shift is formed by an extra block of the forward y transform that follows
  c.bulk_nblk = bulk ? (int)nblk : 0;
}

// y transforms of the spectrum buffer (DIR -1 forward, +1 inverse)
template <typename T, int DIR, bool SOLVE, int DCT = 0>
static decltype(&k_fft_lines<T, DIR, SOLVE, 0, DCT>) lines_kernel(int ppt) {
  return ppt == 0 ? k_fft_lines<T, DIR, SOLVE, 0, DCT>
                  : (ppt == 8 ? k_fft_lines<T, DIR, SOLVE, 8, DCT> : k_fft_lines<T, DIR, SOLVE, 16, DCT>);
}
template <typename T, int DIR, bool SOLVE>
static decltype(&k_fft_lines3<T, DIR, SOLVE, 0>) lines3_kernel(int ppt) {
  return ppt == 0 ? k_fft_lines3<T, DIR, SOLVE, 0>
                  : (ppt == 8 ? k_fft_lines3<T, DIR, SOLVE, 8> : k_fft_lines3<T, DIR, SOLVE, 16>);
}

template <typename T, int DIR>
static void ffty(Ctx& c, const char* name) {
  const int nxh = c.g.nx / 2 + 1;
  const int ny = c.g.ny, nz = c.g.nz;
  const double spec_bytes = (double)nxh * ny * nz * 2 * sizeof(T);
  const FftPlan P = make_plan(ny);
  const LineShape ls = line_shape(ny, sizeof(cpx<T>));
  const int L = ls.L;
  dim3 grid((nxh + L - 1) / L, nz);
  // ducts: the cosine transform of the wall-bounded y direction
  auto kern = c.g.ywall ? lines_kernel<T, DIR, false, 1>(ls.ppt) : lines_kernel<T, DIR, false, 0>(ls.ppt);
  LES_LAUNCH(c, name, 2 * spec_bytes, kern, grid, dim3(256), ls.sh, P, (cpx<T>*)c.spec, nxh, (int64_t)c.g.nxp,
             (int64_t)c.g.nxp * ny, L, c.t.twy, c.t.twy_f, c.t.lamx, c.t.lamy, c.t.lamz, 1.0, nullptr, 0.0, c.t.twc,
             c.t.twc_f);
}

// periodic z: FFT, divide by the operator's eigenvalue, inverse FFT (hg = 0: Poisson)
template <typename T>
static void fftz_solve(Ctx& c, const char* name, double hg) {
  const int nxh = c.g.nx / 2 + 1;
  const int ny = c.g.ny, nz = c.g.nz;
  const double spec_bytes = (double)nxh * ny * nz * 2 * sizeof(T);
  const FftPlan P = make_plan(nz);
  const LineShape ls = line_shape(nz, sizeof(cpx<T>));
  const int L = ls.L;
  dim3 grid((nxh + L - 1) / L, ny);
  const double norm = 1.0 / ((double)c.g.nx * ny * nz);
  LES_LAUNCH(c, name, 2 * spec_bytes, (lines_kernel<T, -1, true>(ls.ppt)), grid, dim3(256), ls.sh, P,
             (cpx<T>*)c.spec, nxh, (int64_t)c.g.nxp * ny, (int64_t)c.g.nxp, L, c.t.twz, c.t.twz_f, c.t.lamx, c.t.lamy,
             c.t.lamz, norm, c.t.dt, hg, (const double*)nullptr, (const float*)nullptr);
}

template <typename T>
static void spectral_solve(Ctx& c) {
  const int nxh = c.g.nx / 2 + 1;
  const int ny = c.g.ny, nz = c.g.nz;
  cpx<T>* sp = (cpx<T>*)c.spec;
  const double spec_bytes = (double)nxh * ny * nz * 2 * sizeof(T);
  if (c.bulk_nblk > 0) {
    const FftPlan P = make_plan(ny);
    const LineShape ls = line_shape(ny, sizeof(cpx<T>));
    const int L = ls.L;
    dim3 grid((nxh + L - 1) / L, nz + 1);
    const size_t sh = std::max(ls.sh, 3 * 256 * sizeof(double));
    const BulkArgs ba{c.t.bulk, c.bulk_nblk, c.t.dt, c.t.hfac + 4 * nz, c.t.dzf, nz, c.cfg.ubulk,
                      (double)c.g.nx * c.g.ny, c.cfg.lz};
    auto kern = c.g.ywall ? (ls.ppt == 0 ? k_ffty_bulk<T, 0, 1> : (ls.ppt == 8 ? k_ffty_bulk<T, 8, 1> : k_ffty_bulk<T, 16, 1>))
                          : (ls.ppt == 0 ? k_ffty_bulk<T, 0, 0> : (ls.ppt == 8 ? k_ffty_bulk<T, 8, 0> : k_ffty_bulk<T, 16, 0>));
    LES_LAUNCH(c, "ffty_fwd", 2 * spec_bytes, kern, grid, dim3(256), sh, P, sp, nxh, (int64_t)c.g.nxp,
               (int64_t)c.g.nxp * ny, L, c.t.twy, c.t.twy_f, c.t.lamx, c.t.lamy, c.t.lamz, ba, c.t.twc, c.t.twc_f);
    c.bulk_nblk = 0;
  } else {
    ffty<T, -1>(c, "ffty_fwd");
  }
  if (c.cfg.zbc == LES_ZBC_PERIODIC) {
    fftz_solve<T>(c, "fftz_solve", 0.0);
  } else {
    const int64_t nchain = 2 * (int64_t)c.g.nxp * ny;
    const ThomasShape sh = thomas_shape(nz, 32, nchain);
    const dim3 block(sh.CG * sh.P);
    const double norm = 1.0 / ((double)c.g.nx * ny);
    const double bytes = 2 * spec_bytes + (double)nxh * factor_modes(c.g) * nz * 16;
    auto go = [&](auto kern, int64_t nb) {
      LES_LAUNCH(c, "thomas_z", bytes, kern, dim3((unsigned)nb), block, 0, c.g, sp, c.t.pa, (const double2*)c.t.pfac,
                 norm, nz);
    };
    if (sh.CG == 64)
      sh.S == 8 ? go(k_thomas_scan<T, 8, 64, true>, (nchain + 64 - 1) / 64)
                : go(k_thomas_scan<T, 16, 64, true>, (nchain + 64 - 1) / 64);
    else
      sh.S == 8 ? go(k_thomas_scan<T, 8, 32, true>, (nchain + 32 - 1) / 32)
                : go(k_thomas_scan<T, 16, 32, true>, (nchain + 32 - 1) / 32);
  }
  ffty<T, 1>(c, "ffty_inv");
}

template <typename T>
static void inv_x(Ctx& c, T* out) {
  const FftPlan P = make_plan(c.g.nx);
  const int pb = pairs_per_block(c.g.nx);
  const int64_t npairs = (int64_t)c.g.nz * (c.g.ny / 2);
  const unsigned nblk = (unsigned)((npairs + pb - 1) / pb);
  const size_t sh = 2 * (size_t)pb * c.g.nx * sizeof(cpx<T>);
  const double spec_bytes = (double)(c.g.nx / 2 + 1) * c.g.ny * c.g.nz * 2 * sizeof(T);
  LES_LAUNCH(c, "irfftx", spec_bytes + (double)c.g.sxy * c.g.nz * sizeof(T), (k_irfftx<T>), dim3(nblk), dim3(256), sh,
             c.g, P, (const cpx<T>*)c.spec, out,
                     c.t.twx, c.t.twx_f, pb);
}

// Crank-Nicolson in all directions (Eq. onestar_imp3d): the predicted components u*, v*, w*
// (right-hand sides of the Helmholtz systems, wall-model flux included) are transformed in x
// and y into three spectrum buffers, solved per wavenumber pair in z (Thomas in FP64 at
// walls, FFT when z is periodic) and transformed back in place; one launch per stage.
template <typename T>
void launch_helmholtz_3d(Ctx& c, int stage) {
  static const double G[3] = {8.0 / 15.0, 2.0 / 15.0, 1.0 / 3.0};
  const double hg = G[stage] * c.cfg.nu / 2.0;
  const int n = c.g.nz, nx = c.g.nx, ny = c.g.ny, nxh = nx / 2 + 1;
  const double spec_bytes = (double)nxh * ny * n * 2 * sizeof(T);
  const int64_t cstride = (int64_t)c.g.nxp * ny * n;   // complex values per component
  cpx<T>* sp = (cpx<T>*)c.spec;
  const int64_t nfac = (int64_t)c.g.nxp * (ny / 2 + 1);
  const double norm_xy = 1.0 / ((double)nx * ny);
  if (c.cfg.zbc != LES_ZBC_PERIODIC)
    LES_LAUNCH(c, "h3d_factor", 2.0 * nfac * n * 16, k_helm3d_factor, dim3((unsigned)((2 * nfac + 255) / 256)), dim3(256),
               0, c.g, c.t.hfac, c.t.lamx, c.t.lamy, c.t.dt, hg, (double2*)c.t.hfac3);
  // forward x of the three components
  {
    const FftPlan P = make_plan(nx);
    const int pb = pairs_per_block(nx);
    const int64_t npairs = (int64_t)n * (ny / 2);
    const size_t sh = 2 * (size_t)pb * nx * sizeof(cpx<T>);
    LES_LAUNCH(c, "h3d_rfftx", 3 * (spec_bytes + (double)c.g.sxy * n * sizeof(T)), (k_rfftx3<T>),
               dim3((unsigned)((npairs + pb - 1) / pb), 3), dim3(256), sh, c.g, P, (const T*)c.us, (const T*)c.vs,
               (const T*)c.wsf, sp, cstride, c.t.twx, c.t.twx_f, pb);
  }
  const FftPlan Py = make_plan(ny);
  const LineShape lsy = line_shape(ny, sizeof(cpx<T>));
  const int Ly = lsy.L;
  const dim3 gy((nxh + Ly - 1) / Ly, n, 3);
  LES_LAUNCH(c, "h3d_ffty_fwd", 6 * spec_bytes, (lines3_kernel<T, -1, false>(lsy.ppt)), gy, dim3(256), lsy.sh, Py, sp,
             cstride, nxh, (int64_t)c.g.nxp, (int64_t)c.g.nxp * ny, Ly, c.t.twy, c.t.twy_f, c.t.lamx, c.t.lamy,
             c.t.lamz, 1.0, nullptr, 0.0);
  if (c.cfg.zbc == LES_ZBC_PERIODIC) {
    const FftPlan Pz = make_plan(n);
    const LineShape lsz = line_shape(n, sizeof(cpx<T>));
    const int Lz = lsz.L;
    LES_LAUNCH(c, "h3d_fftz_solve", 6 * spec_bytes, (lines3_kernel<T, -1, true>(lsz.ppt)),
               dim3((nxh + Lz - 1) / Lz, ny, 3), dim3(256), lsz.sh, Pz, sp, cstride, nxh, (int64_t)c.g.nxp * ny,
               (int64_t)c.g.nxp, Lz, c.t.twz, c.t.twz_f, c.t.lamx, c.t.lamy, c.t.lamz, 1.0 / ((double)nx * ny * n),
               c.t.dt, hg);
  } else {
    const int64_t nchain = 2 * (int64_t)c.g.nxp * ny;
    const ThomasShape sh = thomas_shape(n, 128, 3 * nchain);
    const dim3 block(sh.CG * sh.P);
    const double* a_uv = c.t.hfac + 6 * n;
    const double* a_w = c.t.hfac + 7 * n;
    const double2* f_uv = (const double2*)c.t.hfac3;
    const double2* f_w = f_uv + (int64_t)n * nfac;
    const double bytes = 6 * spec_bytes + 3.0 * nfac * n * 16;
    auto go = [&](auto kern, int64_t nb) {
      LES_LAUNCH(c, "h3d_thomas_z", bytes, kern, dim3((unsigned)nb, 3), block, 0, c.g, sp, cstride, a_uv, a_w, f_uv,
                 f_w, norm_xy);
    };
    if (sh.CG == 64)
      sh.S == 8 ? go(k_thomas_scan3<T, 8, 64>, (nchain + 64 - 1) / 64)
                : go(k_thomas_scan3<T, 16, 64>, (nchain + 64 - 1) / 64);
    else
      sh.S == 8 ? go(k_thomas_scan3<T, 8, 32>, (nchain + 32 - 1) / 32)
                : go(k_thomas_scan3<T, 16, 32>, (nchain + 32 - 1) / 32);
  }
  LES_LAUNCH(c, "h3d_ffty_inv", 6 * spec_bytes, (lines3_kernel<T, 1, false>(lsy.ppt)), gy, dim3(256), lsy.sh, Py, sp,
             cstride, nxh, (int64_t)c.g.nxp, (int64_t)c.g.nxp * ny, Ly, c.t.twy, c.t.twy_f, c.t.lamx, c.t.lamy,
             c.t.lamz, 1.0, nullptr, 0.0);
  {
    const FftPlan P = make_plan(nx);
    const int pb = pairs_per_block(nx);
    const int64_t npairs = (int64_t)n * (ny / 2);
    const size_t sh = 2 * (size_t)pb * nx * sizeof(cpx<T>);
    LES_LAUNCH(c, "h3d_irfftx", 3 * (spec_bytes + (double)c.g.sxy * n * sizeof(T)), (k_irfftx3<T>),
               dim3((unsigned)((npairs + pb - 1) / pb), 3), dim3(256), sh, c.g, P, (const cpx<T>*)sp, cstride,
               (T*)c.us, (T*)c.vs, (T*)c.wsf, c.t.twx, c.t.twx_f, pb);
  }
}

template <typename T>
void launch_poisson_rhs_fwd(Ctx& c, const T* us, const T* vs, const T* ws, double gamma, int stage) {
  (void)stage;
  fwd_x<T>(c, 0, us, vs, ws, nullptr, gamma, c.cfg.ubulk > 0.0);
}

template <typename T>
void launch_poisson_solve_spectral(Ctx& c) {
  spectral_solve<T>(c);
}

template <typename T>
void launch_poisson_inverse(Ctx& c, T* phi_out) {
  inv_x<T>(c, phi_out);
}

template <typename T>
void launch_poisson_field(Ctx& c, T* f) {
  fwd_x<T>(c, 1, nullptr, nullptr, nullptr, f, 1.0, false);
  spectral_solve<T>(c);
  inv_x<T>(c, f);
  LES_LAUNCH(c, "scalar_ghosts", 4.0 * c.g.sxy * sizeof(T), k_scalar_ghosts<T>, dim3((unsigned)((c.g.sxy + 255) / 256)),
             dim3(256), 0, c.g, f);
  if (c.g.ywall) launch_fill_y_scalar<T>(c, f, 1.0);
}

// ============================================================================ initial projection
// One projection of the bound velocity with the substep's operators (Eqs. poi, correc without
// the time factor): phi solves D G phi = D u, u -= G phi; with a constant flow rate the
// streamwise velocity is then shifted uniformly so that its volume mean is U_b.  The interior
// cells are cut into PROJ_BLOCKS contiguous chunks, one block each, so that the flow-rate sum
// runs in a fixed order.
constexpr int PROJ_BLOCKS = 64;

template <typename T>
__global__ void __launch_bounds__(256) k_project_correct(GridP g, T* __restrict__ u, T* __restrict__ v,
                                                         T* __restrict__ w, const T* __restrict__ phi,
                                                         double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t nxy = (int64_t)g.nx * g.ny;
  const int64_t total = (int64_t)g.nz * nxy;
  const int64_t chunk = (total + PROJ_BLOCKS - 1) / PROJ_BLOCKS;
  const int64_t e0 = blockIdx.x * chunk, e1 = e0 + chunk < total ? e0 + chunk : total;
  const bool walls = g.zbc != LES_ZBC_PERIODIC;
  double su = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int k = (int)(e / nxy) + 1;
    const int64_t r = e % nxy;
    const int i = (int)(r % g.nx), j = (int)(r / g.nx);
    const int64_t c = idx3(g, k, j, i);
    const T ph = phi[c];
    const T un = u[c] - (phi[idx3(g, k, j, wrap_p(i, g.nx))] - ph) * (T)g.rdx;
    u[c] = un;
    // the y wall face y = ly of a duct (row ny - 1) and the z wall face on top stay at rest
    v[c] = (g.ywall && j == g.ny - 1) ? (T)0 : v[c] - (phi[idx3(g, k, wrap_p(j, g.nys), i)] - ph) * (T)g.rdy;
    w[c] = (walls && k == g.nz) ? (T)0 : w[c] - (phi[c + g.sxy] - ph) * (T)g.rdzc[k];
    su += (double)un * g.dzf[k];
  }
  red[threadIdx.x] = su;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// u += U_b - <u> on every interior cell; each block sums the chunk partials in block order.
template <typename T>
__global__ void __launch_bounds__(256) k_project_shift(GridP g, T* __restrict__ u, const double* __restrict__ part,
                                                       double ubulk, double lz) {
  __shared__ double shift;
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int b = 0; b < PROJ_BLOCKS; ++b) a += part[b];
    shift = ubulk - a / ((double)g.nx * g.ny * lz);
  }
  __syncthreads();
  const T s = (T)shift;
  const int64_t nxy = (int64_t)g.nx * g.ny;
  const int64_t total = (int64_t)g.nz * nxy;
  const int64_t chunk = (total + PROJ_BLOCKS - 1) / PROJ_BLOCKS;
  const int64_t e0 = blockIdx.x * chunk, e1 = e0 + chunk < total ? e0 + chunk : total;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int k = (int)(e / nxy) + 1;
    const int64_t r = e % nxy;
    u[(int64_t)k * g.sxy + r] += s;
  }
}

template <typename T>
void launch_project(Ctx& c) {
  T* u = (T*)c.u;
  T* v = (T*)c.v;
  T* w = (T*)c.w;
  T* phi = (T*)c.phi;
  launch_bc_fill<T>(c, u, v, w, (T*)c.p);   // wall faces of w (and the periodic copies)
  if (c.g.ywall) launch_bc_fill_y<T>(c, u, v, w, (T*)c.p);
  fwd_x<T>(c, 0, u, v, w, nullptr, 0.0, false);
  spectral_solve<T>(c);
  inv_x<T>(c, phi);
  LES_LAUNCH(c, "scalar_ghosts", 4.0 * c.g.sxy * sizeof(T), k_scalar_ghosts<T>, dim3((unsigned)((c.g.sxy + 255) / 256)),
             dim3(256), 0, c.g, phi);
  if (c.g.ywall) launch_fill_y_scalar<T>(c, phi, 1.0);
  const double cells = (double)c.g.nx * c.g.ny * c.g.nz;
  LES_LAUNCH(c, "project_correct", 7.0 * cells * sizeof(T), k_project_correct<T>, dim3(PROJ_BLOCKS), dim3(256), 0,
             c.g, u, v, w, (const T*)phi, c.t.red);
  if (c.cfg.ubulk > 0.0)
    LES_LAUNCH(c, "project_shift", 2.0 * cells * sizeof(T), k_project_shift<T>, dim3(PROJ_BLOCKS), dim3(256), 0, c.g,
               u, (const double*)c.t.red, c.cfg.ubulk, c.cfg.lz);
}

// ============================================================================ batch launchers
template <typename T>
void batch_poisson(hipStream_t st, const BatchMap& m, const int* totals, size_t sh_x, size_t sh_y, size_t sh_z,
                   int stage) {
  static const double G[3] = {8.0 / 15.0, 2.0 / 15.0, 1.0 / 3.0};
  hipLaunchKernelGGL(kb_rfftx<T>, dim3(totals[BK_RFFTX]), dim3(256), sh_x, st, m, G[stage]);
  hipLaunchKernelGGL((kb_fft_lines<T, -1, false>), dim3(totals[BK_FFTY]), dim3(256), sh_y, st, m);
  hipLaunchKernelGGL((kb_fft_lines<T, -1, true>), dim3(totals[BK_FFTZ]), dim3(256), sh_z, st, m);
  hipLaunchKernelGGL((kb_fft_lines<T, 1, false>), dim3(totals[BK_FFTY]), dim3(256), sh_y, st, m);
  hipLaunchKernelGGL(kb_irfftx<T>, dim3(totals[BK_RFFTX]), dim3(256), sh_x, st, m);
}
template void batch_poisson<float>(hipStream_t, const BatchMap&, const int*, size_t, size_t, size_t, int);
template void batch_poisson<double>(hipStream_t, const BatchMap&, const int*, size_t, size_t, size_t, int);

int fft_pairs_per_block(int nx) { return pairs_per_block(nx); }
int fft_lines_per_block(int n) { return lines_per_block(n); }

#define INST(T)                                                                              \
  template void launch_poisson_rhs_fwd<T>(Ctx&, const T*, const T*, const T*, double, int); \
  template void launch_poisson_solve_spectral<T>(Ctx&);                                      \
  template void launch_poisson_inverse<T>(Ctx&, T*);                                         \
  template void launch_poisson_field<T>(Ctx&, T*);                                          \
  template void launch_project<T>(Ctx&);                                                     \
  template void launch_helmholtz_3d<T>(Ctx&, int);
INST(double)
INST(float)

}  // namespace les
