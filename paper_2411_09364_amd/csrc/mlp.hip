// Learned Smagorinsky-coefficient closure: 7 -> 64 -> 64 -> 1 perceptron with SiLU.
//
// The paper motivates SGS closures trained on data produced by the LES solver itself
// (Sec. 1); the network, its features and the fallback to the dynamic model are this
// library's design.  Matrix products run on the matrix cores in bfloat16 with float32
// accumulation (v_mfma_f32_16x16x16_bf16); biases, SiLU, the 64 -> 1 output layer and all
// gradient reductions are float32.
//
// Products are computed transposed: Z1^T = W1 X^T and Z2^T = W2 H1^T with the weights as
// the A operand.  The accumulator layout of a 16x16 tile (lane l holds rows 4(l/16)+i,
// column l%16) is then exactly the B-operand layout of the next product, so the forward
// pass keeps activations in registers.  Contractions over samples (weight gradients) go
// through a per-wave transpose in LDS.
//
// Parameter vector (float32, 4737): W1[64][7] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.
#include "mlp_core.h"

#include <mutex>

namespace les {
namespace mlp {

// ============================================================================ inference
// y = MLP(x) for normalised features x[n][7] (float32).
__global__ void __launch_bounds__(NT) k_mlp_forward(const float* __restrict__ P, const float* __restrict__ x,
                                                    int64_t n, float* __restrict__ y) {
  __shared__ Weights W;
  __shared__ unsigned short xs[WAVES][64 * FP];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  load_weights(P, W, tid, NT);
  const int64_t s0 = ((int64_t)blockIdx.x * WAVES + wave) * 64;
  const int64_t s = s0 + lane;
  for (int f = 0; f < FP; ++f) xs[wave][lane * FP + f] = (f < F && s < n) ? f2bf(x[s * F + f]) : (unsigned short)0;
  __syncthreads();
  Fwd o;
  forward_wave<false>(W, xs[wave], lane, o);
  if (lane < 16)
    for (int sb = 0; sb < 4; ++sb) {
      const int64_t q = s0 + 16 * sb + lane;
      if (q < n) y[q] = o.y[sb];
    }
}

// ============================================================================ training
// Per-block partial gradients of L = mean((y - t)^2) (plus the partial sum of squared
// errors in slot NPARAM) over the block's chunks of 256 samples; x is normalised.
// Rounding points follow forward_wave; dz2 and dz1 are rounded to bf16 for the products.
__global__ void __launch_bounds__(NT) k_mlp_grad(const float* __restrict__ P, const float* __restrict__ x,
                                                 const float* __restrict__ t, int64_t n, float* __restrict__ part) {
  __shared__ Weights W;
  __shared__ unsigned short w2t[H * LD2];             // W2^T, rows padded like W2
  __shared__ unsigned short xs[WAVES][64 * FP];
  __shared__ unsigned short tr[WAVES][2][H * LD2];  // transposes: [0] dz2b or dz1b, [1] h1b (rows padded)
  __shared__ float acc[NPARAM + 1];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int r16 = lane % 16, g4 = 4 * (lane / 16);
  load_weights(P, W, tid, NT);
  for (int e = tid; e < H * H; e += NT) w2t[(e % H) * LD2 + e / H] = f2bf(P[P_W2 + e]);
  for (int e = tid; e < NPARAM + 1; e += NT) acc[e] = 0.f;
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  f4 gW2[4][4], gW1[4];
  for (int a = 0; a < 4; ++a) {
    gW1[a] = zero;
    for (int b = 0; b < 4; ++b) gW2[a][b] = zero;
  }
  float gb1[4][4], gb2[4][4], gw3[4][4];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 4; ++i) gb1[a][i] = gb2[a][i] = gw3[a][i] = 0.f;
  float gb3 = 0.f, sse = 0.f;
  const float inv_n = 1.0f / (float)n;
  const int64_t nchunk = (n + NT - 1) / NT;
  __syncthreads();
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int64_t s0 = ch * NT + (int64_t)wave * 64;
    const int64_t s = s0 + lane;
    for (int f = 0; f < FP; ++f) xs[wave][lane * FP + f] = (f < F && s < n) ? f2bf(x[s * F + f]) : (unsigned short)0;
    __syncthreads();
    Fwd o;
    forward_wave<true>(W, xs[wave], lane, o);
    float dy[4];
    for (int sb = 0; sb < 4; ++sb) {
      const int64_t q = s0 + 16 * sb + r16;
      const bool ok = q < n;
      const float e = ok ? o.y[sb] - t[q] : 0.f;
      dy[sb] = 2.0f * e * inv_n;
      if (lane < 16) {
        sse += e * e;
        gb3 += dy[sb];
      }
    }
    // output layer and dz2
    s4 dz2b[4][4];
    for (int a = 0; a < 4; ++a)
      for (int sb = 0; sb < 4; ++sb) {
        float d[4];
        for (int i = 0; i < 4; ++i) {
          const int h = 16 * a + g4 + i;
          gw3[a][i] += dy[sb] * o.h2[a][sb][i];
          d[i] = W.w3[h] * dy[sb] * dsilu(o.z2[a][sb][i]);
          gb2[a][i] += d[i];
        }
        dz2b[a][sb] = pack4(d[0], d[1], d[2], d[3]);
      }
    // dH1^T = W2^T dZ2^T (B operand = dz2b registers), dz1 = dH1 * silu'(z1)
    s4 dz1b[4][4];
    for (int kb = 0; kb < 4; ++kb)
      for (int sb = 0; sb < 4; ++sb) {
        f4 d = zero;
        for (int a = 0; a < 4; ++a) d = mfma(lds4(&w2t[(16 * kb + r16) * LD2 + 16 * a + g4]), dz2b[a][sb], d);
        float z[4];
        for (int i = 0; i < 4; ++i) {
          z[i] = d[i] * dsilu(o.z1[kb][sb][i]);
          gb1[kb][i] += z[i];
        }
        dz1b[kb][sb] = pack4(z[0], z[1], z[2], z[3]);
      }
    // transposes: tr[0] = dz2b[row][sample], tr[1] = h1b[row][sample]
    unsigned short* T0 = tr[wave][0];
    unsigned short* T1 = tr[wave][1];
    for (int a = 0; a < 4; ++a)
      for (int sb = 0; sb < 4; ++sb) {
        const s4 v0 = dz2b[a][sb], v1 = o.h1b[a][sb];
        const short e0[4] = {v0.x, v0.y, v0.z, v0.w}, e1[4] = {v1.x, v1.y, v1.z, v1.w};
        for (int i = 0; i < 4; ++i) {
          T0[(16 * a + g4 + i) * LD2 + 16 * sb + r16] = (unsigned short)e0[i];
          T1[(16 * a + g4 + i) * LD2 + 16 * sb + r16] = (unsigned short)e1[i];
        }
      }
    __syncthreads();
    // dW2(out, in) += sum_s dz2b(out, s) h1b(in, s)
    for (int a = 0; a < 4; ++a)
      for (int kb = 0; kb < 4; ++kb)
        for (int sb = 0; sb < 4; ++sb)
          gW2[a][kb] = mfma(lds4(&T0[(16 * a + r16) * LD2 + 16 * sb + g4]), lds4(&T1[(16 * kb + r16) * LD2 + 16 * sb + g4]),
                            gW2[a][kb]);
    __syncthreads();
    // dW1(h, f) += sum_s dz1b(h, s) xb(s, f)
    for (int a = 0; a < 4; ++a)
      for (int sb = 0; sb < 4; ++sb) {
        const s4 v0 = dz1b[a][sb];
        const short e0[4] = {v0.x, v0.y, v0.z, v0.w};
        for (int i = 0; i < 4; ++i) T0[(16 * a + g4 + i) * LD2 + 16 * sb + r16] = (unsigned short)e0[i];
      }
    __syncthreads();
    for (int a = 0; a < 4; ++a)
      for (int sb = 0; sb < 4; ++sb) {
        s4 B;
        const unsigned short* xw = xs[wave];
        B.x = (short)xw[(16 * sb + g4 + 0) * FP + r16];
        B.y = (short)xw[(16 * sb + g4 + 1) * FP + r16];
        B.z = (short)xw[(16 * sb + g4 + 2) * FP + r16];
        B.w = (short)xw[(16 * sb + g4 + 3) * FP + r16];
        gW1[a] = mfma(lds4(&T0[(16 * a + r16) * LD2 + 16 * sb + g4]), B, gW1[a]);
      }
    __syncthreads();
  }
  // reduce per-lane partials over the 16 lanes of a group (fixed order) for the vectors
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 4; ++i)
      for (int off = 1; off < 16; off <<= 1) {
        gb1[a][i] += __shfl_xor(gb1[a][i], off, 64);
        gb2[a][i] += __shfl_xor(gb2[a][i], off, 64);
        gw3[a][i] += __shfl_xor(gw3[a][i], off, 64);
      }
  for (int off = 1; off < 16; off <<= 1) {
    gb3 += __shfl_xor(gb3, off, 64);
    sse += __shfl_xor(sse, off, 64);
  }
  // waves add into the block accumulator one after another (deterministic)
  for (int w = 0; w < WAVES; ++w) {
    if (wave == w) {
      for (int a = 0; a < 4; ++a)
        for (int kb = 0; kb < 4; ++kb)
          for (int i = 0; i < 4; ++i) acc[P_W2 + (16 * a + g4 + i) * H + 16 * kb + r16] += gW2[a][kb][i];
      if (r16 < F)
        for (int a = 0; a < 4; ++a)
          for (int i = 0; i < 4; ++i) acc[P_W1 + (16 * a + g4 + i) * F + r16] += gW1[a][i];
      if (r16 == 0)
        for (int a = 0; a < 4; ++a)
          for (int i = 0; i < 4; ++i) {
            const int h = 16 * a + g4 + i;
            acc[P_B1 + h] += gb1[a][i];
            acc[P_B2 + h] += gb2[a][i];
            acc[P_W3 + h] += gw3[a][i];
          }
      if (lane == 0) {
        acc[P_B3] += gb3;
        acc[NPARAM] += sse;
      }
    }
    __syncthreads();
  }
  float* out = part + (int64_t)blockIdx.x * (NPARAM + 1);
  for (int e = tid; e < NPARAM + 1; e += NT) out[e] = acc[e];
}

// Sum the block partials in block order: grad[p]; loss = sse / n.
__global__ void k_mlp_reduce(const float* __restrict__ part, int nblk, int64_t n, float* __restrict__ grad,
                             float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > NPARAM) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * (NPARAM + 1) + p];
  if (p < NPARAM) grad[p] = s;
  else if (loss) loss[0] = s / (float)n;
}

// Adam (Kingma & Ba) on the float32 master parameters; step is 1-based.
__global__ void k_mlp_adam(float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, int step, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.f - b1) * gi;
  const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  const float mh = mi / (1.f - powf(b1, (float)step));
  const float vh = vi / (1.f - powf(b2, (float)step));
  P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// x = (x_raw - lo) / (hi - lo) per feature (float32 in and out).
struct Norm7 {
  double lo[7], hi[7];
};
__global__ void k_mlp_normalize(const float* __restrict__ xr, int64_t n, Norm7 nm, float* __restrict__ x) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * F) return;
  const int a = (int)(e % F);
  x[e] = (float)(((double)xr[e] - nm.lo[a]) / (nm.hi[a] - nm.lo[a]));
}

}  // namespace mlp

// ============================================================================ host launchers
void launch_mlp_normalize(hipStream_t st, const float* xr, int64_t n, const double* lo, const double* hi, float* x) {
  mlp::Norm7 nm;
  for (int a = 0; a < 7; ++a) {
    nm.lo[a] = lo[a];
    nm.hi[a] = hi[a];
  }
  hipLaunchKernelGGL(mlp::k_mlp_normalize, dim3((unsigned)((n * 7 + 255) / 256)), dim3(256), 0, st, xr, n, nm, x);
}

int64_t mlp_grad_blocks(int64_t n) {
  const int64_t chunks = (n + mlp::NT - 1) / mlp::NT;
  return chunks < 1024 ? (chunks < 1 ? 1 : chunks) : 1024;
}

void launch_mlp_forward(hipStream_t st, const float* P, const float* x, int64_t n, float* y) {
  const int64_t nb = (n + mlp::NT - 1) / mlp::NT;
  hipLaunchKernelGGL(mlp::k_mlp_forward, dim3((unsigned)nb), dim3(mlp::NT), 0, st, P, x, n, y);
}

void launch_mlp_grad(hipStream_t st, const float* P, const float* x, const float* t, int64_t n, float* part,
                     float* grad, float* loss) {
  const int64_t nb = mlp_grad_blocks(n);
  hipLaunchKernelGGL(mlp::k_mlp_grad, dim3((unsigned)nb), dim3(mlp::NT), 0, st, P, x, t, n, part);
  hipLaunchKernelGGL(mlp::k_mlp_reduce, dim3((mlp::NPARAM + 1 + 255) / 256), dim3(256), 0, st, part, (int)nb, n, grad,
                     loss);
}

// ---------------------------------------------------------------- gradient without a workspace
// The block partials of k_mlp_grad live in a file-scope device array instead of a caller
// workspace.  Each device holds its own copy; its address is looked up once per device with
// that device current and kept here.  Host code never passes the array's name to a kernel: in
// host code that name is a stand-in, not a device address.
static __device__ __align__(256) float scratch[MLP_NOALLOC_BLOCKS * (mlp::NPARAM + 1)];
static_assert(MLP_NOALLOC_BLOCKS * mlp::NT >= LES_MLP_NOALLOC_MAX_SAMPLES, "one chunk per block up to the limit");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t mlp_scratch_ptr(int device, float** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = static_cast<float*>(p);
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

void launch_mlp_adam(hipStream_t st, float* P, const float* g, float* m, float* v, int step, float lr) {
  hipLaunchKernelGGL(mlp::k_mlp_adam, dim3((mlp::NPARAM + 255) / 256), dim3(256), 0, st, P, g, m, v, step, lr, 0.9f,
                     0.999f, 1e-8f);
}

}  // namespace les
