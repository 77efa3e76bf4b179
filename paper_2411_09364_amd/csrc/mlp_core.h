// Device building blocks of the learned-closure perceptron shared by the training kernels
// (mlp.hip) and the fused eddy-viscosity inference (sgs.hip).  See mlp.hip for the design.
#pragma once

#include "les_internal.h"

namespace les {
namespace mlp {

constexpr int H = 64, F = 7, FP = 16;
constexpr int P_W1 = 0, P_B1 = 448, P_W2 = 512, P_B2 = 4608, P_W3 = 4672, P_B3 = 4736, NPARAM = 4737;
constexpr int WAVES = 4, NT = 64 * WAVES;   // 4 waves of 64 samples per block

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even float32 -> bfloat16 bits
__device__ inline unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
// Logistic function from the hardware base-2 exponential and reciprocal (about 1 ulp each):
// sigma(z) = 1 / (1 + 2^(-z log2 e)); saturates to 0 and 1 without special cases.
__device__ inline float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}
__device__ inline float silu(float z) { return z * sigmoid(z); }
__device__ inline float dsilu(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}
__device__ inline f4 mfma(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
__device__ inline s4 lds4(const unsigned short* p) {
  const unsigned int* q = reinterpret_cast<const unsigned int*>(p);
  const unsigned int a = q[0], b = q[1];
  s4 r;
  r.x = (short)(a & 0xFFFF);
  r.y = (short)(a >> 16);
  r.z = (short)(b & 0xFFFF);
  r.w = (short)(b >> 16);
  return r;
}
// four float32 -> bfloat16 (round to nearest even) with the packed hardware conversion
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));
__device__ inline s4 pack4(float a, float b, float c, float d) {
  const fl2 lo = {a, b}, hi = {c, d};
  const unsigned int x = __builtin_bit_cast(unsigned int, __builtin_convertvector(lo, bf2));
  const unsigned int y = __builtin_bit_cast(unsigned int, __builtin_convertvector(hi, bf2));
  s4 r;
  r.x = (short)(x & 0xFFFF);
  r.y = (short)(x >> 16);
  r.z = (short)(y & 0xFFFF);
  r.w = (short)(y >> 16);
  return r;
}

// Weights staged once per block: bf16 W1 (padded to 16 features) and W2; float32 biases and
// output layer.  W2 rows are padded to LD2 = 72 halfwords: with 128-byte rows the 16 rows a
// matrix-core operand read touches (one per lane of a 16-lane group) would all start in one
// LDS bank; 144-byte rows spread them over the 32 banks.
constexpr int LD2 = H + 8;
struct alignas(16) Weights {
  unsigned short w1[H * FP];
  unsigned short w2[H * LD2];
  float b1[H], b2[H], w3[H];
  float b3;
};

__device__ void load_weights(const float* __restrict__ P, Weights& W, int tid, int nthr) {
  for (int e = tid; e < H * FP; e += nthr) {
    const int r = e / FP, f = e % FP;
    W.w1[e] = f < F ? f2bf(P[P_W1 + r * F + f]) : (unsigned short)0;
  }
  for (int e = tid; e < H * H; e += nthr) W.w2[(e / H) * LD2 + e % H] = f2bf(P[P_W2 + e]);
  for (int e = tid; e < H; e += nthr) {
    W.b1[e] = P[P_B1 + e];
    W.b2[e] = P[P_B2 + e];
    W.w3[e] = P[P_W3 + e];
  }
  if (tid == 0) W.b3 = P[P_B3];
}

// Forward pass of one wave over 64 samples whose bf16 features sit in xb[64][XS]: XS = 16, or
// XS = 8, where the features 8..15 of the padded input (zero) are not stored and the lanes
// holding that half of the K operand take zeros.
// Outputs (registers, tile (a, sb) holds hidden rows 16a + 4(l/16) + i, sample 16sb + l%16):
// z1, h1b (bf16 of silu(z1)), z2, h2 = silu(z2), and y[sb] for sample 16sb + l%16.
struct Fwd {
  f4 z1[4][4];
  s4 h1b[4][4];
  f4 z2[4][4];
  f4 h2[4][4];
  float y[4];
};

template <bool KEEP, int XS = FP>
__device__ void forward_wave(const Weights& W, const unsigned short* xb, int lane, Fwd& o) {
  static_assert(XS == FP || (XS == 8 && F <= 8), "input row stride");
  const int r16 = lane % 16, g4 = 4 * (lane / 16);
  // layer 1: Z1^T(16a.., 16sb..) = W1 tile a  x  X^T tile sb, the accumulator starting at the
  // bias of the lane's four rows
  for (int a = 0; a < 4; ++a) {
    const s4 A = lds4(&W.w1[(16 * a + r16) * FP + g4]);
    const f4 bias = *reinterpret_cast<const f4*>(&W.b1[16 * a + g4]);
    for (int sb = 0; sb < 4; ++sb) {
      const s4 B = (XS == FP || g4 < XS) ? lds4(&xb[(16 * sb + r16) * XS + g4]) : s4{0, 0, 0, 0};
      const f4 z = mfma(A, B, bias);
      float h[4];
      for (int i = 0; i < 4; ++i) h[i] = silu(z[i]);
      if (KEEP) o.z1[a][sb] = z;
      o.h1b[a][sb] = pack4(h[0], h[1], h[2], h[3]);
    }
  }
  // layer 2: Z2^T(16a.., 16sb..) = sum_kb W2 tile (a, kb)  x  H1^T tile (kb, sb); layer 3
  // (float32, y = W3 . h2 + b3) accumulated per lane as the tiles come, then reduced over the
  // four lane groups
  float py[4] = {0.f, 0.f, 0.f, 0.f};
  for (int a = 0; a < 4; ++a) {
    const f4 bias = *reinterpret_cast<const f4*>(&W.b2[16 * a + g4]);
    const f4 w3 = *reinterpret_cast<const f4*>(&W.w3[16 * a + g4]);
    for (int sb = 0; sb < 4; ++sb) {
      f4 z = bias;
      for (int kb = 0; kb < 4; ++kb) z = mfma(lds4(&W.w2[(16 * a + r16) * LD2 + 16 * kb + g4]), o.h1b[kb][sb], z);
      f4 h;
      for (int i = 0; i < 4; ++i) {
        h[i] = silu(z[i]);
        py[sb] += w3[i] * h[i];
      }
      if (KEEP) {
        o.z2[a][sb] = z;
        o.h2[a][sb] = h;
      }
    }
  }
  for (int sb = 0; sb < 4; ++sb) {
    float p = py[sb];
    p += __shfl_xor(p, 16, 64);
    p += __shfl_xor(p, 32, 64);
    o.y[sb] = p + W.b3;
  }
}

}  // namespace mlp
}  // namespace les
