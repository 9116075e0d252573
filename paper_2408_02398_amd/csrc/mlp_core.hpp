// mlp_core.hpp -- BF16 matrix-core (MFMA) building blocks of the learned start.
//
// Network: x (K <= 32 features, zero padded) -> 64 -> relu -> 64 -> relu -> 3
// (output padded to 16).  Weights are BF16, products accumulate in FP32,
// activations are rounded to BF16 before they feed the next product.
//
// v_mfma_f32_16x16x16_bf16 operand layout (wave64, lane L, j = 0..3):
//   A (16 x 16, row-major M x K): lane L holds A[L % 16][4 (L / 16) + j]
//   B (16 x 16, K x N):           lane L holds B[4 (L / 16) + j][L % 16]
//   D (16 x 16, M x N):           lane L holds D[4 (L / 16) + j][L % 16]
#pragma once

#include <hip/hip_runtime.h>

namespace ttm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 32;     // padded input width
constexpr int kMlpHid = 64;
constexpr int kMlpOut = 16;    // padded output width (3 used)

// FP32 master parameter layout (floats): W1 [32][64], b1[64], W2 [64][64], b2[64],
// W3 [64][16], b3[16].  Rows of W1 beyond K and columns of W3 beyond d' are 0.
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHid;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;   // 7312

// Packed inference layout (bytes).  Weights are stored in matrix-core
// fragment order so that one 8-byte load per lane yields a B operand:
// fragment (s, nt) of W holds, for lane L and j < 4, W[16 s + 4 (L/16) + j][16 nt + L % 16].
//   W1: s < 2, nt < 4 (8 fragments); W2: s < 4, nt < 4 (16); W3: s < 4, nt = 0 (4)
// followed by f32 b1[64], b2[64], b3[16].
constexpr int kFragBytes = 64 * 4 * 2;
constexpr int kPkW1 = 0;
constexpr int kPkW2 = kPkW1 + 8 * kFragBytes;
constexpr int kPkW3 = kPkW2 + 16 * kFragBytes;
constexpr int kPkB1 = kPkW3 + 4 * kFragBytes;
constexpr int kPkB2 = kPkB1 + kMlpHid * 4;
constexpr int kPkB3 = kPkB2 + kMlpHid * 4;
constexpr int kMlpPackedBytes = kPkB3 + kMlpOut * 4;   // 14912

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}
__device__ __forceinline__ float bf16_round(float f) { return bf16_val(bf16_bits(f)); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 load_frag(const unsigned char* wp, int off, int frag, int lane) {
  const uint2 v = *reinterpret_cast<const uint2*>(wp + off + (frag * 64 + lane) * 8);
  bf16x4 r;
  r[0] = (short)(v.x & 0xffffu);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xffffu);
  r[3] = (short)(v.y >> 16);
  return r;
}

// One lane's share of the packed network, held in registers for the life of
// a wavefront: its B fragments of W1 (8), W2 (16), W3 (4) and the biases of
// its output columns (16 nt + lane % 16).
struct MlpRegs {
  bf16x4 w1[8], w2[16], w3[4];
  float b1[4], b2[4], b3;
};

__device__ __forceinline__ void load_mlp_regs(const unsigned char* __restrict__ wp, int lane,
                                              MlpRegs& r) {
  const float* b1 = reinterpret_cast<const float*>(wp + kPkB1);
  const float* b2 = reinterpret_cast<const float*>(wp + kPkB2);
  const float* b3 = reinterpret_cast<const float*>(wp + kPkB3);
  const int r16 = lane & 15;
#pragma unroll
  for (int f = 0; f < 8; ++f) r.w1[f] = load_frag(wp, kPkW1, f, lane);
#pragma unroll
  for (int f = 0; f < 16; ++f) r.w2[f] = load_frag(wp, kPkW2, f, lane);
#pragma unroll
  for (int f = 0; f < 4; ++f) r.w3[f] = load_frag(wp, kPkW3, f, lane);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    r.b1[nt] = b1[16 * nt + r16];
    r.b2[nt] = b2[16 * nt + r16];
  }
  r.b3 = r16 < 3 ? b3[r16] : 0.0f;
}

// Forward pass of one wavefront's 64 rows (rows = lanes); the workgroup is
// this one wavefront (the barriers order its LDS traffic).
//   hs: [64][64] bf16 LDS scratch; its upper half (bytes 4096..8191) holds the
//       input features x as [64][32] bf16 on entry.
//   ys: [64][4] f32 LDS scratch.
// Returns y (3 floats) of the calling lane's row.
__device__ __forceinline__ void mlp_forward(unsigned short* hs, float* ys, const MlpRegs& w,
                                            int lane, float& y0, float& y1, float& y2) {
  const unsigned short* xs = hs + 64 * kMlpIn;   // upper half
  const int r16 = lane & 15, q = lane >> 4;
  // ---- layer 1: h1 = relu(x W1 + b1); row block m of h1 overwrites x rows
  //      already consumed (x sits in rows 32..63 of the scratch)
  for (int m = 0; m < 4; ++m) {
    f32x4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < kMlpIn / 16; ++s) {
      bf16x4 a;
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = (short)xs[(16 * m + r16) * kMlpIn + 16 * s + 4 * q + j];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma16(a, w.w1[s * 4 + nt], acc[nt]);
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        hs[(16 * m + 4 * q + j) * kMlpHid + 16 * nt + r16] =
            bf16_bits(fmaxf(acc[nt][j] + w.b1[nt], 0.0f));
    __syncthreads();
  }
  // ---- layer 2: h2 = relu(h1 W2 + b2), in place row block by row block
  for (int m = 0; m < 4; ++m) {
    f32x4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < kMlpHid / 16; ++s) {
      bf16x4 a;
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = (short)hs[(16 * m + r16) * kMlpHid + 16 * s + 4 * q + j];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma16(a, w.w2[s * 4 + nt], acc[nt]);
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        hs[(16 * m + 4 * q + j) * kMlpHid + 16 * nt + r16] =
            bf16_bits(fmaxf(acc[nt][j] + w.b2[nt], 0.0f));
    __syncthreads();
  }
  // ---- layer 3: y = h2 W3 + b3 (16 padded outputs, 3 used)
  for (int m = 0; m < 4; ++m) {
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < kMlpHid / 16; ++s) {
      bf16x4 a;
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = (short)hs[(16 * m + r16) * kMlpHid + 16 * s + 4 * q + j];
      acc = mfma16(a, w.w3[s], acc);
    }
    if (r16 < 3) {
#pragma unroll
      for (int j = 0; j < 4; ++j) ys[(16 * m + 4 * q + j) * 4 + r16] = acc[j] + w.b3;
    }
  }
  __syncthreads();
  y0 = ys[lane * 4 + 0];
  y1 = ys[lane * 4 + 1];
  y2 = ys[lane * 4 + 2];
}

}  // namespace ttm
