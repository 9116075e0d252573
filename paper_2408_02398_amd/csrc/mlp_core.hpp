// mlp_core.hpp -- BF16 matrix-core (MFMA) building blocks of the learned start.
//
// Network: x (K features, zero padded to 16 KT: 32 for K <= 32, 48 for
// K <= 48) -> 64 -> relu -> 64 -> relu -> d' (output padded to 16).  Weights
// are BF16, products accumulate in FP32, activations are rounded to BF16
// before they feed the next product.
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

constexpr int kMlpIn = 32;     // padded input width of the K <= 32 network
constexpr int kMlpInMax = 48;  // the widest network (K <= 48)
constexpr int kMlpHid = 64;
constexpr int kMlpOut = 16;    // padded output width (d' used)

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

// The same layouts for a network of KT input tiles of 16 (W1 [16 KT][64]:
// 4 KT fragments); KT = 2 is the layout above.
template <int KT>
struct MlpLayout {
  static constexpr int kin = 16 * KT;
  static constexpr int off_w1 = 0;
  static constexpr int off_b1 = off_w1 + kin * kMlpHid;
  static constexpr int off_w2 = off_b1 + kMlpHid;
  static constexpr int off_b2 = off_w2 + kMlpHid * kMlpHid;
  static constexpr int off_w3 = off_b2 + kMlpHid;
  static constexpr int off_b3 = off_w3 + kMlpHid * kMlpOut;
  static constexpr int params = off_b3 + kMlpOut;
  static constexpr int w1_frags = 4 * KT;
  static constexpr int pk_w1 = 0;
  static constexpr int pk_w2 = pk_w1 + w1_frags * kFragBytes;
  static constexpr int pk_w3 = pk_w2 + 16 * kFragBytes;
  static constexpr int pk_b1 = pk_w3 + 4 * kFragBytes;
  static constexpr int pk_b2 = pk_b1 + kMlpHid * 4;
  static constexpr int pk_b3 = pk_b2 + kMlpHid * 4;
  static constexpr int packed = pk_b3 + kMlpOut * 4;
};
static_assert(MlpLayout<2>::params == kMlpParams && MlpLayout<2>::packed == kMlpPackedBytes &&
                  MlpLayout<2>::pk_b3 == kPkB3 && MlpLayout<2>::off_w3 == kOffW3,
              "the K <= 32 network is MlpLayout<2>");

// Input tiles of the network for K components.
__host__ __device__ constexpr int mlp_tiles(int K) { return K <= 32 ? 2 : 3; }

// MlpLayout as run-time values, for the training kernels and the host.
struct MlpRt {
  int kt, kin, off_b1, off_w2, off_b2, off_w3, off_b3, params, w1_frags, pk_w2, pk_w3, pk_b1,
      pk_b2, pk_b3, packed;
};
template <int KT>
__host__ __device__ constexpr MlpRt mlp_rt() {
  using L = MlpLayout<KT>;
  return MlpRt{KT, L::kin, L::off_b1, L::off_w2, L::off_b2, L::off_w3, L::off_b3, L::params,
               L::w1_frags, L::pk_w2, L::pk_w3, L::pk_b1, L::pk_b2, L::pk_b3, L::packed};
}
__host__ __device__ constexpr MlpRt mlp_rt_for(int K) { return K <= 32 ? mlp_rt<2>() : mlp_rt<3>(); }

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
// a wavefront.  The network runs transposed, H^T = W^T X^T, so that the
// weights are the A operands and each layer's D fragments are exactly the
// next layer's B fragments (no exchange between layers).  The packed B
// fragment (s, nt) of W, W[16 s + 4 (L/16) + j][16 nt + L % 16], is the A
// fragment of W^T for row tile nt and k tile s, so the packed layout serves
// unchanged.  Biases are held for the D rows of this lane: unit 16 m + 4 (L/16) + j.
struct MlpRegs {
  bf16x4 w1[8], w2[16], w3[4];
  float b1[4][4], b2[4][4], b3[4];
};

__device__ __forceinline__ void load_mlp_regs(const unsigned char* __restrict__ wp, int lane,
                                              MlpRegs& r) {
  const float* b1 = reinterpret_cast<const float*>(wp + kPkB1);
  const float* b2 = reinterpret_cast<const float*>(wp + kPkB2);
  const float* b3 = reinterpret_cast<const float*>(wp + kPkB3);
  const int q = lane >> 4;
#pragma unroll
  for (int f = 0; f < 8; ++f) r.w1[f] = load_frag(wp, kPkW1, f, lane);
#pragma unroll
  for (int f = 0; f < 16; ++f) r.w2[f] = load_frag(wp, kPkW2, f, lane);
#pragma unroll
  for (int f = 0; f < 4; ++f) r.w3[f] = load_frag(wp, kPkW3, f, lane);
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      r.b1[m][j] = b1[16 * m + 4 * q + j];
      r.b2[m][j] = b2[16 * m + 4 * q + j];
    }
#pragma unroll
  for (int j = 0; j < 4; ++j) r.b3[j] = b3[4 * q + j];
}

// Fragments and biases of the packed network read from an LDS copy of it on
// demand (the same layout as in global memory), for kernels that keep their
// registers for other work.
template <int KT>
struct MlpLdsT {
  using Lay = MlpLayout<KT>;
  const unsigned char* pk;   // LDS copy of the Lay::packed packed bytes
  int lane;
  __device__ __forceinline__ bf16x4 w1(int f) const { return load_frag(pk, Lay::pk_w1, f, lane); }
  __device__ __forceinline__ bf16x4 w2(int f) const { return load_frag(pk, Lay::pk_w2, f, lane); }
  __device__ __forceinline__ bf16x4 w3(int f) const { return load_frag(pk, Lay::pk_w3, f, lane); }
  __device__ __forceinline__ float b1(int m, int j) const {
    return reinterpret_cast<const float*>(pk + Lay::pk_b1)[16 * m + 4 * (lane >> 4) + j];
  }
  __device__ __forceinline__ float b2(int m, int j) const {
    return reinterpret_cast<const float*>(pk + Lay::pk_b2)[16 * m + 4 * (lane >> 4) + j];
  }
  __device__ __forceinline__ float b3(int j) const {
    return reinterpret_cast<const float*>(pk + Lay::pk_b3)[4 * (lane >> 4) + j];
  }
};
using MlpLds = MlpLdsT<2>;

// The same accessors over the registers of MlpRegs.
struct MlpRegView {
  const MlpRegs& r;
  __device__ __forceinline__ bf16x4 w1(int f) const { return r.w1[f]; }
  __device__ __forceinline__ bf16x4 w2(int f) const { return r.w2[f]; }
  __device__ __forceinline__ bf16x4 w3(int f) const { return r.w3[f]; }
  __device__ __forceinline__ float b1(int m, int j) const { return r.b1[m][j]; }
  __device__ __forceinline__ float b2(int m, int j) const { return r.b2[m][j]; }
  __device__ __forceinline__ float b3(int j) const { return r.b3[j]; }
};

template <class W>
__device__ __forceinline__ bf16x4 relu_bf16_w(const f32x4& acc, const W& w, int layer, int m) {
  bf16x4 h;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float b = layer == 1 ? w.b1(m, j) : w.b2(m, j);
    h[j] = (short)bf16_bits(fmaxf(acc[j] + b, 0.0f));
  }
  return h;
}

// Forward pass of one wavefront's 64 voxels (voxel = lane), weights from w,
// for a network of KT input tiles.
//   xs: this wavefront's [64][16 KT] bf16 features in LDS, written by the
//       lanes and made visible to the wavefront before the call.
// Returns y[0..3] (the first four outputs) of the calling lane's voxel.
template <int KT, class W>
__device__ __forceinline__ void mlp_forward_t(const unsigned short* xs, const W& w, int lane,
                                              float (&y)[4]) {
  constexpr int kin = 16 * KT;
  const int r16 = lane & 15, q = lane >> 4;
  // B fragments of X^T: lane L holds x[voxel 16 nt + L % 16][feature 16 s + 4 (L/16) + j]
  bf16x4 xb[KT][4];
#pragma unroll
  for (int s = 0; s < KT; ++s)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) xb[s][nt][j] = (short)xs[(16 * nt + r16) * kin + 16 * s + 4 * q + j];
  // layer 1: H1^T (64 x 64) = W1^T (64 x 16 KT) X^T (16 KT x 64)
  bf16x4 h1[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    bf16x4 a[KT];
#pragma unroll
    for (int s = 0; s < KT; ++s) a[s] = w.w1(4 * s + m);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KT; ++s) acc = mfma16(a[s], xb[s][nt], acc);
      h1[m][nt] = relu_bf16_w(acc, w, 1, m);
    }
  }
  // layer 2: H2^T = W2^T H1^T
  bf16x4 h2[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    bf16x4 a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = w.w2(s * 4 + m);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = mfma16(a[s], h1[s][nt], acc);
      h2[m][nt] = relu_bf16_w(acc, w, 2, m);
    }
  }
  // layer 3: Y^T (16 x 64) = W3^T H2^T; lanes 0..15 hold rows 0..3 (outputs)
  // of voxel columns 16 nt + lane
  bf16x4 a3[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) a3[s] = w.w3(s);
  float yv[4][4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = mfma16(a3[s], h2[s][nt], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) yv[i][nt] = acc[i] + w.b3(i);
  }
  // each voxel lane fetches its outputs from lane (voxel % 16) of tile voxel / 16
  const int src = lane & 15, tile = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float pick = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const float t = __shfl(yv[i][nt], src);
      pick = (tile == nt) ? t : pick;
    }
    y[i] = pick;
  }
}

// The K <= 32 network with three outputs (d' = 3).
template <class W>
__device__ __forceinline__ void mlp_forward_w(const unsigned short* xs, const W& w, int lane,
                                              float& y0, float& y1, float& y2) {
  float y[4];
  mlp_forward_t<2>(xs, w, lane, y);
  y0 = y[0];
  y1 = y[1];
  y2 = y[2];
}

// Forward pass with the network in registers, for one-wavefront workgroups
// (starts with the workgroup barrier that makes xs visible).
__device__ __forceinline__ void mlp_forward(const unsigned short* xs, const MlpRegs& w, int lane,
                                            float& y0, float& y1, float& y2) {
  __syncthreads();
  mlp_forward_w(xs, MlpRegView{w}, lane, y0, y1, y2);
}

}  // namespace ttm
