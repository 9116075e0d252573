// mlp.hip -- training of the learned start on the GPU (BF16 matrix cores, FP32
// accumulation and FP32 master weights with Adam), and packing of the
// inference parameters.
//
// One training step on a batch of B (tensor, target direction) pairs, for the
// network of kin = 32 (K <= 32) or 48 (K <= 48) inputs and d' outputs:
//   X  = features(C)                         B x kin
//   Z1 = X W1 + b1,  H1 = bf16(relu Z1)      B x 64
//   Z2 = H1 W2 + b2, H2 = bf16(relu Z2)      B x 64
//   Y  = H2 W3 + b3                          B x 16 (d' used)
//   L  = mean_b 1 - (y_b . t_b / |y_b||t_b|)^2
//   dY, then dW3 = H2^T dY, dZ2 = (dY W3^T) * [Z2 > 0], dW2 = H1^T dZ2,
//   dZ1 = (dZ2 W2^T) * [Z1 > 0], dW1 = X^T dZ1, bias gradients = column sums,
//   Adam on the FP32 masters, then the BF16 fragment-ordered inference copy.
// Every product goes through one BF16 MFMA GEMM kernel (operands rounded to
// BF16 on load, FP32 accumulation).
#include "internal.hpp"
#include "mlp_core.hpp"
#include "sym_tables.hpp"

namespace ttm {

namespace {

// C[M][N] = op(A)[M][K] op(B)[K][N] with op = transpose when TA / TB.
// A element (m, k) = TA ? A[k * lda + m] : A[m * lda + k]; B (k, n) likewise.
// Epilogues: 0 store; 1 + bias[n]; 2 + bias[n], store Z to C and
// bf16(relu(Z)) to C2; 3 multiply by [mask[m][n] > 0].
// Workgroup: 4 wavefronts, 32 x 32 output tile, K in steps of 16.
// With gridDim.z > 1 (split K, epilogue 0 only) workgroup z covers K-chunk z
// and writes its partial tile to C + z * M * ldc; k_splitk_sum adds them in order.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_bf16(const float* __restrict__ A, int lda,
                                                   const float* __restrict__ B, int ldb,
                                                   float* __restrict__ C, int ldc, int M, int N,
                                                   int K, int epi, const float* __restrict__ bias,
                                                   float* __restrict__ C2,
                                                   const float* __restrict__ mask, int kchunk) {
  __shared__ unsigned short As[32][16 + 2];
  __shared__ unsigned short Bs[16][32 + 2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
  const int wm = (w >> 1) * 16, wn = (w & 1) * 16;
  const int r16 = lane & 15, q = lane >> 4;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  C += (size_t)blockIdx.z * M * ldc;
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    // 512 A elements and 512 B elements per step; 2 of each per thread
    for (int e = tid; e < 512; e += 256) {
      const int r = e / 16, c = e % 16;       // A tile (32 x 16)
      const int m = m0 + r, k = k0 + c;
      float va = 0.0f;
      if (m < M && k < kend) va = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
      As[r][c] = bf16_bits(va);
      const int kb = e / 32, nb = e % 32;     // B tile (16 x 32)
      const int kk = k0 + kb, n = n0 + nb;
      float vb = 0.0f;
      if (kk < kend && n < N) vb = TB ? B[(size_t)n * ldb + kk] : B[(size_t)kk * ldb + n];
      Bs[kb][nb] = bf16_bits(vb);
    }
    __syncthreads();
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = (short)As[wm + r16][4 * q + j];
      b[j] = (short)Bs[4 * q + j][wn + r16];
    }
    acc = mfma16(a, b, acc);
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int m = m0 + wm + 4 * q + j, n = n0 + wn + r16;
    if (m >= M || n >= N) continue;
    float v = acc[j];
    const size_t o = (size_t)m * ldc + n;
    if (epi == 1 || epi == 2) v += bias[n];
    if (epi == 3) v = mask[o] > 0.0f ? v : 0.0f;
    C[o] = v;
    if (epi == 2) C2[o] = bf16_round(fmaxf(v, 0.0f));
  }
}

__global__ void k_splitk_sum(const float* __restrict__ part, int nsplit, size_t n,
                             float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int z = 0; z < nsplit; ++z) s += part[(size_t)z * n + i];
  out[i] = s;
}

// x = sqrt(mu_a) C_a / ||C||_F, zero padded to kin columns; C is B x K (row
// per sample); the weights mu of the d' = 3 (DP = 3) or quaternion (DP = 4) form.
template <int N, int DP>
__global__ void k_features(const float* __restrict__ Cin, int B, int kin, float* __restrict__ X) {
  constexpr int K = DP == 3 ? ncomp3(N) : ncomp4(N);
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float c[K];
  float f2 = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float mu;
    if constexpr (DP == 3) {
      constexpr Sym3<N> sy{};
      mu = sy.mu[k];
    } else {
      constexpr Sym4<N> sy{};
      mu = sy.mu[k];
    }
    c[k] = Cin[(size_t)b * K + k] * sqrtf(mu);
    f2 = fmaf(c[k], c[k], f2);
  }
  const float inv = f2 > 0.0f ? 1.0f / sqrtf(f2) : 0.0f;
  for (int k = 0; k < kin; ++k) X[(size_t)b * kin + k] = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) X[(size_t)b * kin + k] = c[k] * inv;
}

// dL/dY for L = mean 1 - (u.t)^2, u = y/|y| over the first dout outputs:
// dY = -2 c (t - c u) / (|y| B); per-block loss sums.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ Y, const float* __restrict__ T,
                                              int B, int dout, float* __restrict__ dY,
                                              float* __restrict__ part) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (b < B) {
    float y[4], t[4], tt = 0.0f, yy = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      y[i] = i < dout ? Y[(size_t)b * kMlpOut + i] : 0.0f;
      t[i] = i < dout ? T[(size_t)dout * b + i] : 0.0f;
      tt = fmaf(t[i], t[i], tt);
      yy = fmaf(y[i], y[i], yy);
    }
    const float tn = 1.0f / sqrtf(tt);
    const float ny = sqrtf(yy);
    const float iy = ny > 0.0f ? 1.0f / ny : 0.0f;
    float u[4], c = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      t[i] *= tn;
      u[i] = y[i] * iy;
      c = fmaf(u[i], t[i], c);
    }
    l = 1.0f - c * c;
    const float s = -2.0f * c * iy / (float)B;
    float* d = dY + (size_t)b * kMlpOut;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < dout) d[i] = s * (t[i] - c * u[i]);
    for (int k = dout; k < kMlpOut; ++k) d[k] = 0.0f;
  }
  __shared__ float red[256];
  red[threadIdx.x] = l;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Column sums of a B x N matrix (bias gradients, N <= 64) in two fixed-order
// stages: each workgroup sums a chunk of kColRows rows, then one pass adds the chunks.
constexpr int kColRows = 256;
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ D, int B, int N,
                                                     float* __restrict__ part) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, sub = threadIdx.x >> 6;
  const int r0 = blockIdx.x * kColRows;
  float s = 0.0f;
  if (c < N)
    for (int r = r0 + sub; r < min(B, r0 + kColRows); r += 4) s += D[(size_t)r * N + c];
  red[sub][c] = s;
  __syncthreads();
  if (sub == 0 && c < N) part[(size_t)blockIdx.x * N + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

__global__ void k_sum(const float* __restrict__ part, int n, float scale, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s += part[i];
    out[0] = s * scale;
  }
}

// Adam with bias correction on the FP32 masters; padded rows / columns stay 0.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, MlpRt r, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, int K, int dout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r.params) return;
  bool pad = false;
  if (i < r.off_b1) pad = (i / kMlpHid) >= K;                               // W1 rows >= K
  else if (i >= r.off_w3 && i < r.off_b3) pad = ((i - r.off_w3) % kMlpOut) >= dout;
  else if (i >= r.off_b3) pad = (i - r.off_b3) >= dout;
  if (pad) {
    p[i] = 0.0f;
    m[i] = 0.0f;
    v[i] = 0.0f;
    return;
  }
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// FP32 masters -> BF16 fragment-ordered weights + FP32 biases.
__global__ void k_pack(const float* __restrict__ p, MlpRt r, unsigned char* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  // fragments: W1 4 KT, W2 16, W3 4, each 64 lanes x 4 values
  const int nw12 = r.w1_frags + 16;
  if (t < (nw12 + 4) * 64) {
    const int frag = t / 64, lane = t % 64, r16 = lane & 15, q = lane >> 4;
    const float* W;
    int ld, s, nt, off, f;
    if (frag < r.w1_frags) {
      W = p; ld = kMlpHid; f = frag; off = 0;
    } else if (frag < nw12) {
      W = p + r.off_w2; ld = kMlpHid; f = frag - r.w1_frags; off = r.pk_w2;
    } else {
      W = p + r.off_w3; ld = kMlpOut; f = frag - nw12; off = r.pk_w3;
    }
    if (frag < nw12) {
      s = f / 4; nt = f % 4;
    } else {
      s = f; nt = 0;
    }
    unsigned short* o = reinterpret_cast<unsigned short*>(out + off) + ((size_t)f * 64 + lane) * 4;
    for (int j = 0; j < 4; ++j) o[j] = bf16_bits(W[(16 * s + 4 * q + j) * ld + 16 * nt + r16]);
  }
  if (t < kMlpHid) {
    reinterpret_cast<float*>(out + r.pk_b1)[t] = p[r.off_b1 + t];
    reinterpret_cast<float*>(out + r.pk_b2)[t] = p[r.off_b2 + t];
  }
  if (t < kMlpOut) reinterpret_cast<float*>(out + r.pk_b3)[t] = p[r.off_b3 + t];
}

void launch_pack(const float* params, const MlpRt& r, unsigned char* packed, hipStream_t s) {
  const int threads = (r.w1_frags + 20) * 64;
  hipLaunchKernelGGL(k_pack, dim3((threads + 255) / 256), dim3(256), 0, s, params, r, packed);
}

template <bool TA, bool TB>
void gemm(const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N, int K,
          int epi, const float* bias, float* C2, const float* mask, hipStream_t s,
          float* splitk_ws = nullptr, int nsplit = 1) {
  if (nsplit > 1) {
    const int kchunk = ((K + nsplit - 1) / nsplit + 15) / 16 * 16;
    const int nz = (K + kchunk - 1) / kchunk;
    hipLaunchKernelGGL((k_gemm_bf16<TA, TB>), dim3((N + 31) / 32, (M + 31) / 32, nz), dim3(256), 0, s,
                       A, lda, B, ldb, splitk_ws, ldc, M, N, K, 0, nullptr, nullptr, nullptr, kchunk);
    const size_t n = (size_t)M * ldc;
    hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, splitk_ws,
                       nz, n, C);
    return;
  }
  hipLaunchKernelGGL((k_gemm_bf16<TA, TB>), dim3((N + 31) / 32, (M + 31) / 32, 1), dim3(256), 0, s,
                     A, lda, B, ldb, C, ldc, M, N, K, epi, bias, C2, mask, K);
}

void colsum(const float* D, int B, int N, float* out, float* part, hipStream_t s) {
  const int nchunk = (B + kColRows - 1) / kColRows;
  hipLaunchKernelGGL(k_colsum_part, dim3(nchunk), dim3(256), 0, s, D, B, N, part);
  hipLaunchKernelGGL(k_splitk_sum, dim3(1), dim3(64), 0, s, part, nchunk, (size_t)N, out);
}

constexpr int kSplit = 64;

}  // namespace

size_t mlp_train_workspace(int B) {
  // X (up to 48) + Z1, H1, Z2, H2, dZ1, dZ2 (64 each) + Y, dY (16 each) per sample,
  // gradient block, loss partials
  // + split-K partial tiles (kSplit x 64 x 64) + column-sum partials
  return ((size_t)B * (kMlpInMax + 6 * 64 + 2 * 16) + MlpLayout<3>::params + (B + 255) / 256 + 64 +
          (size_t)kSplit * 64 * 64 + (size_t)((B + 255) / 256) * 64) * 4 + 1024;
}

int mlp_train_step(int degree, int dprime, const float* Cin, const float* T, int B, float* params,
                   float* adam_m, float* adam_v, int step, float lr, unsigned char* packed,
                   float* loss_out, float* grads_out, void* ws, hipStream_t s) {
  const int K = dprime == 3 ? ncomp3(degree) : ncomp4(degree);
  const MlpRt r = mlp_rt_for(K);
  const int kin = r.kin, dout = dprime;
  float* w = static_cast<float*>(ws);
  float* X = w;
  float* Z1 = X + (size_t)B * kin;
  float* H1 = Z1 + (size_t)B * 64;
  float* Z2 = H1 + (size_t)B * 64;
  float* H2 = Z2 + (size_t)B * 64;
  float* dZ1 = H2 + (size_t)B * 64;
  float* dZ2 = dZ1 + (size_t)B * 64;
  float* Y = dZ2 + (size_t)B * 64;
  float* dY = Y + (size_t)B * 16;
  float* G = dY + (size_t)B * 16;
  float* part = G + r.params;
  const int nb = (B + 255) / 256;
  float* skw = part + nb + 64;                         // split-K partials
  float* cpart = skw + (size_t)kSplit * 64 * 64;       // column-sum partials
  switch (dprime * 10 + degree) {
    case 32: hipLaunchKernelGGL((k_features<2, 3>), dim3(nb), dim3(256), 0, s, Cin, B, kin, X); break;
    case 34: hipLaunchKernelGGL((k_features<4, 3>), dim3(nb), dim3(256), 0, s, Cin, B, kin, X); break;
    case 36: hipLaunchKernelGGL((k_features<6, 3>), dim3(nb), dim3(256), 0, s, Cin, B, kin, X); break;
    case 42: hipLaunchKernelGGL((k_features<2, 4>), dim3(nb), dim3(256), 0, s, Cin, B, kin, X); break;
    case 44: hipLaunchKernelGGL((k_features<4, 4>), dim3(nb), dim3(256), 0, s, Cin, B, kin, X); break;
    default: set_error("mlp: degree %d not built for d'=%d", degree, dprime); return -4;
  }
  const float* W1 = params;
  const float* W2 = params + r.off_w2;
  const float* W3 = params + r.off_w3;
  // forward
  gemm<false, false>(X, kin, W1, 64, Z1, 64, B, 64, kin, 2, params + r.off_b1, H1, nullptr, s);
  gemm<false, false>(H1, 64, W2, 64, Z2, 64, B, 64, 64, 2, params + r.off_b2, H2, nullptr, s);
  gemm<false, false>(H2, 64, W3, 16, Y, 16, B, 16, 64, 1, params + r.off_b3, nullptr, nullptr, s);
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, Y, T, B, dout, dY, part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, part, nb, 1.0f / (float)B, loss_out);
  // backward
  const int ns = B >= 2048 ? kSplit : 1;
  gemm<true, false>(H2, 64, dY, 16, G + r.off_w3, 16, 64, 16, B, 0, nullptr, nullptr, nullptr, s, skw, ns);
  colsum(dY, B, 16, G + r.off_b3, cpart, s);
  gemm<false, true>(dY, 16, W3, 16, dZ2, 64, B, 64, 16, 3, nullptr, nullptr, Z2, s);
  gemm<true, false>(H1, 64, dZ2, 64, G + r.off_w2, 64, 64, 64, B, 0, nullptr, nullptr, nullptr, s, skw, ns);
  colsum(dZ2, B, 64, G + r.off_b2, cpart, s);
  gemm<false, true>(dZ2, 64, W2, 64, dZ1, 64, B, 64, 64, 3, nullptr, nullptr, Z1, s);
  gemm<true, false>(X, kin, dZ1, 64, G, 64, kin, 64, B, 0, nullptr, nullptr, nullptr, s, skw, ns);
  colsum(dZ1, B, 64, G + r.off_b1, cpart, s);
  if (grads_out) {
    TTM_HIP(hipMemcpyAsync(grads_out, G, (size_t)r.params * 4, hipMemcpyDeviceToDevice, s));
  }
  if (lr > 0.0f) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float bc1 = 1.0f - powf(b1, (float)step), bc2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((r.params + 255) / 256), dim3(256), 0, s, params, G, adam_m,
                       adam_v, r, lr, b1, b2, eps, bc1, bc2, K, dout);
  }
  if (packed) launch_pack(params, r, packed, s);
  TTM_HIP(hipGetLastError());
  return 0;
}

int mlp_pack(int K, const float* params, unsigned char* packed, hipStream_t s) {
  launch_pack(params, mlp_rt_for(K), packed, s);
  TTM_HIP(hipGetLastError());
  return 0;
}

}  // namespace ttm
