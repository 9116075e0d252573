// api.hip -- the C ABI of libttm: argument checks, tiling, and the kernels
// that are not FFT passes (prefilter and its FP64 statistics, the local
// variance combine, template normalisation, the tensor template of Alg. 1).
#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ttm.h"
#include "internal.hpp"
#include "mlp_core.hpp"

struct ttm_ctx {
  int device;
  ttm::cf* twiddles;
  void* scratch;   // device address of `scratch` on this context's GPU
};

// Scratch of ttm_extract_noalloc, for callers that cannot allocate: one copy
// per GPU the library runs on, held until the process ends.  In host code the
// name is a stand-in, not a device address: ttm_create resolves the address
// on each context's device (hipGetSymbolAddress) and only that is used.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace ttm {


namespace {
thread_local char g_err[512] = "";

__global__ void k_zero(unsigned* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}
}  // namespace

void fill_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;
  const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_zero, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, static_cast<unsigned*>(p), n);
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hip_status(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return TTM_EDEVICE;
}

namespace {

constexpr int kPfZ = 16;  // z slices per prefilter thread

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int BS>
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sa[BS / 64], sb[BS / 64];
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off);
    b += __shfl_down(b, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sa[wv] = a;
    sb[wv] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < BS / 64; ++i) {
      a += sa[i];
      b += sb[i];
    }
  }
}

// g = h * f with taps [a, 1-2a, a] on every axis, border voxels replicated;
// per-block FP64 sums of g and g^2.
__global__ __launch_bounds__(256) void k_prefilter(const float* __restrict__ f, float* __restrict__ g,
                                                   int nz, int ny, int nx, float a,
                                                   double* __restrict__ part) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  const int z0 = blockIdx.z * kPfZ;
  const float w0 = a, w1 = 1.0f - 2.0f * a;
  double s1 = 0.0, s2 = 0.0;
  if (x < nx) {
    const int xm = clampi(x - 1, 0, nx - 1), xp = clampi(x + 1, 0, nx - 1);
    const int ym = clampi(y - 1, 0, ny - 1), yp = clampi(y + 1, 0, ny - 1);
    const int ys[3] = {ym, y, yp};
    // x- and y-filtered value of plane zz at (y, x)
    auto plane_yx = [&](int zz) {
      float acc_y = 0.0f;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float* row = f + ((size_t)zz * ny + ys[j]) * nx;
        const float hx = w0 * row[xm] + w1 * row[x] + w0 * row[xp];
        acc_y += (j == 1 ? w1 : w0) * hx;
      }
      return acc_y;
    };
    // planes z - 1, z, z + 1 slide along z: each plane is filtered once
    float pm = plane_yx(clampi(z0 - 1, 0, nz - 1)), pc = plane_yx(min(z0, nz - 1));
    float pp = plane_yx(clampi(z0 + 1, 0, nz - 1));
    for (int z = z0; z < min(z0 + kPfZ, nz); ++z) {
      if (z > z0) {
        pm = pc;
        pc = pp;
        pp = plane_yx(clampi(z + 1, 0, nz - 1));
      }
      float acc_z = 0.0f;
      acc_z += w0 * pm;
      acc_z += w1 * pc;
      acc_z += w0 * pp;
      g[((size_t)z * ny + y) * nx + x] = acc_z;
      s1 += (double)acc_z;
      s2 += (double)acc_z * (double)acc_z;
    }
  }
  block_sum2<256>(s1, s2);
  if (threadIdx.x == 0) {
    const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * b] = s1;
    part[2 * b + 1] = s2;
  }
}

__global__ __launch_bounds__(1024) void k_stats(const double* __restrict__ part, size_t nb,
                                                double inv_n, double* __restrict__ stats) {
  double s1 = 0.0, s2 = 0.0;
  for (size_t i = threadIdx.x; i < nb; i += 1024) {
    s1 += part[2 * i];
    s2 += part[2 * i + 1];
  }
  block_sum2<1024>(s1, s2);
  if (threadIdx.x == 0) {
    stats[0] = s1 * inv_n;
    stats[1] = s2 * inv_n;
  }
}

// var = s2 - s1^2 / M in FP64; w = 1/sqrt(var) above the guard, else 0.
__global__ void k_var_combine(const float* __restrict__ s1, const float* __restrict__ s2, int sz,
                              int sy, int sx, double M, double eps, const double* __restrict__ stats,
                              float* __restrict__ w, int ny, int nx, int oz, int oy, int ox) {
  const size_t n = (size_t)sz * sy * sx;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % sx), y = (int)((i / sx) % sy), z = (int)(i / ((size_t)sx * sy));
  const double a = (double)s1[i], b = (double)s2[i];
  const double var = b - a * a / M;
  const double thr = eps * M * stats[1];
  w[((size_t)(oz + z) * ny + (oy + y)) * nx + (ox + x)] = (var > thr) ? (float)(1.0 / sqrt(var)) : 0.0f;
}

__global__ void k_mask(float* __restrict__ m, int L, float r) {
  const int n = L * L * L;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = L / 2;
  const int x = i % L - c, y = (i / L) % L - c, z = i / (L * L) - c;
  m[i] = ((float)(x * x + y * y + z * z) <= r * r) ? 1.0f : 0.0f;
}

// t' = m (S(t) - mu) / sigma_t, S(t) = m (h * t) with zero padding (Eq. norm_t).
// One workgroup; the box has at most 64^3 voxels.
__global__ __launch_bounds__(1024) void k_template_norm(const float* __restrict__ t, int L, float r,
                                                        float a, float* __restrict__ tn) {
  const int n = L * L * L, c = L / 2;
  const float w0 = a, w1 = 1.0f - 2.0f * a;
  double sm = 0.0, s1 = 0.0, s2 = 0.0, mm = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const int x = i % L, y = (i / L) % L, z = i / (L * L);
    const int dx = x - c, dy = y - c, dz = z - c;
    const bool in = (float)(dx * dx + dy * dy + dz * dz) <= r * r;
    float st = 0.0f;
    if (in) {
      for (int k = -1; k <= 1; ++k) {
        const int zz = z + k;
        if (zz < 0 || zz >= L) continue;
        for (int j = -1; j <= 1; ++j) {
          const int yy = y + j;
          if (yy < 0 || yy >= L) continue;
          const float* row = t + ((size_t)zz * L + yy) * L;
          float hx = w1 * row[x];
          if (x > 0) hx += w0 * row[x - 1];
          if (x < L - 1) hx += w0 * row[x + 1];
          st += (k == 0 ? w1 : w0) * (j == 0 ? w1 : w0) * hx;
        }
      }
      mm += 1.0;
    }
    tn[i] = st;
    sm += (double)st;          // <S(t), m> = <S(t), 1> for a binary mask
    s2 += (double)st * (double)st;
  }
  s1 = sm;
  __shared__ double red[3][16];
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_down(s1, off);
    s2 += __shfl_down(s2, off);
    mm += __shfl_down(mm, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = s1;
    red[1][wv] = s2;
    red[2][wv] = mm;
  }
  __syncthreads();
  __shared__ double mu_s, inv_sig;
  if (threadIdx.x == 0) {
    double A = 0, B = 0, Mv = 0;
    for (int i = 0; i < 16; ++i) {
      A += red[0][i];
      B += red[1][i];
      Mv += red[2][i];
    }
    mu_s = A / Mv;
    const double var = B - A * A / Mv;
    inv_sig = var > 0.0 ? 1.0 / sqrt(var) : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 1024) {
    const int x = i % L - c, y = (i / L) % L - c, z = i / (L * L) - c;
    const bool in = (float)(x * x + y * y + z * z) <= r * r;
    tn[i] = in ? (float)(((double)tn[i] - mu_s) * inv_sig) : 0.0f;
  }
}

constexpr int kMaxK = 165;    // n = 8, d' = 4
constexpr int kCompBlock = 32;
constexpr int kQChunk = 64;

struct Exponents {
  unsigned char e[kMaxK][4];
};

// T_a(p) = (1/nq) sum_q v_q^a t'(c + R(q)^T (p - c)) for a in [a0, a0 + na).
__global__ __launch_bounds__(256) void k_build(const float* __restrict__ tn, int L,
                                               const float* __restrict__ quats, int nq, int dprime,
                                               float ax, float ay, float az, int a0, int na,
                                               Exponents ex, float* __restrict__ T) {
  __shared__ float sR[kQChunk][9];
  __shared__ float sMono[kQChunk][kCompBlock];
  const int n = L * L * L;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const float c = (float)(L / 2);
  const float px = (float)(i % L) - c, py = (float)((i / L) % L) - c, pz = (float)(i / (L * L)) - c;
  double acc[kCompBlock];
#pragma unroll
  for (int k = 0; k < kCompBlock; ++k) acc[k] = 0.0;
  for (int q0 = 0; q0 < nq; q0 += kQChunk) {
    const int nc = min(kQChunk, nq - q0);
    __syncthreads();
    if ((int)threadIdx.x < nc) {
      const float* q = quats + 4 * (q0 + threadIdx.x);
      float w = q[0], x = q[1], y = q[2], z = q[3];
      const float rn = 1.0f / sqrtf(w * w + x * x + y * y + z * z);
      w *= rn; x *= rn; y *= rn; z *= rn;
      float R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                    2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                    2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
#pragma unroll
      for (int k = 0; k < 9; ++k) sR[threadIdx.x][k] = R[k];
      float v[4];
      if (dprime == 4) {
        v[0] = w; v[1] = x; v[2] = y; v[3] = z;
      } else {
        v[0] = R[0] * ax + R[1] * ay + R[2] * az;
        v[1] = R[3] * ax + R[4] * ay + R[5] * az;
        v[2] = R[6] * ax + R[7] * ay + R[8] * az;
        v[3] = 1.0f;
      }
      for (int k = 0; k < na; ++k) {
        float m = 1.0f;
        for (int d = 0; d < dprime; ++d)
          for (int e = 0; e < ex.e[a0 + k][d]; ++e) m *= v[d];
        sMono[threadIdx.x][k] = m;
      }
    }
    __syncthreads();
    if (i < n) {
      float part[kCompBlock];
#pragma unroll
      for (int k = 0; k < kCompBlock; ++k) part[k] = 0.0f;
      for (int qi = 0; qi < nc; ++qi) {
        const float* R = sR[qi];
        // source point c + R^T p
        const float sx = c + R[0] * px + R[3] * py + R[6] * pz;
        const float sy = c + R[1] * px + R[4] * py + R[7] * pz;
        const float sz = c + R[2] * px + R[5] * py + R[8] * pz;
        const float fx = floorf(sx), fy = floorf(sy), fz = floorf(sz);
        const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
        const float tx = sx - fx, ty = sy - fy, tz = sz - fz;
        float val = 0.0f;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz) {
          const int zz = iz + dz;
          if (zz < 0 || zz >= L) continue;
          const float wz = dz ? tz : 1.0f - tz;
#pragma unroll
          for (int dy = 0; dy < 2; ++dy) {
            const int yy = iy + dy;
            if (yy < 0 || yy >= L) continue;
            const float wy = dy ? ty : 1.0f - ty;
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
              const int xx = ix + dx;
              if (xx < 0 || xx >= L) continue;
              const float wx = dx ? tx : 1.0f - tx;
              val += wz * wy * wx * tn[((size_t)zz * L + yy) * L + xx];
            }
          }
        }
#pragma unroll
        for (int k = 0; k < kCompBlock; ++k) part[k] = fmaf(sMono[qi][k], val, part[k]);
      }
#pragma unroll
      for (int k = 0; k < kCompBlock; ++k) acc[k] += (double)part[k];
    }
  }
  if (i < n) {
    const double inv = 1.0 / (double)nq;
    for (int k = 0; k < na; ++k) T[(size_t)(a0 + k) * n + i] = (float)(acc[k] * inv);
  }
}

// ---------------------------------------------------------------------------
// wedge-aware tensor template: every rotated t' through the missing-wedge
// filter (on its box zero-padded to P^3) and renormalised over the mask
// ---------------------------------------------------------------------------

// Edge of the padded box: the smallest supported FFT edge >= L.
int wedge_box(int L) {
  int P = 32;
  while (P < L) P *= 2;
  return P;
}
// Rotations handled per batch: at most 2^24 box voxels, at most 256.
int wedge_batch(int P) {
  const long b = (1L << 24) / ((long)P * P * P);
  return (int)(b < 1 ? 1 : (b > 256 ? 256 : b));
}

__device__ __forceinline__ void quat_rotation(const float* q, float (&R)[9], float (&qn)[4]) {
  float w = q[0], x = q[1], y = q[2], z = q[3];
  const float rn = 1.0f / sqrtf(w * w + x * x + y * y + z * z);
  w *= rn; x *= rn; y *= rn; z *= rn;
  qn[0] = w; qn[1] = x; qn[2] = y; qn[3] = z;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

// Box b (rotation q0 + b) holds t'(c + R^T (p - c)) at p in [0, L)^3 and 0
// elsewhere in [0, P)^3 (trilinear, zero outside the template box).
__global__ __launch_bounds__(256) void k_rotate_boxes(const float* __restrict__ tn, int L,
                                                      const float* __restrict__ quats, int q0, int P,
                                                      float* __restrict__ boxes) {
  const int b = blockIdx.y;
  const size_t n = (size_t)P * P * P;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % P), y = (int)((i / P) % P), z = (int)(i / ((size_t)P * P));
  float val = 0.0f;
  if (x < L && y < L && z < L) {
    float R[9], qn[4];
    quat_rotation(quats + 4 * (size_t)(q0 + b), R, qn);
    const float c = (float)(L / 2);
    const float px = (float)x - c, py = (float)y - c, pz = (float)z - c;
    const float sx = c + R[0] * px + R[3] * py + R[6] * pz;
    const float sy = c + R[1] * px + R[4] * py + R[7] * pz;
    const float sz = c + R[2] * px + R[5] * py + R[8] * pz;
    const float fx = floorf(sx), fy = floorf(sy), fz = floorf(sz);
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    const float tx = sx - fx, ty = sy - fy, tz = sz - fz;
    for (int dz = 0; dz < 2; ++dz) {
      const int zz = iz + dz;
      if (zz < 0 || zz >= L) continue;
      const float wz = dz ? tz : 1.0f - tz;
      for (int dy = 0; dy < 2; ++dy) {
        const int yy = iy + dy;
        if (yy < 0 || yy >= L) continue;
        const float wy = dy ? ty : 1.0f - ty;
        for (int dx = 0; dx < 2; ++dx) {
          const int xx = ix + dx;
          if (xx < 0 || xx >= L) continue;
          const float wx = dx ? tx : 1.0f - tx;
          val += wz * wy * wx * tn[((size_t)zz * L + yy) * L + xx];
        }
      }
    }
  }
  boxes[(size_t)b * n + i] = val;
}

// Zero the half-spectrum coefficients ([kz][kx][ky], ky fastest) inside the
// wedge: |f_z| > tan * f_x (integer frequencies, f_z signed), DC kept.
__global__ __launch_bounds__(256) void k_wedge(cf* __restrict__ spec, size_t stride, int P, float tanv) {
  const int b = blockIdx.y;
  const size_t n = (size_t)P * (P / 2 + 1) * P;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int kx = (int)((i / P) % (P / 2 + 1)), kz = (int)(i / ((size_t)P * (P / 2 + 1)));
  const int fz = kz <= P / 2 ? kz : P - kz;   // |f_z|; kz = P/2 is the Nyquist plane
  if ((float)fz > tanv * (float)kx) spec[(size_t)b * stride + i] = cf{0.0f, 0.0f};
}

// Per box: mu = <v, m>/M and 1/sigma over the ball mask of the template box,
// in FP64 (0 where sigma = 0).
__global__ __launch_bounds__(256) void k_box_stats(const float* __restrict__ boxes, int P, int L,
                                                   float r, double* __restrict__ stats) {
  __shared__ double r1[256], r2[256], rm[256];
  const int b = blockIdx.x;
  const size_t n = (size_t)P * P * P;
  const int c = L / 2;
  double s1 = 0.0, s2 = 0.0, sm = 0.0;
  for (int i = threadIdx.x; i < L * L * L; i += blockDim.x) {
    const int x = i % L, y = (i / L) % L, z = i / (L * L);
    const float dx = (float)(x - c), dy = (float)(y - c), dz = (float)(z - c);
    if (dx * dx + dy * dy + dz * dz > r * r) continue;
    const double v = boxes[(size_t)b * n + ((size_t)z * P + y) * P + x];
    s1 += v;
    s2 += v * v;
    sm += 1.0;
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  rm[threadIdx.x] = sm;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      r1[threadIdx.x] += r1[threadIdx.x + off];
      r2[threadIdx.x] += r2[threadIdx.x + off];
      rm[threadIdx.x] += rm[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double M = rm[0];
    const double var = r2[0] - r1[0] * r1[0] / M;
    stats[2 * b] = r1[0] / M;
    stats[2 * b + 1] = var > 0.0 ? 1.0 / sqrt(var) : 0.0;
  }
}

// Tacc[a][p] += sum_b v_b^a m(p) (box_b(p) - mu_b) / sigma_b for a in
// [a0, a0 + na), p in [0, L)^3, boxes of rotations q0 .. q0 + nb - 1.
__global__ __launch_bounds__(256) void k_wedge_accumulate(const float* __restrict__ boxes, int P, int L,
                                                          float r, const float* __restrict__ quats,
                                                          int q0, int nb, int dprime, float ax, float ay,
                                                          float az, int a0, int na, Exponents ex,
                                                          const double* __restrict__ stats,
                                                          double* __restrict__ Tacc) {
  __shared__ float sMono[kQChunk][kCompBlock];
  __shared__ float sMu[kQChunk], sIs[kQChunk];
  const int n = L * L * L;
  const size_t nbox = (size_t)P * P * P;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = L / 2;
  int x = 0, y = 0, z = 0;
  bool inside = false;
  if (i < n) {
    x = i % L; y = (i / L) % L; z = i / (L * L);
    const float dx = (float)(x - c), dy = (float)(y - c), dz = (float)(z - c);
    inside = dx * dx + dy * dy + dz * dz <= r * r;
  }
  double acc[kCompBlock];
#pragma unroll
  for (int k = 0; k < kCompBlock; ++k) acc[k] = 0.0;
  for (int b0 = 0; b0 < nb; b0 += kQChunk) {
    const int nc = min(kQChunk, nb - b0);
    __syncthreads();
    if ((int)threadIdx.x < nc) {
      float R[9], qn[4];
      quat_rotation(quats + 4 * (size_t)(q0 + b0 + threadIdx.x), R, qn);
      float v[4];
      if (dprime == 4) {
        v[0] = qn[0]; v[1] = qn[1]; v[2] = qn[2]; v[3] = qn[3];
      } else {
        v[0] = R[0] * ax + R[1] * ay + R[2] * az;
        v[1] = R[3] * ax + R[4] * ay + R[5] * az;
        v[2] = R[6] * ax + R[7] * ay + R[8] * az;
        v[3] = 1.0f;
      }
      for (int k = 0; k < na; ++k) {
        float m = 1.0f;
        for (int d = 0; d < dprime; ++d)
          for (int e = 0; e < ex.e[a0 + k][d]; ++e) m *= v[d];
        sMono[threadIdx.x][k] = m;
      }
      sMu[threadIdx.x] = (float)stats[2 * (b0 + threadIdx.x)];
      sIs[threadIdx.x] = (float)stats[2 * (b0 + threadIdx.x) + 1];
    }
    __syncthreads();
    if (inside) {
      float part[kCompBlock];
#pragma unroll
      for (int k = 0; k < kCompBlock; ++k) part[k] = 0.0f;
      const size_t off = ((size_t)z * P + y) * P + x;
      for (int bi = 0; bi < nc; ++bi) {
        const float val = (boxes[(size_t)(b0 + bi) * nbox + off] - sMu[bi]) * sIs[bi];
#pragma unroll
        for (int k = 0; k < kCompBlock; ++k) part[k] = fmaf(sMono[bi][k], val, part[k]);
      }
#pragma unroll
      for (int k = 0; k < kCompBlock; ++k) acc[k] += (double)part[k];
    }
  }
  if (i < n)
    for (int k = 0; k < na; ++k) Tacc[(size_t)(a0 + k) * n + i] += acc[k];
}

__global__ void k_wedge_finish(const double* __restrict__ Tacc, size_t total, double inv,
                               float* __restrict__ T) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) T[i] = (float)(Tacc[i] * inv);
}

__global__ void k_zero_f64(double* __restrict__ p, size_t total) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) p[i] = 0.0;
}

int ncomp(int n, int d) {
  if (n < 0 || n > 8 || (d != 3 && d != 4)) return -1;
  long num = 1, den = 1;
  for (int i = 1; i <= d - 1; ++i) {
    num *= (n + i);
    den *= i;
  }
  return (int)(num / den);
}

// graded-lex exponents, descending leading counts (same order as the d'=3 tables)
void exponents(int n, int d, Exponents& ex) {
  int k = 0;
  std::memset(&ex, 0, sizeof(ex));
  if (d == 3) {
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        ex.e[k][0] = (unsigned char)a;
        ex.e[k][1] = (unsigned char)b;
        ex.e[k][2] = (unsigned char)(n - a - b);
        ++k;
      }
  } else {
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b)
        for (int c2 = n - a - b; c2 >= 0; --c2) {
          ex.e[k][0] = (unsigned char)a;
          ex.e[k][1] = (unsigned char)b;
          ex.e[k][2] = (unsigned char)c2;
          ex.e[k][3] = (unsigned char)(n - a - b - c2);
          ++k;
        }
  }
}

bool valid_desc(const ttm_desc* d) {
  if (!d) {
    set_error("desc is NULL");
    return false;
  }
  if (d->degree < 0 || d->degree > 8 || (d->degree & 1)) {
    set_error("degree %d must be even and in 0..8", d->degree);
    return false;
  }
  if (d->dprime != 3 && d->dprime != 4) {
    set_error("dprime %d must be 3 or 4", d->dprime);
    return false;
  }
  if (d->L < 2 || d->L > 64) {
    set_error("template edge L=%d must be in 2..64", d->L);
    return false;
  }
  if (!(d->mask_radius > 0.0f) || !(d->mask_radius < 0.5f * d->L)) {
    set_error("mask radius %g must be in (0, L/2)", (double)d->mask_radius);
    return false;
  }
  if (!(d->filter_a > 0.0f) || !(d->filter_a < 0.25f)) {
    set_error("filter a=%g must be in (0, 1/4)", (double)d->filter_a);
    return false;
  }
  if (!(d->eps_w >= 0.0f)) {
    set_error("eps_w must be >= 0");
    return false;
  }
  return true;
}

// Forms and degrees the learned start is built for (K <= kMlpInMax inputs).
bool mlp_form_ok(const ttm_desc* d) {
  return (d->dprime == 3 && (d->degree == 2 || d->degree == 4 || d->degree == 6)) ||
         (d->dprime == 4 && (d->degree == 2 || d->degree == 4));
}

bool fft_ok(int N) {
  return N == 32 || N == 64 || N == 128 || N == 256 || N == 512 || N == 96 || N == 160 || N == 192;
}

size_t spec_elems(int N) { return (size_t)N * (N / 2 + 1) * N; }
// x/y-transformed template: its L nonzero z planes only
size_t tspec_elems(int N, int L) { return (size_t)L * (N / 2 + 1) * N; }
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t wedge_workspace(int L, int K) {
  const int P = wedge_box(L), B = wedge_batch(P);
  const size_t nbox = (size_t)P * P * P;
  return align256((size_t)B * nbox * 4) + align256((size_t)B * spec_elems(P) * 8) +
         align256((size_t)B * 16) + align256((size_t)K * L * L * L * 8);
}


double mask_count(int L, float r) {
  const int c = L / 2;
  double m = 0;
  for (int z = 0; z < L; ++z)
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        const int dx = x - c, dy = y - c, dz = z - c;
        if ((float)(dx * dx + dy * dy + dz * dz) <= r * r) m += 1.0;
      }
  return m;
}

size_t prefilter_blocks(int nz, int ny, int nx) {
  return (size_t)((nx + 255) / 256) * ny * ((nz + kPfZ - 1) / kPfZ);
}

}  // namespace
}  // namespace ttm

namespace ttm {
int find_peaks_batch(const ttm_peak_item* items, int n_items, const int32_t max_valid[3],
                     hipStream_t s);
}

using namespace ttm;

extern "C" {

const char* ttm_last_error(void) { return ttm::g_err; }

int ttm_n_components(int degree, int dprime) { return ncomp(degree, dprime); }

size_t ttm_spectrum_elems(int fft_n) { return fft_ok(fft_n) ? spec_elems(fft_n) : 0; }

size_t ttm_template_spectrum_elems(int fft_n, int L) {
  return fft_ok(fft_n) && L >= 1 && L <= fft_n ? tspec_elems(fft_n, L) : 0;
}

int ttm_fft_supported(int fft_n) { return fft_ok(fft_n) ? 1 : 0; }

int ttm_create(ttm_ctx** out, int device) {
  if (!out) {
    set_error("ttm_create: out is NULL");
    return TTM_EINVAL;
  }
  *out = nullptr;
  int n = 0;
  TTM_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) {
    set_error("ttm_create: device %d not present (%d devices)", device, n);
    return TTM_EINVAL;
  }
  TTM_HIP(hipSetDevice(device));
  void* scratch_ptr = nullptr;
  TTM_HIP(hipGetSymbolAddress(&scratch_ptr, HIP_SYMBOL(scratch)));
  ttm_ctx* c = new (std::nothrow) ttm_ctx{device, nullptr, scratch_ptr};
  if (!c) {
    set_error("ttm_create: out of host memory");
    return TTM_ENOMEM;
  }
  if (hipMalloc(&c->twiddles, sizeof(cf) * kTwiddleTotal) != hipSuccess) {
    delete c;
    set_error("ttm_create: device allocation failed");
    return TTM_ENOMEM;
  }
  int rc = init_twiddles(c->twiddles, nullptr);
  if (rc == 0) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = hip_status(e, "ttm_create");
  }
  if (rc != 0) {
    (void)hipFree(c->twiddles);
    delete c;
    return rc;
  }
  *out = c;
  return TTM_OK;
}

void ttm_destroy(ttm_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipFree(ctx->twiddles);
  delete ctx;
}

size_t ttm_workspace_size(const ttm_desc* desc, int op, int fft_n, int nz, int ny, int nx) {
  if (!desc) return 0;
  const int K = ncomp(desc->degree, desc->dprime);
  if (K < 0) return 0;
  const size_t L = (size_t)desc->L;
  switch (op) {
    case TTM_OP_SPECTRA:
      return align256(L * L * L * 4);
    case TTM_OP_PREFILTER:
      if (nz < 1 || ny < 1 || nx < 1) return 0;
      return align256(prefilter_blocks(nz, ny, nx) * 16);
    case TTM_OP_NORMALIZE: {
      if (!fft_ok(fft_n) || desc->L > fft_n) return 0;
      const size_t step = (size_t)(fft_n - desc->L + 1);
      return 4 * align256(spec_elems(fft_n) * 8) + 2 * align256(step * step * step * 4) +
             align256(prefilter_blocks(nz, ny, nx) * 16);
    }
    case TTM_OP_CORRELATE:
      if (!fft_ok(fft_n) || desc->L > fft_n) return 0;
      return (size_t)(1 + K) * align256(spec_elems(fft_n) * 8);
    case TTM_OP_PEAKS:
      return align256(peaks_workspace((int64_t)nz * ny * nx));
    case TTM_OP_EXTRACT:
      if (nz < 1 || ny < 1 || nx < 1) return 0;
      return desc->dprime == 4 ? extract_workspace4((size_t)nz * ny * nx)
                               : extract_workspace((size_t)nz * ny * nx, desc->degree);
    case TTM_OP_MLP_TRAIN:
      if (nz < 1) return 0;
      return align256(mlp_train_workspace(nz));
    case TTM_OP_REFINE:
      if (nz < 1 || ny < 0 || ny > max_refine_radius()) return 0;
      return refine_workspace(K, nz, (float)ny);
    case TTM_OP_TENSOR_WEDGE:
      if (desc->L < 1 || desc->L > 512) return 0;
      return wedge_workspace(desc->L, K);
    case TTM_OP_NORM_CORR: {
      if (!fft_ok(fft_n) || desc->L > fft_n) return 0;
      const size_t step = (size_t)(fft_n - desc->L + 1);
      return (size_t)(2 + std::max(K, 2)) * align256(spec_elems(fft_n) * 8) +
             2 * align256(step * step * step * 4);
    }
    default:
      return 0;
  }
}

int ttm_build_tensor(ttm_ctx* ctx, const ttm_desc* desc, const float* tmpl, const float* quats,
                     int nq, float* T_out, float* tn_out, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!tmpl || !quats || !T_out || !tn_out || nq < 1) {
    set_error("ttm_build_tensor: null pointer or nq < 1");
    return TTM_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  const int L = desc->L, K = ncomp(desc->degree, desc->dprime);
  hipLaunchKernelGGL(k_template_norm, dim3(1), dim3(1024), 0, s, tmpl, L, desc->mask_radius,
                     desc->filter_a, tn_out);
  Exponents ex;
  exponents(desc->degree, desc->dprime, ex);
  float ax = desc->axis[0], ay = desc->axis[1], az = desc->axis[2];
  const float an = std::sqrt(ax * ax + ay * ay + az * az);
  if (desc->dprime == 3) {
    if (!(an > 0.0f)) {
      set_error("ttm_build_tensor: template axis is zero");
      return TTM_EINVAL;
    }
    ax /= an; ay /= an; az /= an;
  }
  const int n = L * L * L;
  for (int a0 = 0; a0 < K; a0 += kCompBlock) {
    const int na = std::min(kCompBlock, K - a0);
    hipLaunchKernelGGL(k_build, dim3((n + 255) / 256), dim3(256), 0, s, tn_out, L, quats, nq,
                       desc->dprime, ax, ay, az, a0, na, ex, T_out);
  }
  TTM_HIP(hipGetLastError());
  return TTM_OK;
}

int ttm_build_tensor_wedge(ttm_ctx* ctx, const ttm_desc* desc, const float* tmpl,
                           const float* quats, int nq, float wedge_deg, float* T_out,
                           float* tn_out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!tmpl || !quats || !T_out || !tn_out || !ws || nq < 1 || !(wedge_deg > 0.0f) ||
      !(wedge_deg < 90.0f)) {
    set_error("ttm_build_tensor_wedge: null pointer, nq < 1 or wedge angle outside (0, 90)");
    return TTM_EINVAL;
  }
  const int L = desc->L, K = ncomp(desc->degree, desc->dprime);
  if (L > 512) {
    set_error("ttm_build_tensor_wedge: L = %d above 512", L);
    return TTM_EUNSUPPORTED;
  }
  const size_t need = wedge_workspace(L, K);
  if (ws_bytes < need) {
    set_error("ttm_build_tensor_wedge: workspace %zu < %zu", ws_bytes, need);
    return TTM_EWORKSPACE;
  }
  float ax = desc->axis[0], ay = desc->axis[1], az = desc->axis[2];
  const float an = std::sqrt(ax * ax + ay * ay + az * az);
  if (desc->dprime == 3) {
    if (!(an > 0.0f)) {
      set_error("ttm_build_tensor_wedge: template axis is zero");
      return TTM_EINVAL;
    }
    ax /= an; ay /= an; az /= an;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_template_norm, dim3(1), dim3(1024), 0, s, tmpl, L, desc->mask_radius,
                     desc->filter_a, tn_out);
  const int P = wedge_box(L), B = wedge_batch(P);
  const size_t nbox = (size_t)P * P * P, nspec = spec_elems(P), n = (size_t)L * L * L;
  char* p = static_cast<char*>(ws);
  float* boxes = reinterpret_cast<float*>(p);
  p += align256((size_t)B * nbox * 4);
  cf* spec = reinterpret_cast<cf*>(p);
  p += align256((size_t)B * nspec * 8);
  double* stats = reinterpret_cast<double*>(p);
  p += align256((size_t)B * 16);
  double* Tacc = reinterpret_cast<double*>(p);
  const size_t total = (size_t)K * n;
  hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Tacc, total);
  Exponents ex;
  exponents(desc->degree, desc->dprime, ex);
  const float tanv = std::tan(wedge_deg * 3.14159265358979323846f / 180.0f);
  for (int q0 = 0; q0 < nq; q0 += B) {
    const int nb = std::min(B, nq - q0);
    hipLaunchKernelGGL(k_rotate_boxes, dim3((unsigned)((nbox + 255) / 256), nb), dim3(256), 0, s,
                       tn_out, L, quats, q0, P, boxes);
    RealSrc src{boxes, nbox, P, P, P, 0, 0, 0, nullptr, 0, 0};
    int rc = fft3d_forward(P, src, nb, spec, nspec, ctx->twiddles, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_wedge, dim3((unsigned)((nspec + 255) / 256), nb), dim3(256), 0, s, spec,
                       nspec, P, tanv);
    for (int b = 0; b < nb; ++b) {
      RealDst d{boxes + (size_t)b * nbox, 0, 0, P, P, 0, 0, 0, P, P, P, nullptr, 0, 0, 0, 0, 0,
                1.0f / (float)nbox};
      cf* sp = spec + (size_t)b * nspec;
      rc = fft3d_inverse_mul(P, sp, nullptr, 0, 0, 1, nullptr, sp, nspec, d, ctx->twiddles, s);
      if (rc) return rc;
    }
    hipLaunchKernelGGL(k_box_stats, dim3(nb), dim3(256), 0, s, boxes, P, L, desc->mask_radius, stats);
    for (int a0 = 0; a0 < K; a0 += kCompBlock) {
      const int na = std::min(kCompBlock, K - a0);
      hipLaunchKernelGGL(k_wedge_accumulate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                         boxes, P, L, desc->mask_radius, quats, q0, nb, desc->dprime, ax, ay, az,
                         a0, na, ex, stats, Tacc);
    }
  }
  hipLaunchKernelGGL(k_wedge_finish, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Tacc,
                     total, 1.0 / (double)nq, T_out);
  TTM_HIP(hipGetLastError());
  return TTM_OK;
}

int ttm_template_spectra(ttm_ctx* ctx, const ttm_desc* desc, const float* T, int fft_n,
                         void* spec_out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!fft_ok(fft_n)) {
    set_error("ttm_template_spectra: FFT edge %d not supported", fft_n);
    return TTM_EUNSUPPORTED;
  }
  if (desc->L > fft_n || !T || !spec_out || !ws) {
    set_error("ttm_template_spectra: L > fft_n or null pointer");
    return TTM_EINVAL;
  }
  const size_t need = ttm_workspace_size(desc, TTM_OP_SPECTRA, fft_n, 0, 0, 0);
  if (ws_bytes < need) {
    set_error("ttm_template_spectra: workspace %zu < %zu", ws_bytes, need);
    return TTM_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  const int L = desc->L, K = ncomp(desc->degree, desc->dprime);
  const size_t se = tspec_elems(fft_n, L);
  cf* out = static_cast<cf*>(spec_out);
  // fields at the origin: z planes L.. of the padded tile are zero
  RealSrc src{T, (size_t)L * L * L, L, L, L, 0, 0, 0, nullptr, 0, 0};
  int rc = fft3d_forward_planes(fft_n, src, K, L, out, se, ctx->twiddles, s);
  if (rc) return rc;
  float* m = static_cast<float*>(ws);
  hipLaunchKernelGGL(k_mask, dim3((L * L * L + 255) / 256), dim3(256), 0, s, m, L, desc->mask_radius);
  RealSrc msrc{m, 0, L, L, L, 0, 0, 0, nullptr, 0, 0};
  return fft3d_forward_planes(fft_n, msrc, 1, L, out + (size_t)K * se, se, ctx->twiddles, s);
}

namespace {

// w on the sub-tiles (edge fft_n - L + 1) of a box of the valid region.
int normalize_boxes(ttm_ctx* ctx, const ttm_desc* desc, const float* g, int nz, int ny, int nx,
                    const double* stats, const void* mask_spec, int fft_n, const int32_t box_lo[3],
                    const int32_t box_size[3], float* w_out, void* ws, hipStream_t s) {
  const int L = desc->L;
  const size_t se = spec_elems(fft_n);
  const size_t sb = align256(se * 8);
  const int step = fft_n - L + 1;
  // G of the centred tile and of its square (sb bytes apart), their two
  // products' work spectra, the local sums s1 and s2 (s_gap floats apart)
  char* w = static_cast<char*>(ws);
  cf* G1 = reinterpret_cast<cf*>(w);
  cf* work = reinterpret_cast<cf*>(w + 2 * sb);
  const size_t s_gap = align256((size_t)step * step * step * 4) / 4;
  float* s1 = reinterpret_cast<float*>(w + 4 * sb);
  float* s2 = s1 + s_gap;
  const int c = L / 2;
  const double M = mask_count(L, desc->mask_radius);
  const cf* mspec = static_cast<const cf*>(mask_spec);
  const float scale = 1.0f / ((float)fft_n * fft_n * fft_n);
  for (int dz = 0; dz < box_size[0]; dz += step) {
    const int szz = std::min(step, box_size[0] - dz);
    for (int dy = 0; dy < box_size[1]; dy += step) {
      const int syy = std::min(step, box_size[1] - dy);
      for (int dx = 0; dx < box_size[2]; dx += step) {
        const int sxx = std::min(step, box_size[2] - dx);
        const int oz = box_lo[0] + dz, oy = box_lo[1] + dy, ox = box_lo[2] + dx;
        // the centred tile and its square in one batched forward transform,
        // both products with the mask spectrum in one batched inverse
        RealSrc src{g, 0, nz, ny, nx, oz - c, oy - c, ox - c, stats, 0, 1};
        int rc = fft3d_forward(fft_n, src, 2, G1, sb / 8, ctx->twiddles, s);
        if (rc) return rc;
        RealDst d1{s1, 0, s_gap, syy, sxx, 0, 0, 0, szz, syy, sxx, nullptr, 0, 0, 0, 0, 0, scale};
        rc = fft3d_inverse_mul(fft_n, G1, mspec, 0, L, 1, nullptr, work, sb / 8, d1, ctx->twiddles, s,
                               2, sb / 8);
        if (rc) return rc;
        const size_t nbx = (size_t)szz * syy * sxx;
        hipLaunchKernelGGL(k_var_combine, dim3((unsigned)((nbx + 255) / 256)), dim3(256), 0, s, s1,
                           s2, szz, syy, sxx, M, (double)desc->eps_w, stats, w_out, ny, nx, oz,
                           oy, ox);
      }
    }
  }
  TTM_HIP(hipGetLastError());
  return TTM_OK;
}

void prefilter_stats(const ttm_desc* desc, const float* vol, int nz, int ny, int nx, float* g_out,
                     double* stats_out, double* part, hipStream_t s) {
  const dim3 pg((nx + 255) / 256, ny, (nz + kPfZ - 1) / kPfZ);
  hipLaunchKernelGGL(k_prefilter, pg, dim3(256), 0, s, vol, g_out, nz, ny, nx, desc->filter_a, part);
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(1024), 0, s, part, prefilter_blocks(nz, ny, nx),
                     1.0 / ((double)nz * ny * nx), stats_out);
}

bool box_in_valid(const ttm_desc* desc, int nz, int ny, int nx, const int32_t box_lo[3],
                  const int32_t box_size[3], const char* fn) {
  const int L = desc->L, c = L / 2;
  const int dims[3] = {nz, ny, nx};
  for (int a = 0; a < 3; ++a) {
    if (box_size[a] < 1 || box_lo[a] < c || box_lo[a] + box_size[a] - 1 > dims[a] - L + c) {
      set_error("%s: box axis %d [%d, +%d) outside the valid region [%d, %d]", fn, a, box_lo[a],
                box_size[a], c, dims[a] - L + c);
      return false;
    }
  }
  return true;
}

}  // namespace

int ttm_prefilter(ttm_ctx* ctx, const ttm_desc* desc, const float* vol, int nz, int ny, int nx,
                  float* g_out, float* w_out, double* stats_out, void* ws, size_t ws_bytes,
                  void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!vol || !g_out || !stats_out || !ws || nz < 1 || ny < 1 || nx < 1) {
    set_error("ttm_prefilter: null pointer or empty volume");
    return TTM_EINVAL;
  }
  const size_t need = ttm_workspace_size(desc, TTM_OP_PREFILTER, 0, nz, ny, nx);
  if (ws_bytes < need) {
    set_error("ttm_prefilter: workspace %zu < %zu", ws_bytes, need);
    return TTM_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  prefilter_stats(desc, vol, nz, ny, nx, g_out, stats_out, static_cast<double*>(ws), s);
  if (w_out) fill_zero(w_out, (size_t)nz * ny * nx * 4, s);
  TTM_HIP(hipGetLastError());
  return TTM_OK;
}

int ttm_normalize_box(ttm_ctx* ctx, const ttm_desc* desc, const float* g, int nz, int ny, int nx,
                      const double* stats, const void* mask_spec, int fft_n,
                      const int32_t box_lo[3], const int32_t box_size[3], float* w_out, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!fft_ok(fft_n)) {
    set_error("ttm_normalize_box: FFT edge %d not supported", fft_n);
    return TTM_EUNSUPPORTED;
  }
  if (!g || !stats || !mask_spec || !w_out || !ws || !box_lo || !box_size || desc->L > fft_n) {
    set_error("ttm_normalize_box: null pointer or L > fft_n");
    return TTM_EINVAL;
  }
  if (!box_in_valid(desc, nz, ny, nx, box_lo, box_size, "ttm_normalize_box")) return TTM_EINVAL;
  const size_t need = ttm_workspace_size(desc, TTM_OP_NORMALIZE, fft_n, nz, ny, nx);
  if (ws_bytes < need) {
    set_error("ttm_normalize_box: workspace %zu < %zu", ws_bytes, need);
    return TTM_EWORKSPACE;
  }
  TTM_HIP(hipSetDevice(ctx->device));
  return normalize_boxes(ctx, desc, g, nz, ny, nx, stats, mask_spec, fft_n, box_lo, box_size, w_out,
                         ws, static_cast<hipStream_t>(stream));
}

int ttm_normalize(ttm_ctx* ctx, const ttm_desc* desc, const float* vol, int nz, int ny, int nx,
                  const void* mask_spec, int fft_n, float* g_out, float* w_out, double* stats_out,
                  void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!fft_ok(fft_n)) {
    set_error("ttm_normalize: FFT edge %d not supported", fft_n);
    return TTM_EUNSUPPORTED;
  }
  const int L = desc->L;
  if (!vol || !mask_spec || !g_out || !w_out || !stats_out || !ws || L > fft_n || nz < L ||
      ny < L || nx < L) {
    set_error("ttm_normalize: null pointer, L > fft_n, or volume smaller than the template");
    return TTM_EINVAL;
  }
  const size_t need = ttm_workspace_size(desc, TTM_OP_NORMALIZE, fft_n, nz, ny, nx);
  if (ws_bytes < need) {
    set_error("ttm_normalize: workspace %zu < %zu", ws_bytes, need);
    return TTM_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  const size_t sb = align256(spec_elems(fft_n) * 8);
  const size_t step = (size_t)(fft_n - L + 1);
  double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + 4 * sb +
                                           2 * align256(step * step * step * 4));
  prefilter_stats(desc, vol, nz, ny, nx, g_out, stats_out, part, s);
  fill_zero(w_out, (size_t)nz * ny * nx * 4, s);
  const int c = L / 2;
  const int32_t lo[3] = {c, c, c};
  const int32_t size[3] = {nz - L + 1, ny - L + 1, nx - L + 1};
  return normalize_boxes(ctx, desc, g_out, nz, ny, nx, stats_out, mask_spec, fft_n, lo, size, w_out,
                         ws, s);
}

int ttm_correlate(ttm_ctx* ctx, const ttm_desc* desc, const float* g, const float* wmap, int nz,
                  int ny, int nx, const double* stats, const void* spec, int fft_n,
                  const int32_t box_lo[3], const int32_t box_size[3], int out_dtype, void* C_out,
                  void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!fft_ok(fft_n)) {
    set_error("ttm_correlate: FFT edge %d not supported", fft_n);
    return TTM_EUNSUPPORTED;
  }
  const int L = desc->L, c = L / 2;
  if (!g || !wmap || !spec || !C_out || !ws || !box_lo || !box_size || L > fft_n ||
      (out_dtype != TTM_F32 && out_dtype != TTM_BF16)) {
    set_error("ttm_correlate: null pointer, bad dtype or L > fft_n");
    return TTM_EINVAL;
  }
  const int dims[3] = {nz, ny, nx};
  for (int a = 0; a < 3; ++a) {
    if (box_size[a] < 1 || box_lo[a] < c || box_lo[a] + box_size[a] - 1 > dims[a] - L + c) {
      set_error("ttm_correlate: box axis %d [%d, +%d) outside the valid region [%d, %d]", a,
                box_lo[a], box_size[a], c, dims[a] - L + c);
      return TTM_EINVAL;
    }
  }
  const size_t need = ttm_workspace_size(desc, TTM_OP_CORRELATE, fft_n, nz, ny, nx);
  if (ws_bytes < need) {
    set_error("ttm_correlate: workspace %zu < %zu", ws_bytes, need);
    return TTM_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  const int K = ncomp(desc->degree, desc->dprime);
  const size_t se = spec_elems(fft_n);
  const size_t sb = align256(se * 8);
  char* w = static_cast<char*>(ws);
  cf* G = reinterpret_cast<cf*>(w);
  cf* work = reinterpret_cast<cf*>(w + sb);
  const int step = fft_n - L + 1;
  const float scale = 1.0f / ((float)fft_n * fft_n * fft_n);
  const size_t plane = (size_t)box_size[0] * box_size[1] * box_size[2];
  for (int dz = 0; dz < box_size[0]; dz += step) {
    const int szz = std::min(step, box_size[0] - dz);
    for (int dy = 0; dy < box_size[1]; dy += step) {
      const int syy = std::min(step, box_size[1] - dy);
      for (int dx = 0; dx < box_size[2]; dx += step) {
        const int sxx = std::min(step, box_size[2] - dx);
        const int oz = box_lo[0] + dz, oy = box_lo[1] + dy, ox = box_lo[2] + dx;
        RealSrc src{g, 0, nz, ny, nx, oz - c, oy - c, ox - c, stats, 0, 0};
        int rc = fft3d_forward(fft_n, src, 1, G, se, ctx->twiddles, s);
        if (rc) return rc;
        RealDst d{C_out, out_dtype, plane, box_size[1], box_size[2], dz, dy, dx, szz, syy, sxx,
                  wmap, ny, nx, oz, oy, ox, scale};
        rc = fft3d_inverse_mul(fft_n, G, static_cast<const cf*>(spec), tspec_elems(fft_n, L), L,
                               K, stats, work, sb / 8, d, ctx->twiddles, s);
        if (rc) return rc;
      }
    }
  }
  return TTM_OK;
}

int ttm_normalize_correlate(ttm_ctx* ctx, const ttm_desc* desc, const float* g, int nz, int ny,
                            int nx, const double* stats, const void* spec, int fft_n,
                            const int32_t box_lo[3], const int32_t box_size[3], float* w_out,
                            int out_dtype, void* C_out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!fft_ok(fft_n)) {
    set_error("ttm_normalize_correlate: FFT edge %d not supported", fft_n);
    return TTM_EUNSUPPORTED;
  }
  const int L = desc->L, c = L / 2;
  if (!g || !stats || !spec || !w_out || !C_out || !ws || !box_lo || !box_size || L > fft_n ||
      (out_dtype != TTM_F32 && out_dtype != TTM_BF16)) {
    set_error("ttm_normalize_correlate: null pointer, bad dtype or L > fft_n");
    return TTM_EINVAL;
  }
  const int step = fft_n - L + 1;
  const int dims[3] = {nz, ny, nx};
  for (int a = 0; a < 3; ++a) {
    if (box_size[a] < 1 || box_size[a] > step || box_lo[a] < c ||
        box_lo[a] + box_size[a] - 1 > dims[a] - L + c) {
      set_error("ttm_normalize_correlate: box axis %d [%d, +%d) outside the valid region [%d, %d] "
                "or longer than one tile (%d)", a, box_lo[a], box_size[a], c, dims[a] - L + c, step);
      return TTM_EINVAL;
    }
  }
  const size_t need = ttm_workspace_size(desc, TTM_OP_NORM_CORR, fft_n, 0, 0, 0);
  if (ws_bytes < need) {
    set_error("ttm_normalize_correlate: workspace %zu < %zu", ws_bytes, need);
    return TTM_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  const int K = ncomp(desc->degree, desc->dprime);
  const size_t se = spec_elems(fft_n);
  const size_t sb = align256(se * 8);
  // G of the centred tile and of its square (sb bytes apart), max(K, 2) work
  // spectra, the local sums s1 and s2 (s_gap floats apart)
  char* w = static_cast<char*>(ws);
  cf* G1 = reinterpret_cast<cf*>(w);
  cf* work = reinterpret_cast<cf*>(w + 2 * sb);
  const size_t s_gap = align256((size_t)step * step * step * 4) / 4;
  float* s1 = reinterpret_cast<float*>(w + (2 + std::max(K, 2)) * sb);
  float* s2 = s1 + s_gap;
  const double M = mask_count(L, desc->mask_radius);
  const size_t tse = tspec_elems(fft_n, L);
  const cf* tspec = static_cast<const cf*>(spec);
  const cf* mspec = tspec + (size_t)K * tse;
  const float scale = 1.0f / ((float)fft_n * fft_n * fft_n);
  const int oz = box_lo[0], oy = box_lo[1], ox = box_lo[2];
  const int szz = box_size[0], syy = box_size[1], sxx = box_size[2];
  // the centred g tile and its square, forward in one batched transform
  RealSrc src{g, 0, nz, ny, nx, oz - c, oy - c, ox - c, stats, 0, 1};
  int rc = fft3d_forward(fft_n, src, 2, G1, sb / 8, ctx->twiddles, s);
  if (rc) return rc;
  // local sums with the mask (both products in one batched inverse), then w on the box
  RealDst d1{s1, 0, s_gap, syy, sxx, 0, 0, 0, szz, syy, sxx, nullptr, 0, 0, 0, 0, 0, scale};
  rc = fft3d_inverse_mul(fft_n, G1, mspec, 0, L, 1, nullptr, work, sb / 8, d1, ctx->twiddles, s,
                         2, sb / 8);
  if (rc) return rc;
  const size_t nbx = (size_t)szz * syy * sxx;
  hipLaunchKernelGGL(k_var_combine, dim3((unsigned)((nbx + 255) / 256)), dim3(256), 0, s, s1, s2,
                     szz, syy, sxx, M, (double)desc->eps_w, stats, w_out, ny, nx, oz, oy, ox);
  // the K correlations from the same forward transform
  RealDst d{C_out, out_dtype, nbx, syy, sxx, 0, 0, 0, szz, syy, sxx, w_out, ny, nx, oz, oy, ox, scale};
  rc = fft3d_inverse_mul(fft_n, G1, tspec, tse, L, K, stats, work, sb / 8, d, ctx->twiddles, s);
  if (rc) return rc;
  TTM_HIP(hipGetLastError());
  return TTM_OK;
}

int ttm_extract(ttm_ctx* ctx, const ttm_desc* desc, const void* C, int in_dtype,
                const int32_t box_size[3], const ttm_extract_opts* opts, float* score, float* lambda,
                float* dir, const int32_t out_lo[3], const int32_t out_dims[3], int32_t* n_fallback,
                void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!C || !box_size || !opts || !out_lo || !out_dims || (in_dtype != TTM_F32 && in_dtype != TTM_BF16)) {
    set_error("ttm_extract: null pointer or bad dtype");
    return TTM_EINVAL;
  }
  for (int a = 0; a < 3; ++a) {
    if (box_size[a] < 1 || out_lo[a] < 0 || out_lo[a] + box_size[a] > out_dims[a]) {
      set_error("ttm_extract: box does not fit the output maps on axis %d", a);
      return TTM_EINVAL;
    }
  }
  const int mode = opts->mode;
  if ((mode & ~31) || !(mode & 3) || ((mode & 24) && !(mode & 4)) || ((mode & 4) && !(mode & 2))) {
    set_error("ttm_extract: mode %d invalid", mode);
    return TTM_EINVAL;
  }
  if ((mode & 1) && !score) {
    set_error("ttm_extract: score map is NULL");
    return TTM_EINVAL;
  }
  const size_t plane = (size_t)box_size[0] * box_size[1] * box_size[2];
  if (desc->dprime == 4 && desc->degree > 6) {
    set_error("ttm_extract: d'=4 scores need degree <= 6");
    return TTM_EUNSUPPORTED;
  }
  if (mode & 2) {
    if (desc->dprime == 3 ? (desc->degree < 2 || desc->degree > 6)
                          : (desc->degree < 2 || desc->degree > 6 ||
                             ((mode & 4) && (desc->degree > 4 || (mode & 8))))) {
      set_error("ttm_extract: orientation needs degree 2..6 (d'=3, or d'=4 with the multistart "
                "search); the learned start at d'=4 needs degree 2 or 4 and no start-only mode");
      return TTM_EUNSUPPORTED;
    }
    if (!opts->starts || opts->n_starts < 1 || opts->n_starts > 64 || opts->max_iter < 1 ||
        opts->max_iter > (1 << 24) ||
        !(opts->tol >= 0.0f) || opts->newton_steps < 0 || opts->newton_steps > 8 ||
        (!lambda && !dir)) {
      set_error("ttm_extract: orientation options invalid");
      return TTM_EINVAL;
    }
    if (mode & 4) {
      if (!opts->mlp || !lambda || !dir || !(opts->fallback_kappa == opts->fallback_kappa)) {
        set_error("ttm_extract: learned start needs mlp, lambda, dir and a kappa");
        return TTM_EINVAL;
      }
      if (!mlp_form_ok(desc)) {
        set_error("ttm_extract: no learned start for d'=%d, degree %d", desc->dprime, desc->degree);
        return TTM_EUNSUPPORTED;
      }
    }
    const size_t need = desc->dprime == 4 ? extract_workspace4(plane)
                                          : extract_workspace(plane, desc->degree);
    if (!ws || ws_bytes < need) {
      set_error("ttm_extract: workspace %zu < %zu", ws_bytes, need);
      return TTM_EWORKSPACE;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  ExtractArgs a{};
  a.C = C;
  a.in_dtype = in_dtype;
  a.plane = plane;
  a.by = box_size[1];
  a.bx = box_size[2];
  a.score = score;
  a.lam = lambda;
  a.dir = dir;
  a.oz = out_lo[0];
  a.oy = out_lo[1];
  a.ox = out_lo[2];
  a.dy = out_dims[1];
  a.dx = out_dims[2];
  a.mode = mode & 7;
  a.starts = opts->starts;
  a.n_starts = (mode & 2) ? opts->n_starts : 0;
  a.max_iter = opts->max_iter;
  a.tol = opts->tol;
  a.newton = opts->newton_steps;
  a.counters = reinterpret_cast<unsigned long long*>(opts->work_counters);
  a.ws = ws;
  if (mode & 4) {
    a.mlp = static_cast<const unsigned char*>(opts->mlp);
    a.kappa = opts->fallback_kappa;
    a.start_only = (mode & 8) ? 1 : 0;
    a.screen = (mode & 16) ? 0 : 1;
    a.fb_total = n_fallback;
  }
  return desc->dprime == 4 ? launch_extract4(desc->degree, a, s)
                           : launch_extract(desc->degree, a, s);
}

int ttm_extract_noalloc(ttm_ctx* ctx, const ttm_desc* desc, const void* C, int in_dtype,
                        const int32_t box_size[3], const ttm_extract_opts* opts, float* score,
                        float* lambda, float* dir, const int32_t out_lo[3],
                        const int32_t out_dims[3], int32_t* n_fallback, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!box_size || !opts) {
    set_error("ttm_extract_noalloc: null pointer");
    return TTM_EINVAL;
  }
  if (box_size[0] < 1 || box_size[1] < 1 || box_size[2] < 1) {
    set_error("ttm_extract_noalloc: empty box");
    return TTM_EINVAL;
  }
  const size_t plane = (size_t)box_size[0] * box_size[1] * box_size[2];
  const size_t need = desc->dprime == 4 ? extract_workspace4(plane)
                                        : extract_workspace(plane, desc->degree);
  if ((opts->mode & 2) && need > kNoAllocScratchBytes) {
    set_error("ttm_extract_noalloc: a box of %zu voxels needs %zu bytes of scratch, more than "
              "the %zu bytes the library holds (use ttm_extract with a workspace)",
              plane, need, kNoAllocScratchBytes);
    return TTM_EUNSUPPORTED;
  }
  return ttm_extract(ctx, desc, C, in_dtype, box_size, opts, score, lambda, dir, out_lo, out_dims,
                     n_fallback, ctx->scratch, kNoAllocScratchBytes, stream);
}

int ttm_refine(ttm_ctx* ctx, const ttm_desc* desc, const float* g, const float* w, int nz, int ny,
               int nx, const float* T, const float* tn, const int32_t* peaks, int n_peaks, float r_s,
               const ttm_extract_opts* opts, int32_t* pos_out, float* quat_out, float* lncc_out,
               float* quat_peak_out, float* lncc_peak_out, void* ws, size_t ws_bytes,
               void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (desc->dprime != 4 || desc->degree < 2 || desc->degree > 6) {
    set_error("ttm_refine: needs the quaternion form (d'=4) at degree 2, 4 or 6");
    return TTM_EUNSUPPORTED;
  }
  if (!g || !w || !T || !tn || !peaks || !opts || !pos_out || !quat_out || !lncc_out || !ws ||
      n_peaks < 1 || nz < desc->L || ny < desc->L || nx < desc->L || !(r_s >= 0.0f) ||
      r_s >= (float)(max_refine_radius() + 1)) {
    set_error("ttm_refine: null pointer, no peaks, volume smaller than the template, or r_s "
              "outside [0, %d]", max_refine_radius());
    return TTM_EINVAL;
  }
  if (!opts->starts || opts->n_starts < 1 || opts->n_starts > 64 || opts->max_iter < 1 ||
      opts->max_iter > (1 << 24) || !(opts->tol >= 0.0f) || opts->newton_steps < 0 ||
      opts->newton_steps > 8) {
    set_error("ttm_refine: orientation options invalid");
    return TTM_EINVAL;
  }
  const int K = ncomp(desc->degree, 4);
  const size_t need = refine_workspace(K, n_peaks, r_s);
  if (ws_bytes < need) {
    set_error("ttm_refine: workspace %zu < %zu", ws_bytes, need);
    return TTM_EWORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  ExtractArgs a{};
  a.starts = opts->starts;
  a.n_starts = opts->n_starts;
  a.max_iter = opts->max_iter;
  a.tol = opts->tol;
  a.newton = opts->newton_steps;
  a.counters = reinterpret_cast<unsigned long long*>(opts->work_counters);
  return refine(desc->degree, K, g, w, nz, ny, nx, T, tn, desc->L, desc->mask_radius, peaks, n_peaks,
                r_s, a, pos_out, quat_out, lncc_out, quat_peak_out, lncc_peak_out, ws, s);
}

static_assert(sizeof(ttm_extract_item) == 80, "ttm_extract_item layout is part of the ABI");

int ttm_extract_batch(ttm_ctx* ctx, const ttm_desc* desc, const ttm_extract_item* items,
                      int n_items, uint64_t total_voxels, int in_dtype,
                      const ttm_extract_opts* opts, int32_t* n_fallback, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!items || n_items < 1 || total_voxels < 1 || total_voxels >= ((uint64_t)1 << 32) || !opts ||
      (in_dtype != TTM_F32 && in_dtype != TTM_BF16)) {
    set_error("ttm_extract_batch: null pointer, no items, total voxels outside 1..2^32-1, or bad dtype");
    return TTM_EINVAL;
  }
  const int mode = opts->mode;
  if ((mode & ~31) || !(mode & 3) || ((mode & 24) && !(mode & 4)) || ((mode & 4) && !(mode & 2))) {
    set_error("ttm_extract_batch: mode %d invalid", mode);
    return TTM_EINVAL;
  }
  const size_t plane = (size_t)total_voxels;
  if (desc->dprime == 4 && desc->degree > 6) {
    set_error("ttm_extract_batch: d'=4 scores need degree <= 6");
    return TTM_EUNSUPPORTED;
  }
  if (mode & 2) {
    if (desc->degree < 2 || desc->degree > 6 ||
        (desc->dprime == 4 && (mode & 4) && (desc->degree > 4 || (mode & 8)))) {
      set_error("ttm_extract_batch: orientation needs degree 2..6; the learned start at d'=4 "
                "needs degree 2 or 4 and no start-only mode");
      return TTM_EUNSUPPORTED;
    }
    if (!opts->starts || opts->n_starts < 1 || opts->n_starts > 64 || opts->max_iter < 1 ||
        opts->max_iter > (1 << 24) || !(opts->tol >= 0.0f) || opts->newton_steps < 0 ||
        opts->newton_steps > 8) {
      set_error("ttm_extract_batch: orientation options invalid");
      return TTM_EINVAL;
    }
    if ((mode & 4) && (!opts->mlp || !(opts->fallback_kappa == opts->fallback_kappa))) {
      set_error("ttm_extract_batch: learned start needs mlp and a kappa");
      return TTM_EINVAL;
    }
    if ((mode & 4) && !mlp_form_ok(desc)) {
      set_error("ttm_extract_batch: no learned start for d'=%d, degree %d", desc->dprime, desc->degree);
      return TTM_EUNSUPPORTED;
    }
    const size_t need = desc->dprime == 4 ? extract_workspace4(plane)
                                          : extract_workspace(plane, desc->degree);
    if (!ws || ws_bytes < need) {
      set_error("ttm_extract_batch: workspace %zu < %zu", ws_bytes, need);
      return TTM_EWORKSPACE;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TTM_HIP(hipSetDevice(ctx->device));
  ExtractArgs a{};
  a.in_dtype = in_dtype;
  a.plane = plane;
  a.by = 1;
  a.bx = (int)plane;
  a.dy = 1;
  a.dx = (int)plane;
  a.mode = mode & 7;
  a.starts = opts->starts;
  a.n_starts = (mode & 2) ? opts->n_starts : 0;
  a.max_iter = opts->max_iter;
  a.tol = opts->tol;
  a.newton = opts->newton_steps;
  a.counters = reinterpret_cast<unsigned long long*>(opts->work_counters);
  a.ws = ws;
  a.items = items;
  a.n_items = n_items;
  if (mode & 4) {
    a.mlp = static_cast<const unsigned char*>(opts->mlp);
    a.kappa = opts->fallback_kappa;
    a.start_only = (mode & 8) ? 1 : 0;
    a.screen = (mode & 16) ? 0 : 1;
    a.fb_total = n_fallback;
  }
  return desc->dprime == 4 ? launch_extract4(desc->degree, a, s)
                           : launch_extract(desc->degree, a, s);
}

size_t ttm_mlp_param_count(const ttm_desc* desc) {
  if (!valid_desc(desc) || !mlp_form_ok(desc)) return 0;
  return (size_t)mlp_rt_for(ncomp(desc->degree, desc->dprime)).params;
}
size_t ttm_mlp_packed_bytes(const ttm_desc* desc) {
  if (!valid_desc(desc) || !mlp_form_ok(desc)) return 0;
  return (size_t)mlp_rt_for(ncomp(desc->degree, desc->dprime)).packed;
}

int ttm_mlp_pack(ttm_ctx* ctx, const ttm_desc* desc, const float* params, void* packed,
                 void* stream) {
  if (!ctx || !params || !packed || !valid_desc(desc)) {
    set_error("ttm_mlp_pack: null pointer or invalid descriptor");
    return TTM_EINVAL;
  }
  if (!mlp_form_ok(desc)) {
    set_error("ttm_mlp_pack: no learned start for d'=%d, degree %d", desc->dprime, desc->degree);
    return TTM_EUNSUPPORTED;
  }
  TTM_HIP(hipSetDevice(ctx->device));
  return mlp_pack(ncomp(desc->degree, desc->dprime), params, static_cast<unsigned char*>(packed),
                  static_cast<hipStream_t>(stream));
}

int ttm_mlp_train_step(ttm_ctx* ctx, const ttm_desc* desc, const float* Cin, const float* targets,
                       int B, float* params, float* adam_m, float* adam_v, int step, float lr,
                       void* packed, float* loss_out, float* grads_out, void* ws, size_t ws_bytes,
                       void* stream) {
  if (!ctx || !valid_desc(desc)) return TTM_EINVAL;
  if (!mlp_form_ok(desc)) {
    set_error("ttm_mlp_train_step: needs d'=3 at degree 2, 4 or 6, or d'=4 at degree 2 or 4");
    return TTM_EUNSUPPORTED;
  }
  if (!Cin || !targets || !params || !loss_out || !ws || B < 1 ||
      (lr > 0.0f && (!adam_m || !adam_v || step < 1)) || !(lr >= 0.0f)) {
    set_error("ttm_mlp_train_step: null pointer, B < 1 or bad Adam arguments");
    return TTM_EINVAL;
  }
  const size_t need = align256(mlp_train_workspace(B));
  if (ws_bytes < need) {
    set_error("ttm_mlp_train_step: workspace %zu < %zu", ws_bytes, need);
    return TTM_EWORKSPACE;
  }
  TTM_HIP(hipSetDevice(ctx->device));
  return mlp_train_step(desc->degree, desc->dprime, Cin, targets, B, params, adam_m, adam_v, step, lr,
                        static_cast<unsigned char*>(packed), loss_out, grads_out, ws,
                        static_cast<hipStream_t>(stream));
}

int ttm_find_peaks(ttm_ctx* ctx, const float* score, int nz, int ny, int nx,
                   const int32_t valid_lo[3], const int32_t valid_hi[3], int top_p, float min_dist,
                   int32_t* peaks_out, float* vals_out, int32_t* n_found, void* ws, size_t ws_bytes,
                   void* stream) {
  if (!ctx || !score || !valid_lo || !valid_hi || !peaks_out || !vals_out || !n_found || !ws ||
      top_p < 1 || !(min_dist >= 0.0f)) {
    set_error("ttm_find_peaks: null pointer, top_p < 1 or negative distance");
    return TTM_EINVAL;
  }
  const int dims[3] = {nz, ny, nx};
  for (int a = 0; a < 3; ++a) {
    if (valid_lo[a] < 0 || valid_hi[a] >= dims[a] || valid_lo[a] > valid_hi[a]) {
      set_error("ttm_find_peaks: region axis %d [%d, %d] outside [0, %d)", a, valid_lo[a],
                valid_hi[a], dims[a]);
      return TTM_EINVAL;
    }
  }
  if ((int64_t)nz * ny * nx >= (int64_t)1 << 32) {
    set_error("ttm_find_peaks: volume exceeds 2^32 voxels");
    return TTM_EUNSUPPORTED;
  }
  TTM_HIP(hipSetDevice(ctx->device));
  *n_found = 0;
  return find_peaks(score, nz, ny, nx, valid_lo, valid_hi, top_p, min_dist, peaks_out, vals_out,
                    n_found, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int ttm_find_peaks_async(ttm_ctx* ctx, const float* score, int nz, int ny, int nx,
                         const int32_t valid_lo[3], const int32_t valid_hi[3], int top_p,
                         float min_dist, int32_t* peaks_out, float* vals_out, int32_t* n_found,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !score || !valid_lo || !valid_hi || !peaks_out || !vals_out || !n_found || !ws ||
      top_p < 1 || !(min_dist >= 0.0f)) {
    set_error("ttm_find_peaks_async: null pointer, top_p < 1 or negative distance");
    return TTM_EINVAL;
  }
  const int dims[3] = {nz, ny, nx};
  for (int a = 0; a < 3; ++a) {
    if (valid_lo[a] < 0 || valid_hi[a] >= dims[a] || valid_lo[a] > valid_hi[a]) {
      set_error("ttm_find_peaks_async: region axis %d [%d, %d] outside [0, %d)", a, valid_lo[a],
                valid_hi[a], dims[a]);
      return TTM_EINVAL;
    }
  }
  if ((int64_t)nz * ny * nx >= (int64_t)1 << 31) {
    set_error("ttm_find_peaks_async: volume exceeds 2^31 voxels");
    return TTM_EUNSUPPORTED;
  }
  TTM_HIP(hipSetDevice(ctx->device));
  return find_peaks_async(score, nz, ny, nx, valid_lo, valid_hi, top_p, min_dist, peaks_out,
                          vals_out, n_found, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

static_assert(sizeof(ttm_peak_item) == 88 && offsetof(ttm_peak_item, dims) == 40,
              "ttm_peak_item layout is part of the ABI");

size_t ttm_peaks_batch_scratch_bytes(const int32_t valid_lo[3], const int32_t valid_hi[3]) {
  if (!valid_lo || !valid_hi) return 0;
  for (int a = 0; a < 3; ++a)
    if (valid_lo[a] < 0 || valid_hi[a] < valid_lo[a]) return 0;
  return peaks_batch_scratch(valid_lo, valid_hi);
}

int ttm_find_peaks_batch(ttm_ctx* ctx, const ttm_peak_item* items, int n_items,
                         const int32_t max_valid[3], void* stream) {
  if (!ctx || !items || n_items < 1 || n_items > 65535 || !max_valid) {
    set_error("ttm_find_peaks_batch: null pointer or n_items outside 1..65535");
    return TTM_EINVAL;
  }
  for (int a = 0; a < 3; ++a) {
    if (max_valid[a] < 1 || max_valid[a] > 32767) {
      set_error("ttm_find_peaks_batch: max_valid axis %d = %d outside 1..32767", a, max_valid[a]);
      return TTM_EINVAL;
    }
  }
  TTM_HIP(hipSetDevice(ctx->device));
  return find_peaks_batch(items, n_items, max_valid, static_cast<hipStream_t>(stream));
}

int ttm_fft3d_r2c(ttm_ctx* ctx, const float* x, int fft_n, void* spec, void* stream) {
  if (!ctx || !x || !spec) {
    set_error("ttm_fft3d_r2c: null pointer");
    return TTM_EINVAL;
  }
  if (!fft_ok(fft_n)) {
    set_error("ttm_fft3d_r2c: FFT edge %d not supported", fft_n);
    return TTM_EUNSUPPORTED;
  }
  TTM_HIP(hipSetDevice(ctx->device));
  RealSrc src{x, 0, fft_n, fft_n, fft_n, 0, 0, 0, nullptr, 0, 0};
  return fft3d_forward(fft_n, src, 1, static_cast<cf*>(spec), spec_elems(fft_n), ctx->twiddles,
                       static_cast<hipStream_t>(stream));
}

int ttm_fft3d_c2r(ttm_ctx* ctx, void* spec, int fft_n, float scale, float* x, void* stream) {
  if (!ctx || !x || !spec) {
    set_error("ttm_fft3d_c2r: null pointer");
    return TTM_EINVAL;
  }
  if (!fft_ok(fft_n)) {
    set_error("ttm_fft3d_c2r: FFT edge %d not supported", fft_n);
    return TTM_EUNSUPPORTED;
  }
  TTM_HIP(hipSetDevice(ctx->device));
  RealDst d{x, 0, 0, fft_n, fft_n, 0, 0, 0, fft_n, fft_n, fft_n, nullptr, 0, 0, 0, 0, 0, scale};
  cf* sp = static_cast<cf*>(spec);
  return fft3d_inverse_mul(fft_n, sp, nullptr, 0, 0, 1, nullptr, sp, spec_elems(fft_n), d,
                           ctx->twiddles, static_cast<hipStream_t>(stream));
}

}  // extern "C"
