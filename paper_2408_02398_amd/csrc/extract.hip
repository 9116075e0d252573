// extract.hip -- per-voxel score and orientation from the tensor field (gfx950).
//
// One lane per voxel; the K components of C(x) live in registers for the
// whole search.  Components are read plane by plane ([K][box] layout), so
// every load is coalesced across the wavefront.
//
// Score: c = ||C||_F = sqrt(sum_a mu_a C_a^2) (Sec. 3.2).
// Orientation (Sec. 3.1): on C / c, the SS-HOPM shift is
// alpha = max(0, -lambda_min(U)) with U the square matrix unfolding.  U is
// zero off the symmetric (n/2)-tensors, where it equals
// B[b, g] = sqrt(mu_b mu_g) C_{b+g}, so lambda_min(U) = min(0, lambda_min(B));
// B (10 x 10 at n = 6) is diagonalised by cyclic Jacobi sweeps in registers.
// Each lane then runs SS-HOPM from every start in turn, moving to its next
// start as soon as the current one has converged, so lanes of a wavefront do
// not wait for each other's slow starts.
#include "internal.hpp"
#include "mlp_core.hpp"
#include "sym_tables.hpp"

namespace ttm {


namespace {

__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

__host__ __device__ constexpr int multinom3(int a, int b, int c) {
  return factorial(a + b + c) / (factorial(a) * factorial(b) * factorial(c));
}

// g = C u^{n-1}: g_i = sum_{|beta| = n-1} mu_beta C_{beta + e_i} u^beta.
template <int N>
__device__ __forceinline__ void contract(const float (&c)[ncomp3(N)], float x, float y, float z,
                                         float& g0, float& g1, float& g2) {
  float px[N], py[N], pz[N];
  px[0] = py[0] = pz[0] = 1.0f;
#pragma unroll
  for (int k = 1; k < N; ++k) {
    px[k] = px[k - 1] * x;
    py[k] = py[k - 1] * y;
    pz[k] = pz[k - 1] * z;
  }
  g0 = g1 = g2 = 0.0f;
#pragma unroll
  for (int a = N - 1; a >= 0; --a) {
#pragma unroll
    for (int b = N - 1 - a; b >= 0; --b) {
      const int cc = N - 1 - a - b;
      const float m = (float)multinom3(a, b, cc) * (px[a] * (py[b] * pz[cc]));
      g0 = fmaf(m, c[comp_index3(N, a + 1, b)], g0);
      g1 = fmaf(m, c[comp_index3(N, a, b + 1)], g1);
      g2 = fmaf(m, c[comp_index3(N, a, b)], g2);
    }
  }
}

// H = C u^{n-2}: H_ij = sum_{|beta| = n-2} mu_beta C_{beta + e_i + e_j} u^beta,
// returned as {xx, xy, xz, yy, yz, zz}.
template <int N>
__device__ __forceinline__ void contract2(const float (&c)[ncomp3(N)], float x, float y, float z,
                                          float (&h)[6]) {
  float px[N - 1], py[N - 1], pz[N - 1];
  px[0] = py[0] = pz[0] = 1.0f;
#pragma unroll
  for (int k = 1; k < N - 1; ++k) {
    px[k] = px[k - 1] * x;
    py[k] = py[k - 1] * y;
    pz[k] = pz[k - 1] * z;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) h[i] = 0.0f;
#pragma unroll
  for (int a = N - 2; a >= 0; --a) {
#pragma unroll
    for (int b = N - 2 - a; b >= 0; --b) {
      const int cc = N - 2 - a - b;
      const float m = (float)multinom3(a, b, cc) * (px[a] * (py[b] * pz[cc]));
      h[0] = fmaf(m, c[comp_index3(N, a + 2, b)], h[0]);
      h[1] = fmaf(m, c[comp_index3(N, a + 1, b + 1)], h[1]);
      h[2] = fmaf(m, c[comp_index3(N, a + 1, b)], h[2]);
      h[3] = fmaf(m, c[comp_index3(N, a, b + 2)], h[3]);
      h[4] = fmaf(m, c[comp_index3(N, a, b + 1)], h[4]);
      h[5] = fmaf(m, c[comp_index3(N, a, b)], h[5]);
    }
  }
}

// Up to `steps` Riemannian Newton steps for max <C, u^n> on the sphere from a
// converged SS-HOPM point: tangent basis e1 = a x u/|a x u| (a = axis of the
// smallest |u_i|), e2 = u x e1; tangent Hessian (n-1) E^T H E - lambda I must be
// negative definite; the step is kept unless lambda drops by more than 1e-7.
template <int N>
__device__ __forceinline__ int newton_polish(const float (&c)[ncomp3(N)], float& ux, float& uy,
                                             float& uz, float& g0, float& g1, float& g2,
                                             float& lam, int steps) {
  int taken = 0;
  for (int s = 0; s < steps; ++s) {
    const float fx = fabsf(ux), fy = fabsf(uy), fz = fabsf(uz);
    float e1x, e1y, e1z;
    if (fx <= fy && fx <= fz) {        // a = e_x: a x u = (0, -uz, uy)
      e1x = 0.0f; e1y = -uz; e1z = uy;
    } else if (fy <= fz) {             // a = e_y: (uz, 0, -ux)
      e1x = uz; e1y = 0.0f; e1z = -ux;
    } else {                           // a = e_z: (-uy, ux, 0)
      e1x = -uy; e1y = ux; e1z = 0.0f;
    }
    const float r1 = 1.0f / sqrtf(e1x * e1x + e1y * e1y + e1z * e1z);
    e1x *= r1; e1y *= r1; e1z *= r1;
    const float e2x = uy * e1z - uz * e1y, e2y = uz * e1x - ux * e1z, e2z = ux * e1y - uy * e1x;
    float h[6];
    contract2<N>(c, ux, uy, uz, h);
    // H e1, H e2
    const float hx1 = h[0] * e1x + h[1] * e1y + h[2] * e1z;
    const float hy1 = h[1] * e1x + h[3] * e1y + h[4] * e1z;
    const float hz1 = h[2] * e1x + h[4] * e1y + h[5] * e1z;
    const float hx2 = h[0] * e2x + h[1] * e2y + h[2] * e2z;
    const float hy2 = h[1] * e2x + h[3] * e2y + h[4] * e2z;
    const float hz2 = h[2] * e2x + h[4] * e2y + h[5] * e2z;
    constexpr float nm1 = (float)(N - 1);
    const float a00 = nm1 * (e1x * hx1 + e1y * hy1 + e1z * hz1) - lam;
    const float a01 = nm1 * (e1x * hx2 + e1y * hy2 + e1z * hz2);
    const float a11 = nm1 * (e2x * hx2 + e2y * hy2 + e2z * hz2) - lam;
    const float det = a00 * a11 - a01 * a01;
    if (!(det > 0.0f && a00 + a11 < 0.0f)) break;
    const float t0 = e1x * g0 + e1y * g1 + e1z * g2, t1 = e2x * g0 + e2y * g1 + e2z * g2;
    const float inv = 1.0f / det;
    const float eta0 = -(a11 * t0 - a01 * t1) * inv;
    const float eta1 = -(a00 * t1 - a01 * t0) * inv;
    float vx = ux + eta0 * e1x + eta1 * e2x, vy = uy + eta0 * e1y + eta1 * e2y,
          vz = uz + eta0 * e1z + eta1 * e2z;
    const float rv = 1.0f / sqrtf(vx * vx + vy * vy + vz * vz);
    vx *= rv; vy *= rv; vz *= rv;
    float q0, q1, q2;
    contract<N>(c, vx, vy, vz, q0, q1, q2);
    const float lam_new = q0 * vx + q1 * vy + q2 * vz;
    ++taken;
    if (lam_new < lam - 1e-7f) break;
    ux = vx; uy = vy; uz = vz;
    g0 = q0; g1 = q1; g2 = q2;
    lam = lam_new;
  }
  return taken;
}

// Sum a per-lane count over the wavefront and add it to a device counter.
__device__ __forceinline__ void count_add(unsigned long long* ctr, unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(ctr, v);
}

// Upper-triangle storage index of (p, q), p <= q, in an M x M matrix.
__host__ __device__ constexpr int tri(int M, int p, int q) {
  return p <= q ? p * M - p * (p - 1) / 2 + (q - p) : q * M - q * (q - 1) / 2 + (p - q);
}

// Lower bound of lambda_min of B[b, g] = sqrt(mu_b mu_g) c_{b+g} over
// |b| = |g| = n/2: three cyclic Jacobi sweeps (orthogonal similarity, so the
// spectrum is unchanged) followed by Gershgorin discs, min_i (A_ii - sum |A_ij|).
// The bound is exact up to the remaining off-diagonal mass and never above
// lambda_min, so the shift -bound is never smaller than the unfolding rule's.
template <int N>
__device__ __forceinline__ float unfolding_lambda_min(const float (&c)[ncomp3(N)]) {
  constexpr int H = N / 2;
  constexpr int M = ncomp3(H);
  constexpr Sym3<H> hs{};
  float A[M * (M + 1) / 2];
#pragma unroll
  for (int p = 0; p < M; ++p) {
#pragma unroll
    for (int q = p; q < M; ++q) {
      const float s = sqrtf(hs.mu[p] * hs.mu[q]);
      A[tri(M, p, q)] = s * c[comp_index3(N, hs.ax[p] + hs.ax[q], hs.ay[p] + hs.ay[q])];
    }
  }
  for (int sweep = 0; sweep < 3; ++sweep) {
#pragma unroll
    for (int p = 0; p < M - 1; ++p) {
#pragma unroll
      for (int q = p + 1; q < M; ++q) {
        const float apq = A[tri(M, p, q)];
        const float app = A[tri(M, p, p)], aqq = A[tri(M, q, q)];
        // theta = (aqq - app) / (2 apq); apq = 0 gives t = 0 (no rotation)
        const float theta = 0.5f * (aqq - app) / apq;
        const float t = copysignf(1.0f / (fabsf(theta) + sqrtf(fmaf(theta, theta, 1.0f))), theta);
        const float tt = (apq == 0.0f || !(fabsf(theta) < 1e30f)) ? 0.0f : t;
        const float cs = 1.0f / sqrtf(fmaf(tt, tt, 1.0f));
        const float sn = tt * cs;
        A[tri(M, p, p)] = app - tt * apq;
        A[tri(M, q, q)] = aqq + tt * apq;
        A[tri(M, p, q)] = 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) {
          if (r == p || r == q) continue;
          const float arp = A[tri(M, r, p)], arq = A[tri(M, r, q)];
          A[tri(M, r, p)] = cs * arp - sn * arq;
          A[tri(M, r, q)] = sn * arp + cs * arq;
        }
      }
    }
  }
  float lmin = INFINITY;
#pragma unroll
  for (int p = 0; p < M; ++p) {
    float rad = 0.0f;
#pragma unroll
    for (int q = 0; q < M; ++q)
      if (q != p) rad += fabsf(A[tri(M, p, q)]);
    lmin = fminf(lmin, A[tri(M, p, p)] - rad);
  }
  return lmin;
}

// SS-HOPM from one start (then Newton polish).  Returns lambda on C/||C||_F;
// u is updated in place; `conv` tells whether |delta lambda| <= tol was reached.
template <int N>
__device__ __forceinline__ float refine(const float (&c)[ncomp3(N)], float alpha, float& ux,
                                        float& uy, float& uz, float tol, int max_iter, int newton,
                                        unsigned long long& n_steps, unsigned long long& n_newton,
                                        bool& conv) {
  {
    const float r = 1.0f / sqrtf(ux * ux + uy * uy + uz * uz);
    ux *= r; uy *= r; uz *= r;
  }
  float g0, g1, g2;
  contract<N>(c, ux, uy, uz, g0, g1, g2);
  float lam = g0 * ux + g1 * uy + g2 * uz;
  conv = false;
  for (int it = 0; it < max_iter; ++it) {
    const float wx = fmaf(alpha, ux, g0), wy = fmaf(alpha, uy, g1), wz = fmaf(alpha, uz, g2);
    const float r = 1.0f / sqrtf(wx * wx + wy * wy + wz * wz);
    ux = wx * r; uy = wy * r; uz = wz * r;
    contract<N>(c, ux, uy, uz, g0, g1, g2);
    const float lam_new = g0 * ux + g1 * uy + g2 * uz;
    ++n_steps;
    const bool done = fabsf(lam_new - lam) <= tol;
    lam = lam_new;
    if (done) {
      conv = true;
      break;
    }
  }
  n_newton += newton_polish<N>(c, ux, uy, uz, g0, g1, g2, lam, newton);
  return lam;
}

// Best of SS-HOPM (+ polish) from every fixed start; a lane moves to its next
// start as soon as the current one ends.  Returns lambda on C/||C||_F.
template <int N>
__device__ __forceinline__ float multistart(const float (&c)[ncomp3(N)], float alpha,
                                            const float* st, int n_starts, float tol, int max_iter,
                                            int newton, float& bx, float& by, float& bz,
                                            unsigned long long& n_steps,
                                            unsigned long long& n_newton) {
  float best = -INFINITY;
  for (int s = 0; s < n_starts; ++s) {
    float ux = st[3 * s], uy = st[3 * s + 1], uz = st[3 * s + 2];
    bool conv;
    const float lam = refine<N>(c, alpha, ux, uy, uz, tol, max_iter, newton, n_steps, n_newton, conv);
    if (lam > best) {
      best = lam;
      bx = ux; by = uy; bz = uz;
    }
  }
  return best;
}

__device__ __forceinline__ void canonical(float& x, float& y, float& z) {
  // u and -u are the same answer: make the last non-zero coordinate positive
  const float sg = (z != 0.0f) ? z : ((y != 0.0f) ? y : x);
  if (sg < 0.0f) {
    x = -x; y = -y; z = -z;
  }
}

// Load the K components of box voxel v, return ||C||_F.
template <int N>
__device__ __forceinline__ float load_tensor(const ExtractArgs& a, size_t v, float (&c)[ncomp3(N)]) {
  constexpr int K = ncomp3(N);
  constexpr Sym3<N> sy{};
  if (a.in_dtype == 1) {
    const unsigned short* p = reinterpret_cast<const unsigned short*>(a.C);
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = bf16_to_f32(p[k * a.plane + v]);
  } else {
    const float* p = reinterpret_cast<const float*>(a.C);
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = p[k * a.plane + v];
  }
  float f2 = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) f2 = fmaf(sy.mu[k] * c[k], c[k], f2);
  return sqrtf(f2);
}

__device__ __forceinline__ size_t map_index(const ExtractArgs& a, size_t v) {
  const int vx = (int)(v % a.bx), vy = (int)((v / a.bx) % a.by), vz = (int)(v / ((size_t)a.bx * a.by));
  return ((size_t)(a.oz + vz) * a.dy + (a.oy + vy)) * a.dx + (a.ox + vx);
}

template <int N, bool MLP>
__global__ __launch_bounds__(256) void k_extract(ExtractArgs a) {
  constexpr int K = ncomp3(N);
  constexpr Sym3<N> sy{};
  __shared__ float st[64 * 3];
  for (int i = threadIdx.x; i < a.n_starts * 3; i += blockDim.x) st[i] = a.starts[i];
  __syncthreads();
  const size_t v0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = v0 < a.plane;
  const size_t v = active ? v0 : a.plane - 1;   // inactive lanes recompute the last voxel, write nothing
  unsigned long long n_steps = 0, n_newton = 0, n_oriented = 0;
  float c[K];
  const float cn = load_tensor<N>(a, v, c);
  const size_t o = map_index(a, v);
  if ((a.mode & 1) && active) a.score[o] = cn;
  if constexpr (N >= 2) {
    if (a.mode & 2) {
      float lam_best = 0.0f, bx0 = 0.0f, by0 = 0.0f, bz0 = 0.0f;
      const float inv = cn > 0.0f ? 1.0f / cn : 0.0f;
      if constexpr (MLP) {
        // ---- learned start: features -> BF16 MLP on the matrix cores;
        // per wavefront [64][64] bf16 activations and [64][4] outputs
        __shared__ unsigned short hs[4][64 * kMlpHid];
        __shared__ float ys[4][64 * 4];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        unsigned short* xs = &hs[wv][64 * kMlpIn];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k)
          xs[lane * kMlpIn + k] = k < K ? bf16_bits(sqrtf(sy.mu[k]) * c[k] * inv) : (unsigned short)0;
        __syncthreads();
        float y0, y1, y2;
        mlp_forward_wave(hs[wv], ys[wv], a.mlp, lane, y0, y1, y2);
        const float ny = sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
        bool fallback = !(ny > 0.0f);
        float ux = fallback ? st[0] : y0, uy = fallback ? st[1] : y1, uz = fallback ? st[2] : y2;
        if (a.start_only) {
          const float r = 1.0f / sqrtf(ux * ux + uy * uy + uz * uz);
          bx0 = ux * r; by0 = uy * r; bz0 = uz * r;
          fallback = false;
        } else if (cn > 0.0f) {
#pragma unroll
          for (int k = 0; k < K; ++k) c[k] *= inv;
          const float alpha = fmaxf(0.0f, -unfolding_lambda_min<N>(c));
          bool conv;
          const float lam = refine<N>(c, alpha, ux, uy, uz, a.tol, a.max_iter, a.newton, n_steps,
                                      n_newton, conv);
          // screening: SS-HOPM never lowers lambda, so a fixed start that already
          // scores above the learned answer proves the multistart answer is higher
          bool beaten = false;
          for (int s = 0; s < (a.screen ? a.n_starts : 0); ++s) {
            const float sx = st[3 * s], sy = st[3 * s + 1], sz = st[3 * s + 2];
            const float rs = 1.0f / sqrtf(sx * sx + sy * sy + sz * sz);
            float q0, q1, q2;
            contract<N>(c, sx * rs, sy * rs, sz * rs, q0, q1, q2);
            beaten = beaten || ((q0 * sx + q1 * sy + q2 * sz) * rs > lam);
          }
          fallback = fallback || !conv || !(lam >= a.kappa) || (beaten && a.screen);
          bx0 = ux; by0 = uy; bz0 = uz;
          canonical(bx0, by0, bz0);
          lam_best = lam * cn;
          n_oriented = 1;
        } else {
          fallback = false;
        }
        if (active && fallback) {
          const unsigned slot = atomicAdd(a.fb_count, 1u);
          a.fb_queue[slot] = (unsigned)v;
        }
      } else if (cn > 0.0f) {
        // ---- plain multistart
#pragma unroll
        for (int k = 0; k < K; ++k) c[k] *= inv;
        const float alpha = fmaxf(0.0f, -unfolding_lambda_min<N>(c));
        const float lam = multistart<N>(c, alpha, st, a.n_starts, a.tol, a.max_iter, a.newton, bx0,
                                        by0, bz0, n_steps, n_newton);
        canonical(bx0, by0, bz0);
        lam_best = lam * cn;
        n_oriented = 1;
      }
      if (active) {
        if (a.lam) a.lam[o] = lam_best;
        if (a.dir) {
          a.dir[3 * o + 0] = bx0;
          a.dir[3 * o + 1] = by0;
          a.dir[3 * o + 2] = bz0;
        }
      }
      if (a.counters) {
        if (!active) n_steps = n_newton = n_oriented = 0;
        count_add(a.counters + 0, n_steps);
        count_add(a.counters + 1, n_newton);
        count_add(a.counters + 2, n_oriented);
      }
    }
  }
}

// Fallback of the learned start: the voxels queued by k_extract run the full
// multistart search; the better of that and the learned answer is kept.
template <int N>
__global__ __launch_bounds__(256) void k_extract_fallback(ExtractArgs a) {
  constexpr int K = ncomp3(N);
  __shared__ float st[64 * 3];
  for (int i = threadIdx.x; i < a.n_starts * 3; i += blockDim.x) st[i] = a.starts[i];
  __syncthreads();
  const unsigned count = *a.fb_count;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.fb_total) atomicAdd(a.fb_total, (int)count);
  if (i >= count) return;
  const size_t v = a.fb_queue[i];
  float c[K];
  const float cn = load_tensor<N>(a, v, c);
  if (!(cn > 0.0f)) return;
  const float inv = 1.0f / cn;
#pragma unroll
  for (int k = 0; k < K; ++k) c[k] *= inv;
  const float alpha = fmaxf(0.0f, -unfolding_lambda_min<N>(c));
  unsigned long long n_steps = 0, n_newton = 0;
  float bx0 = 0.0f, by0 = 0.0f, bz0 = 0.0f;
  const float lam = multistart<N>(c, alpha, st, a.n_starts, a.tol, a.max_iter, a.newton, bx0, by0,
                                  bz0, n_steps, n_newton) * cn;
  const size_t o = map_index(a, v);
  if (lam > a.lam[o]) {
    canonical(bx0, by0, bz0);
    a.lam[o] = lam;
    a.dir[3 * o + 0] = bx0;
    a.dir[3 * o + 1] = by0;
    a.dir[3 * o + 2] = bz0;
  }
  if (a.counters) {
    atomicAdd(a.counters + 0, n_steps);
    atomicAdd(a.counters + 1, n_newton);
  }
}

}  // namespace

template <int N>
int launch_n(const ExtractArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)((a.plane + 255) / 256);
  if constexpr (N >= 2) {
    if ((a.mode & 6) == 6) {
      hipLaunchKernelGGL((k_extract<N, true>), dim3(nb), dim3(256), 0, s, a);
      if (!a.start_only) hipLaunchKernelGGL(k_extract_fallback<N>, dim3(nb), dim3(256), 0, s, a);
    } else {
      hipLaunchKernelGGL((k_extract<N, false>), dim3(nb), dim3(256), 0, s, a);
    }
  } else {
    hipLaunchKernelGGL((k_extract<N, false>), dim3(nb), dim3(256), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : hip_status(e, "extract launch");
}

int launch_extract(int degree, const ExtractArgs& a, hipStream_t s) {
  switch (degree) {
    case 0: return launch_n<0>(a, s);
    case 2: return launch_n<2>(a, s);
    case 4: return launch_n<4>(a, s);
    case 6: return launch_n<6>(a, s);
    default: set_error("ttm_extract: degree %d not built for d'=3 extraction", degree); return -4;
  }
}

}  // namespace ttm
