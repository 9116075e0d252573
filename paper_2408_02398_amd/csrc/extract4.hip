// extract4.hip -- per-voxel score and orientation for the quaternion form
// (d' = 4, the paper's construction: v_q = q, Sec. 3, Alg. 1).
//
// The tensor C(x) is a degree-n symmetric tensor over R^4 with
// K = binom(n + 3, 3) independent components, alpha = (aw, ax, ay, az) in
// graded-lex order (descending aw, then ax, then ay); component alpha holds
// the full-tensor entry, so <C, q^n> = sum_a mu_a C_a q^a, mu_a = n!/prod(a_i!).
//
// Score: c = ||C||_F (Sec. 3.2).  Orientation (Sec. 3.1): the dominant
// eigenpair of C / c on the unit sphere S^3 of quaternions by SS-HOPM with
// the unfolding shift, from every fixed start, each answer polished by
// Riemannian Newton steps, the largest lambda winning (first on ties).  The
// quaternion and its negative are one rotation; the answer is signed so that
// its first non-zero coordinate (w) is positive.
//
// The runs use the pooled scheme of the d' = 3 kernels: k_prepare4 (score and
// shift per voxel), persistent k_runs4 wavefronts that drain a queue of
// (voxel, start) runs and refill lanes as runs end, k_reduce4 (polish each
// run, keep the best).  The tangent space of S^3 at u has the orthonormal
// basis u*i, u*j, u*k (quaternion products with the imaginary units), so the
// Newton system is a 3 x 3 Cholesky solve.
//
// Learned start (degree 2 and 4, K <= 48): k_learned4 runs the network
// (K -> 64 -> 64 -> 4 on the BF16 matrix cores) on 64 voxels per wavefront,
// SS-HOPM from q0 = y / |y| with the unfolding shift, the Newton polish, the
// certification and the screen by the fixed starts, as the d' = 3 learned
// start without its Newton-first search; the voxels that fall back are
// listed and take the pooled multistart above, whose answer replaces the
// learned one only where its lambda is larger.
#include "extract_items.hpp"
#include "internal.hpp"
#include "mlp_core.hpp"
#include "sym_tables.hpp"

namespace ttm {

namespace {

constexpr int kRefill4 = 8;        // a pooled wavefront refills once this many lanes wait
constexpr int kPoolGroups4 = 4096; // persistent pooled grid (one wavefront per group)
constexpr int kStartBlock4 = 16;   // starts whose run results are held at once
constexpr unsigned kItemGroups4 = 1024;
constexpr float kShiftMargin4 = 1e-5f;
constexpr int kShiftSteps4 = 12;

// Workspace: header (64-bit pool counters, one per start block), shift per
// voxel, carried best (u, lambda), run results [start][voxel] (u, lambda).
struct Ws4 {
  unsigned long long* ctr;   // [0, 4): pool counters; [kListCount4]: fallback list length
  float* alpha;
  float4* best_u;
  float* best_l;
  float4* res_u;
  float* res_l;
  unsigned* list;            // learned start: voxels that fall back
};
constexpr int kListCount4 = 16;

__host__ __device__ inline size_t al256_4(size_t b) { return (b + 255) & ~(size_t)255; }

__host__ __device__ inline Ws4 ws4_layout(void* base, size_t plane) {
  char* p = static_cast<char*>(base);
  Ws4 w;
  w.ctr = reinterpret_cast<unsigned long long*>(p);
  p += 256;
  w.alpha = reinterpret_cast<float*>(p);
  p += al256_4(plane * 4);
  w.best_u = reinterpret_cast<float4*>(p);
  p += al256_4(plane * 16);
  w.best_l = reinterpret_cast<float*>(p);
  p += al256_4(plane * 4);
  w.res_u = reinterpret_cast<float4*>(p);
  p += al256_4((size_t)kStartBlock4 * plane * 16);
  w.res_l = reinterpret_cast<float*>(p);
  p += al256_4((size_t)kStartBlock4 * plane * 4);
  w.list = reinterpret_cast<unsigned*>(p);
  return w;
}

// The items of a pass: every box voxel (list == nullptr), or the listed ones.
struct Items4 {
  const unsigned* list;
  const unsigned long long* count;
  __device__ __forceinline__ size_t n(const ExtractArgs& a) const {
    return list ? (size_t)*count : a.plane;
  }
  __device__ __forceinline__ size_t voxel(size_t j) const { return list ? (size_t)list[j] : j; }
};

__device__ __forceinline__ float bf16_to_f32_4(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

using Vox4 = VoxelRef;
__device__ __forceinline__ Vox4 vox4(const ExtractArgs& a, size_t v) { return voxel_ref(a, v); }

// Load the K components of a voxel; returns ||C||_F.
template <int N>
__device__ __forceinline__ float load4_at(const ExtractArgs& a, const Vox4& r, float (&c)[ncomp4(N)]) {
  constexpr int K = ncomp4(N);
  constexpr Sym4<N> sy{};
  if (a.in_dtype == 1) {
    const unsigned short* p = reinterpret_cast<const unsigned short*>(r.C);
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = bf16_to_f32_4(p[k * r.stride + r.lv]);
  } else {
    const float* p = reinterpret_cast<const float*>(r.C);
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = p[k * r.stride + r.lv];
  }
  float f2 = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) f2 = fmaf(sy.mu[k] * c[k], c[k], f2);
  return sqrtf(f2);
}

template <int N>
__device__ __forceinline__ float load4(const ExtractArgs& a, size_t v, float (&c)[ncomp4(N)]) {
  return load4_at<N>(a, vox4(a, v), c);
}

// g = C u^{n-1}: g_i = sum_{|beta| = n-1} mu_beta C_{beta + e_i} u^beta.
template <int N>
__device__ __forceinline__ void contract4(const float (&c)[ncomp4(N)], const float (&u)[4],
                                          float (&g)[4]) {
  float p[4][N];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    p[d][0] = 1.0f;
#pragma unroll
    for (int k = 1; k < N; ++k) p[d][k] = p[d][k - 1] * u[d];
  }
  g[0] = g[1] = g[2] = g[3] = 0.0f;
#pragma unroll
  for (int a = N - 1; a >= 0; --a) {
#pragma unroll
    for (int b = N - 1 - a; b >= 0; --b) {
#pragma unroll
      for (int cc = N - 1 - a - b; cc >= 0; --cc) {
        const int dd = N - 1 - a - b - cc;
        const float m = (float)multinom4(a, b, cc, dd) * ((p[0][a] * p[1][b]) * (p[2][cc] * p[3][dd]));
        g[0] = fmaf(m, c[comp_index4(N, a + 1, b, cc)], g[0]);
        g[1] = fmaf(m, c[comp_index4(N, a, b + 1, cc)], g[1]);
        g[2] = fmaf(m, c[comp_index4(N, a, b, cc + 1)], g[2]);
        g[3] = fmaf(m, c[comp_index4(N, a, b, cc)], g[3]);
      }
    }
  }
}

// H = C u^{n-2}, symmetric 4 x 4, packed {00, 01, 02, 03, 11, 12, 13, 22, 23, 33}.
template <int N>
__device__ __forceinline__ void contract4_2(const float (&c)[ncomp4(N)], const float (&u)[4],
                                            float (&h)[10]) {
  float p[4][N - 1];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    p[d][0] = 1.0f;
#pragma unroll
    for (int k = 1; k < N - 1; ++k) p[d][k] = p[d][k - 1] * u[d];
  }
#pragma unroll
  for (int i = 0; i < 10; ++i) h[i] = 0.0f;
#pragma unroll
  for (int a = N - 2; a >= 0; --a) {
#pragma unroll
    for (int b = N - 2 - a; b >= 0; --b) {
#pragma unroll
      for (int cc = N - 2 - a - b; cc >= 0; --cc) {
        const int dd = N - 2 - a - b - cc;
        const float m = (float)multinom4(a, b, cc, dd) * ((p[0][a] * p[1][b]) * (p[2][cc] * p[3][dd]));
        h[0] = fmaf(m, c[comp_index4(N, a + 2, b, cc)], h[0]);
        h[1] = fmaf(m, c[comp_index4(N, a + 1, b + 1, cc)], h[1]);
        h[2] = fmaf(m, c[comp_index4(N, a + 1, b, cc + 1)], h[2]);
        h[3] = fmaf(m, c[comp_index4(N, a + 1, b, cc)], h[3]);
        h[4] = fmaf(m, c[comp_index4(N, a, b + 2, cc)], h[4]);
        h[5] = fmaf(m, c[comp_index4(N, a, b + 1, cc + 1)], h[5]);
        h[6] = fmaf(m, c[comp_index4(N, a, b + 1, cc)], h[6]);
        h[7] = fmaf(m, c[comp_index4(N, a, b, cc + 2)], h[7]);
        h[8] = fmaf(m, c[comp_index4(N, a, b, cc + 1)], h[8]);
        h[9] = fmaf(m, c[comp_index4(N, a, b, cc)], h[9]);
      }
    }
  }
}

__device__ __forceinline__ float dot4(const float (&a)[4], const float (&b)[4]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

// Tangent model of max <C, q^n> on S^3 at u (g = C u^{n-1}, lambda = g.u):
// the tangent basis E = (u*i, u*j, u*k), m = -A with A = (n-1) E^T H E -
// lambda I the tangent Hessian (H = C u^{n-2}), and the tangent gradient t = E^T g.
template <int N>
__device__ __forceinline__ void tangent_model4(const float (&c)[ncomp4(N)], const float (&u)[4],
                                               const float (&g)[4], float lam, float (&E)[3][4],
                                               float (&m)[3][3], float (&t)[3]) {
  E[0][0] = -u[1]; E[0][1] = u[0];  E[0][2] = u[3];  E[0][3] = -u[2];
  E[1][0] = -u[2]; E[1][1] = -u[3]; E[1][2] = u[0];  E[1][3] = u[1];
  E[2][0] = -u[3]; E[2][1] = u[2];  E[2][2] = -u[1]; E[2][3] = u[0];
  float h[10];
  contract4_2<N>(c, u, h);
  float HE[3][4];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float* e = E[k];
    HE[k][0] = h[0] * e[0] + h[1] * e[1] + h[2] * e[2] + h[3] * e[3];
    HE[k][1] = h[1] * e[0] + h[4] * e[1] + h[5] * e[2] + h[6] * e[3];
    HE[k][2] = h[2] * e[0] + h[5] * e[1] + h[7] * e[2] + h[8] * e[3];
    HE[k][3] = h[3] * e[0] + h[6] * e[1] + h[8] * e[2] + h[9] * e[3];
  }
  constexpr float nm1 = (float)(N - 1);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float eh = E[i][0] * HE[j][0] + E[i][1] * HE[j][1] + E[i][2] * HE[j][2] + E[i][3] * HE[j][3];
      m[i][j] = -(nm1 * eh - (i == j ? lam : 0.0f));
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) t[k] = E[k][0] * g[0] + E[k][1] * g[1] + E[k][2] * g[2] + E[k][3] * g[3];
}

// Cholesky solve of m e = t for symmetric m; false unless m is positive definite.
__device__ __forceinline__ bool solve_pd3(const float (&m)[3][3], const float (&t)[3], float (&e)[3]) {
  const float p0 = m[0][0];
  if (!(p0 > 0.0f)) return false;
  const float r00 = sqrtf(p0);
  const float l10 = m[1][0] / r00, l20 = m[2][0] / r00;
  const float p1 = m[1][1] - l10 * l10;
  if (!(p1 > 0.0f)) return false;
  const float r11 = sqrtf(p1);
  const float l21 = (m[2][1] - l20 * l10) / r11;
  const float p2 = m[2][2] - l20 * l20 - l21 * l21;
  if (!(p2 > 0.0f)) return false;
  const float r22 = sqrtf(p2);
  const float y0 = t[0] / r00, y1 = (t[1] - l10 * y0) / r11, y2 = (t[2] - l20 * y0 - l21 * y1) / r22;
  e[2] = y2 / r22;
  e[1] = (y1 - l21 * e[2]) / r11;
  e[0] = (y0 - l10 * e[1] - l20 * e[2]) / r00;
  return true;
}

// Riemannian Newton direction on S^3 at u: d = E eta with -A eta = E^T g,
// where -A must be positive definite (else there is no step).
template <int N>
__device__ __forceinline__ bool newton_dir4(const float (&c)[ncomp4(N)], const float (&u)[4],
                                            const float (&g)[4], float lam, float (&dv)[4]) {
  float E[3][4], m[3][3], t[3], e[3];
  tangent_model4<N>(c, u, g, lam, E, m, t);
  if (!solve_pd3(m, t, e)) return false;
#pragma unroll
  for (int d = 0; d < 4; ++d) dv[d] = e[0] * E[0][d] + e[1] * E[1][d] + e[2] * E[2][d];
  return true;
}

// Up to `steps` Newton steps from an SS-HOPM end point; a step is kept unless
// lambda drops by more than 1e-7.  (g, lambda) hold C u^{n-1} and <C, u^n>.
template <int N>
__device__ __forceinline__ int newton_polish4(const float (&c)[ncomp4(N)], float (&u)[4],
                                              float (&g)[4], float& lam, int steps) {
  int taken = 0;
  for (int s = 0; s < steps; ++s) {
    float dv[4];
    if (!newton_dir4<N>(c, u, g, lam, dv)) break;
    ++taken;
    float v[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) v[d] = u[d] + dv[d];
    const float rv = 1.0f / sqrtf(dot4(v, v));
#pragma unroll
    for (int d = 0; d < 4; ++d) v[d] *= rv;
    float q[4];
    contract4<N>(c, v, q);
    const float lam_v = dot4(q, v);
    if (lam_v < lam - 1e-7f) break;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      u[d] = v[d];
      g[d] = q[d];
    }
    lam = lam_v;
  }
  return taken;
}

// Lower bound of lambda_min of the unfolding's symmetric block
// B[b, g] = sqrt(mu_b mu_g) c_{b+g}, |b| = |g| = n/2 (Gershgorin, narrowed by
// bisection with Cholesky tests, minus a rounding margin), as for d' = 3.
__host__ __device__ constexpr int tri4(int M, int p, int q) {
  return p <= q ? p * M - p * (p - 1) / 2 + (q - p) : q * M - q * (q - 1) / 2 + (p - q);
}

template <int N>
__device__ __forceinline__ float unfold4(const float (&c)[ncomp4(N)], int p, int q) {
  constexpr Sym4<N / 2> hs{};
  return sqrtf(hs.mu[p] * hs.mu[q]) *
         c[comp_index4(N, hs.e[p][0] + hs.e[q][0], hs.e[p][1] + hs.e[q][1], hs.e[p][2] + hs.e[q][2])];
}

template <int N>
__device__ __forceinline__ float unfolding_lambda_min4(const float (&c)[ncomp4(N)]) {
  constexpr int M = ncomp4(N / 2);
  float lo = INFINITY, hi = INFINITY;
#pragma unroll
  for (int p = 0; p < M; ++p) {
    float rad = 0.0f;
#pragma unroll
    for (int q = 0; q < M; ++q)
      if (q != p) rad += fabsf(unfold4<N>(c, p, q));
    const float d = unfold4<N>(c, p, p);
    lo = fminf(lo, d - rad);
    hi = fminf(hi, d);
  }
  for (int step = 0; step < kShiftSteps4; ++step) {
    const float mid = 0.5f * (lo + hi);
    float R[M * (M + 1) / 2];
    bool pd = true;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      float d = unfold4<N>(c, j, j) - mid;
#pragma unroll
      for (int k = 0; k < j; ++k) d = fmaf(-R[tri4(M, k, j)], R[tri4(M, k, j)], d);
      pd = pd && d > 0.0f;
      const float r = pd ? 1.0f / sqrtf(d) : 0.0f;
      R[tri4(M, j, j)] = d * r;
#pragma unroll
      for (int i = j + 1; i < M; ++i) {
        float e = unfold4<N>(c, j, i);
#pragma unroll
        for (int k = 0; k < j; ++k) e = fmaf(-R[tri4(M, k, j)], R[tri4(M, k, i)], e);
        R[tri4(M, j, i)] = e * r;
      }
    }
    if (pd) lo = mid; else hi = mid;
  }
  return lo - kShiftMargin4;
}

__device__ __forceinline__ void count_add4(unsigned long long* ctr, unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(ctr, v);
}

template <int N>
__global__ __launch_bounds__(256) void k_score4(ExtractArgs a) {
  const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= a.plane) return;
  float c[ncomp4(N)];
  const Vox4 r = vox4(a, v);
  r.score[r.o] = load4_at<N>(a, r, c);
}

// Score (mode bit 1, all voxels only) and the SS-HOPM shift of every item,
// shift stored per item.
template <int N>
__global__ __launch_bounds__(256) void k_prepare4(ExtractArgs a, Items4 it) {
  const Ws4 w = ws4_layout(a.ws, a.plane);
  unsigned long long n_shift = 0;
  const size_t n = it.n(a);
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (size_t)gridDim.x * blockDim.x) {
    const size_t v = it.voxel(j);
    float c[ncomp4(N)];
    const Vox4 r = vox4(a, v);
    const float cn = load4_at<N>(a, r, c);
    if ((a.mode & 1) && r.score && !it.list) r.score[r.o] = cn;
    float alpha = 0.0f;
    if (cn > 0.0f) {
      const float inv = 1.0f / cn;
#pragma unroll
      for (int k = 0; k < ncomp4(N); ++k) c[k] *= inv;
      alpha = fmaxf(0.0f, -unfolding_lambda_min4<N>(c));
      n_shift += 1;
    }
    w.alpha[j] = alpha;
  }
  if (a.counters) count_add4(a.counters + 3, n_shift);
}

// Persistent pooled SS-HOPM runs over (item, start) pairs: run q of a chunk
// is item chunk_base + q / R with start s0 + q % R.  A wavefront takes up to
// 64 voxels at a time from a global counter and stages their normalised
// tensors and shifts in LDS; lanes whose run has ended take the chunk's next
// runs as soon as kRefill4 of them wait.  A run ends at |delta lambda| <= tol
// or max_iter updates; its (u, lambda) goes to slot (q % R) * plane + item.
template <int N>
__global__ __launch_bounds__(64) void k_runs4(ExtractArgs a, Items4 it, int R, int s0,
                                              unsigned long long* ctr) {
  constexpr int K = ncomp4(N);
  constexpr Sym4<N> sy{};
  __shared__ float st[64 * 4];
  __shared__ float cs[K][64];
  __shared__ float ca[64];
  __shared__ float cz[64];
  const int lane = threadIdx.x;
  for (int i = lane; i < a.n_starts * 4; i += 64) st[i] = a.starts[i];
  __syncthreads();
  const Ws4 w = ws4_layout(a.ws, a.plane);
  const unsigned n_items = (unsigned)it.n(a);
  const unsigned per_wave = (n_items + 4 * gridDim.x - 1) / (4 * gridDim.x);
  const unsigned chunk = per_wave < 1 ? 1 : (per_wave > 64 ? 64 : per_wave);
  unsigned chunk_base = 0;
  int chunk_runs = 0, next_q = 0;
  bool exhausted = n_items == 0;
  float c[K];
#pragma unroll
  for (int k = 0; k < K; ++k) c[k] = 0.0f;
  float alpha = 0.0f, u[4] = {0.0f, 0.0f, 0.0f, 0.0f}, g[4] = {0.0f, 0.0f, 0.0f, 0.0f}, lam = 0.0f;
  int iters = 0, s = 0;
  unsigned j = 0;
  bool first = false, busy = false;
  unsigned long long n_steps = 0, n_runs = 0;
  while (true) {
    unsigned long long waiting = __ballot(!busy);
    int n_wait = __popcll(waiting);
    if (n_wait == 64 && exhausted && next_q == chunk_runs) break;
    if (n_wait >= kRefill4 || n_wait == 64) {
      while (n_wait > 0) {
        if (next_q == chunk_runs) {
          if (exhausted) break;
          unsigned long long base = 0;
          if (lane == 0) base = atomicAdd(ctr, (unsigned long long)chunk);
          base = __shfl(base, 0);
          if (base >= n_items) {
            exhausted = true;
            break;
          }
          const int cnt = (n_items - base) < chunk ? (int)(n_items - base) : (int)chunk;
          if (base + chunk >= n_items) exhausted = true;
          chunk_base = (unsigned)base;
          chunk_runs = cnt * R;
          next_q = 0;
          __syncthreads();   // the previous chunk's LDS reads are complete
          if (lane < cnt) {
            const size_t jj = chunk_base + lane;
            float cv[K];
            const float cn = load4<N>(a, it.voxel(jj), cv);
            const float inv = cn > 0.0f ? 1.0f / cn : 0.0f;
#pragma unroll
            for (int k = 0; k < K; ++k) cs[k][lane] = cv[k] * inv;
            cz[lane] = cn;
            ca[lane] = w.alpha[jj];
          }
          __syncthreads();
        }
        const int avail = chunk_runs - next_q;
        const int take = n_wait < avail ? n_wait : avail;
        if (!busy) {
          const int rank = __popcll(waiting & ((1ull << lane) - 1ull));
          if (rank < take) {
            const int q = next_q + rank;
            const int jl = q / R;
            s = q % R;
            j = chunk_base + jl;
            if (cz[jl] > 0.0f) {
#pragma unroll
              for (int k = 0; k < K; ++k) c[k] = cs[k][jl];
              alpha = ca[jl];
              const float* sv = &st[4 * (s0 + s)];
              const float rs = 1.0f / sqrtf(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2] + sv[3] * sv[3]);
#pragma unroll
              for (int d = 0; d < 4; ++d) u[d] = sv[d] * rs;
              iters = 0;
              first = true;
              busy = true;
              ++n_runs;
            } else {
              w.res_u[(size_t)s * a.plane + j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
              w.res_l[(size_t)s * a.plane + j] = 0.0f;
            }
          }
        }
        next_q += take;
        waiting = __ballot(!busy);
        n_wait = __popcll(waiting);
      }
    }
    if (busy) {
      if (!first) {
        float v[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) v[d] = fmaf(alpha, u[d], g[d]);
        const float rn = rsqrtf(dot4(v, v));
#pragma unroll
        for (int d = 0; d < 4; ++d) u[d] = v[d] * rn;
      }
      contract4<N>(c, u, g);
      const float lam_new = dot4(g, u);
      bool end = false;
      if (first) {
        first = false;
      } else {
        ++iters;
        ++n_steps;
        end = fabsf(lam_new - lam) <= a.tol || iters >= a.max_iter;
      }
      lam = lam_new;
      if (end) {
        w.res_u[(size_t)s * a.plane + j] = make_float4(u[0], u[1], u[2], u[3]);
        w.res_l[(size_t)s * a.plane + j] = lam;
        busy = false;
      }
    }
  }
  (void)sy;
  if (a.counters) {
    count_add4(a.counters + 0, n_steps);
    count_add4(a.counters + 4, n_runs);
  }
}

// Per item: every run of one start block takes the Newton polish and the
// largest polished lambda wins (first in start order on ties), carried across
// blocks; after the last block the winner is signed (w >= 0) and written
// (merge: only where its lambda beats the answer already in the maps).
template <int N>
__global__ __launch_bounds__(256) void k_reduce4(ExtractArgs a, Items4 it, int nsb, int first_block,
                                                 int last_block, int merge) {
  constexpr int K = ncomp4(N);
  const Ws4 w = ws4_layout(a.ws, a.plane);
  unsigned long long n_newton = 0, n_oriented = 0;
  const size_t n = it.n(a);
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (size_t)gridDim.x * blockDim.x) {
    const size_t v = it.voxel(j);
    float c[K];
    const Vox4 rv = vox4(a, v);
    const float cn = load4_at<N>(a, rv, c);
    float4 bu = first_block ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : w.best_u[j];
    float bl = first_block ? -INFINITY : w.best_l[j];
    if (cn > 0.0f) {
      const float inv = 1.0f / cn;
#pragma unroll
      for (int k = 0; k < K; ++k) c[k] *= inv;
      for (int s = 0; s < nsb; ++s) {
        const float4 r = w.res_u[(size_t)s * a.plane + j];
        float u[4] = {r.x, r.y, r.z, r.w}, g[4];
        contract4<N>(c, u, g);
        float lam = dot4(g, u);
        n_newton += newton_polish4<N>(c, u, g, lam, a.newton);
        if (lam > bl) {
          bl = lam;
          bu = make_float4(u[0], u[1], u[2], u[3]);
        }
      }
    }
    if (!last_block) {
      w.best_u[j] = bu;
      w.best_l[j] = bl;
    } else {
      float out[4] = {0.0f, 0.0f, 0.0f, 0.0f}, lam = 0.0f;
      if (cn > 0.0f) {
        out[0] = bu.x; out[1] = bu.y; out[2] = bu.z; out[3] = bu.w;
        const float sg = out[0] != 0.0f ? out[0] : (out[1] != 0.0f ? out[1] : (out[2] != 0.0f ? out[2] : out[3]));
        if (sg < 0.0f) {
#pragma unroll
          for (int d = 0; d < 4; ++d) out[d] = -out[d];
        }
        lam = bl * cn;
        n_oriented += merge ? 0 : 1;
      }
      const size_t o = rv.o;
      if (!merge || lam > rv.lam[o]) {
        if (rv.lam) rv.lam[o] = lam;
        if (rv.dir) {
#pragma unroll
          for (int d = 0; d < 4; ++d) rv.dir[4 * o + d] = out[d];
        }
      }
    }
  }
  if (a.counters) {
    count_add4(a.counters + 1, n_newton);
    count_add4(a.counters + 2, n_oriented);
  }
}

// ---------------------------------------------------------------------------
// learned start
// ---------------------------------------------------------------------------

constexpr int kLearnedWaves4 = 4;
constexpr unsigned kLearnedGroups4 = 1024;
constexpr float kCertify4 = 1e-2f;       // Newton step length that certifies
constexpr float kCertifyGrad4 = 3e-5f;   // |g - lambda u| that certifies with ...
constexpr float kCertifyCurv4 = 1e-3f;   // ... no tangent-Hessian eigenvalue above this
constexpr int kCertifySteps4 = 4;
constexpr int kHalvings4 = 2;

// Certification of u as near a local maximum (the learned start's acceptance
// test): |t| <= kCertifyGrad4 with every eigenvalue of A at most kCertifyCurv4
// (m + kCertifyCurv4 I positive definite, m = -A), or m positive definite and
// the Newton step at most kCertify4 long; otherwise a guarded Newton step
// (halved while lambda falls by more than 1e-6) and the test again, at most
// kCertifySteps4 times.  u, g, lambda follow the steps taken.
template <int N>
__device__ __forceinline__ bool certify4(const float (&c)[ncomp4(N)], float (&u)[4], float (&g)[4],
                                         float& lam, unsigned long long& taken) {
  for (int k = 0; k <= kCertifySteps4; ++k) {
    float E[3][4], m[3][3], t[3];
    ++taken;
    tangent_model4<N>(c, u, g, lam, E, m, t);
    float ms[3][3], tmp[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) ms[i][j] = m[i][j] + (i == j ? kCertifyCurv4 : 0.0f);
    if (t[0] * t[0] + t[1] * t[1] + t[2] * t[2] <= kCertifyGrad4 * kCertifyGrad4 &&
        solve_pd3(ms, t, tmp))
      return true;
    float eta[3];
    if (!solve_pd3(m, t, eta)) return false;
    float dv[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) dv[d] = eta[0] * E[0][d] + eta[1] * E[1][d] + eta[2] * E[2][d];
    if (dot4(dv, dv) <= kCertify4 * kCertify4) return true;
    if (k == kCertifySteps4) return false;
    float tt = 1.0f, v[4], q[4], lam_v = 0.0f;
    bool up = false;
    for (int h = 0; h <= kHalvings4; ++h) {
#pragma unroll
      for (int d = 0; d < 4; ++d) v[d] = u[d] + tt * dv[d];
      const float rv = 1.0f / sqrtf(dot4(v, v));
#pragma unroll
      for (int d = 0; d < 4; ++d) v[d] *= rv;
      contract4<N>(c, v, q);
      lam_v = dot4(q, v);
      if (lam_v >= lam - 1e-6f) {
        up = true;
        break;
      }
      tt *= 0.5f;
    }
    if (!up) return false;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      u[d] = v[d];
      g[d] = q[d];
    }
    lam = lam_v;
  }
  return false;
}

// Learned start: persistent workgroups of kLearnedWaves4 wavefronts, each
// taking 64 voxels at a time (voxel = lane).  Per voxel: the score; the
// network's q0 = y / |y| (start 0 where y = 0, which also forces the
// fallback); SS-HOPM from q0 with the unfolding shift until |delta lambda| <=
// tol or max_iter updates; the Newton polish; the certification; the screen
// (a fixed start s with <C, s^n> above lambda).  The answer is written, and a
// voxel that did not converge, is not certified, has lambda / ||C||_F below
// kappa or is beaten by a fixed start is appended to the fallback list.
template <int N, int KT>
__global__ __launch_bounds__(64 * kLearnedWaves4) void k_learned4(ExtractArgs a) {
  constexpr int K = ncomp4(N);
  constexpr Sym4<N> sy{};
  using Lay = MlpLayout<KT>;
  constexpr int kin = Lay::kin;
  __shared__ float st[64 * 4];
  __shared__ float mono[64 * K];
  __shared__ __align__(16) unsigned char pk[Lay::packed];
  __shared__ unsigned short xs_all[kLearnedWaves4][64 * kin];
  static_assert(Lay::packed % 16 == 0, "packed network copied in 16-byte pieces");
  for (int i = threadIdx.x; i < a.n_starts * 4; i += blockDim.x) st[i] = a.starts[i];
  for (int i = threadIdx.x; i < Lay::packed / 16; i += blockDim.x)
    reinterpret_cast<uint4*>(pk)[i] = reinterpret_cast<const uint4*>(a.mlp)[i];
  __syncthreads();
  // mono[s K + k] = mu_k s^alpha_k for the unit fixed starts
  for (int i = threadIdx.x; i < a.n_starts * K; i += blockDim.x) {
    const int s = i / K, k = i % K;
    const float* sv = &st[4 * s];
    const float rn = 1.0f / sqrtf(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2] + sv[3] * sv[3]);
    float m = sy.mu[k];
    for (int d = 0; d < 4; ++d)
      for (int p = 0; p < sy.e[k][d]; ++p) m *= sv[d] * rn;
    mono[i] = m;
  }
  __syncthreads();
  const Ws4 w = ws4_layout(a.ws, a.plane);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned short* xs = xs_all[wave];
  const MlpLdsT<KT> net{pk, lane};
  const size_t n_groups = (a.plane + 63) / 64;
  const size_t gstride = (size_t)gridDim.x * kLearnedWaves4;
  unsigned long long n_steps = 0, n_newton = 0, n_oriented = 0, n_shift = 0;
  for (size_t gi = (size_t)blockIdx.x * kLearnedWaves4 + wave; gi < n_groups; gi += gstride) {
    const size_t v0 = gi * 64 + lane;
    const bool active = v0 < a.plane;
    const size_t v = active ? v0 : a.plane - 1;
    float c[K];
    const Vox4 rv = vox4(a, v);
    const float cn = load4_at<N>(a, rv, c);
    const size_t o = rv.o;
    if ((a.mode & 1) && active && rv.score) rv.score[o] = cn;
    const float inv = cn > 0.0f ? 1.0f / cn : 0.0f;
    for (int k = 0; k < kin; ++k) xs[lane * kin + k] = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) xs[lane * kin + k] = bf16_bits(sqrtf(sy.mu[k]) * c[k] * inv);
    wave_lds_sync();
    float y[4];
    mlp_forward_t<KT>(xs, net, lane, y);
    wave_lds_sync();   // xs is rewritten by the next group
    const float ny = sqrtf(y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3]);
    const bool forced = !(ny > 0.0f);
    float u[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) u[d] = forced ? st[d] : y[d];
    const float ru = 1.0f / sqrtf(dot4(u, u));
#pragma unroll
    for (int d = 0; d < 4; ++d) u[d] *= ru;
    if (!active) continue;
    if (!(cn > 0.0f)) {
      if (rv.lam) rv.lam[o] = 0.0f;
      if (rv.dir) {
#pragma unroll
        for (int d = 0; d < 4; ++d) rv.dir[4 * o + d] = 0.0f;
      }
      continue;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] *= inv;
    const float alpha = fmaxf(0.0f, -unfolding_lambda_min4<N>(c));
    ++n_shift;
    float g[4];
    contract4<N>(c, u, g);
    float lam = dot4(g, u);
    bool conv = false;
    for (int it = 0; it < a.max_iter; ++it) {
      float vv[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) vv[d] = fmaf(alpha, u[d], g[d]);
      const float rn = rsqrtf(dot4(vv, vv));
#pragma unroll
      for (int d = 0; d < 4; ++d) u[d] = vv[d] * rn;
      contract4<N>(c, u, g);
      const float ln = dot4(g, u);
      ++n_steps;
      conv = fabsf(ln - lam) <= a.tol;
      lam = ln;
      if (conv) break;
    }
    n_newton += newton_polish4<N>(c, u, g, lam, a.newton);
    const bool certified = certify4<N>(c, u, g, lam, n_newton);
    bool beaten = false;
    if (a.screen) {
      for (int s = 0; s < a.n_starts; ++s) {
        float f = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) f = fmaf(mono[s * K + k], c[k], f);
        beaten = beaten || f > lam;
      }
    }
    ++n_oriented;
    const bool fallback = forced || !conv || !certified || !(lam >= a.kappa) || beaten;
    const float sg = u[0] != 0.0f ? u[0] : (u[1] != 0.0f ? u[1] : (u[2] != 0.0f ? u[2] : u[3]));
    if (sg < 0.0f) {
#pragma unroll
      for (int d = 0; d < 4; ++d) u[d] = -u[d];
    }
    if (rv.lam) rv.lam[o] = lam * cn;
    if (rv.dir) {
#pragma unroll
      for (int d = 0; d < 4; ++d) rv.dir[4 * o + d] = u[d];
    }
    if (fallback) {
      const unsigned long long slot = atomicAdd(&w.ctr[kListCount4], 1ull);
      w.list[slot] = (unsigned)v;
      if (a.fb_total) atomicAdd(a.fb_total, 1);
    }
  }
  if (a.counters) {
    count_add4(a.counters + 0, n_steps);
    count_add4(a.counters + 1, n_newton);
    count_add4(a.counters + 2, n_oriented);
    count_add4(a.counters + 3, n_shift);
  }
}

// The pooled multistart over the items (all box voxels, or a listed subset
// whose answers are merged into the maps).
template <int N>
void launch_multistart4(const ExtractArgs& a, const Items4& it, int merge, hipStream_t s) {
  const Ws4 w = ws4_layout(a.ws, a.plane);
  const unsigned nb = (unsigned)((a.plane + 255) / 256);
  const unsigned ib = nb < kItemGroups4 ? nb : kItemGroups4;
  hipLaunchKernelGGL(k_prepare4<N>, dim3(ib), dim3(256), 0, s, a, it);
  const int n_blocks = (a.n_starts + kStartBlock4 - 1) / kStartBlock4;
  for (int b = 0; b < n_blocks; ++b) {
    const int nsb = (a.n_starts - b * kStartBlock4) < kStartBlock4 ? (a.n_starts - b * kStartBlock4)
                                                                   : kStartBlock4;
    hipLaunchKernelGGL(k_runs4<N>, dim3(kPoolGroups4), dim3(64), 0, s, a, it, nsb, b * kStartBlock4,
                       w.ctr + b);
    hipLaunchKernelGGL(k_reduce4<N>, dim3(ib), dim3(256), 0, s, a, it, nsb, b == 0 ? 1 : 0,
                       b == n_blocks - 1 ? 1 : 0, merge);
  }
}

template <int N>
int launch4_n(const ExtractArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)((a.plane + 255) / 256);
  if constexpr (N >= 2 && N <= 6) {
    if (a.mode & 2) {
      const Ws4 w = ws4_layout(a.ws, a.plane);
      fill_zero(w.ctr, 256, s);
      if (a.mode & 4) {
        if constexpr (ncomp4(N) <= kMlpInMax) {
          constexpr int KT = mlp_tiles(ncomp4(N));
          const unsigned groups = (unsigned)((a.plane + 64 * kLearnedWaves4 - 1) / (64 * kLearnedWaves4));
          hipLaunchKernelGGL((k_learned4<N, KT>), dim3(groups < kLearnedGroups4 ? groups : kLearnedGroups4),
                             dim3(64 * kLearnedWaves4), 0, s, a);
          launch_multistart4<N>(a, Items4{w.list, w.ctr + kListCount4}, 1, s);
        } else {
          set_error("ttm_extract: learned start (d'=4) takes at most %d components", kMlpInMax);
          return -4;
        }
      } else {
        launch_multistart4<N>(a, Items4{nullptr, nullptr}, 0, s);
      }
      hipError_t e = hipGetLastError();
      return e == hipSuccess ? 0 : hip_status(e, "extract (d'=4) launch");
    }
  }
  hipLaunchKernelGGL(k_score4<N>, dim3(nb), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : hip_status(e, "extract (d'=4) launch");
}

}  // namespace

size_t extract_workspace4(size_t plane) {
  return 256 + al256_4(plane * 4) + al256_4(plane * 16) + al256_4(plane * 4) +
         al256_4((size_t)kStartBlock4 * plane * 16) + al256_4((size_t)kStartBlock4 * plane * 4) +
         plane * 4;
}

int launch_extract4(int degree, const ExtractArgs& a, hipStream_t s) {
  switch (degree) {
    case 0: return launch4_n<0>(a, s);
    case 2: return launch4_n<2>(a, s);
    case 4: return launch4_n<4>(a, s);
    case 6: return launch4_n<6>(a, s);
    default: set_error("ttm_extract: degree %d not built for d'=4", degree); return -4;
  }
}

}  // namespace ttm
