// extract.hip -- per-voxel score and orientation from the tensor field (gfx950).
//
// Score: c = ||C||_F = sqrt(sum_a mu_a C_a^2) (Sec. 3.2).
// Orientation (Sec. 3.1): SS-HOPM on C / c with the shift
// alpha = max(0, -lambda_min(U)), U the square matrix unfolding.  U is zero
// off the symmetric (n/2)-tensors, where it equals
// B[b, g] = sqrt(mu_b mu_g) C_{b+g}, so lambda_min(U) = min(0, lambda_min(B));
// the kernels bound lambda_min(B) from below (Gershgorin interval narrowed by
// bisection with Cholesky tests), so their shift is never below the rule's value.
//
// SS-HOPM runs take very different numbers of steps (a handful near a sharp
// maximum, hundreds on a flat one), and a wavefront advances at the pace of its
// slowest lane.  The kernels therefore do not tie a lane to a voxel:
//
//   multistart (all voxels, or the voxels the learned start hands back):
//     k_prepare  one lane per voxel: score and the shift
//     k_runs     persistent wavefronts drain a global queue of (voxel, start)
//                runs; a lane that finishes a run takes the next one as soon
//                as kRefill lanes of its wavefront wait, so lanes stay busy;
//                each run's (u, lambda) goes to its own slot
//     k_reduce   one lane per voxel: every run's answer takes the Newton
//                polish, the largest polished lambda wins (first on ties)
//   learned start:
//     k_learned  persistent wavefronts, 64 voxels at a time: the BF16 MLP on
//                the matrix cores gives each voxel's start u0, then each lane
//                takes at most kNewtonFirst Riemannian Newton steps (halved
//                when lambda falls; no shift needed); converged voxels are
//                screened and written.  The others run SS-HOPM from u0 in
//                k_runs (queue of saved iterates, shift from k_prepare), then
//                k_learned_post polishes, screens and writes them.  Voxels
//                that fail the checks go to the multistart path above, whose
//                answer replaces the learned one when it is larger.
//     k_mlp_start  the network alone, for the start directions only
#include "extract_items.hpp"
#include "internal.hpp"
#include "mlp_core.hpp"
#include "sym_tables.hpp"

namespace ttm {

namespace {

constexpr int kNewtonFirst = 5;   // Newton steps from the learned start inside k_learned
constexpr int kRefill = 8;        // a pooled wavefront refills once this many lanes wait
constexpr int kPoolGroups = 4096; // persistent pooled grid (one wavefront per group)
constexpr int kStartBlock = 16;   // starts whose run results are held at once

// Workspace layout (one 256-byte aligned array each, `plane` entries):
// header (counters), fallback list, continuation list, continuation state
// (u, lambda), continuation step count, shift, continuation flags, carried best
// (u, lambda), run results [kStartBlock][plane] (u, lambda).
enum HeaderSlot {
  kHdrFallbacks = 0,   // fallback list length
  kHdrContinue = 1,    // continuation list length
  kHdrPoolCont = 2,    // k_runs work counters (64-bit, 8-byte aligned)
  kHdrPoolDense = 4,   // + 2 per start block
  kHdrPoolFb = 20,     // + 2 per start block
  kHdrWords = 64
};

struct Ws {
  unsigned* hdr;
  unsigned* fb_list;
  unsigned* cont_list;
  float4* cont_state;   // per box voxel: learned start u0 and its lambda
  int* cont_it;         // per box voxel: 1 << 30 when the network gave no direction
  float* alpha;
  unsigned char* conv;
  float4* best;      // carried multistart best; learned start u0 before that
  unsigned char* status;  // per box voxel: 0 answered, 1 continue with SS-HOPM, 2 fall back
  unsigned* blocksum;     // per compaction block: count, then offset
  float4* res;
  float4* stage;   // per box voxel handed on by the learned start: C / ||C||_F, then ||C||_F
};

constexpr int kCompactBlock = 4096;   // voxels per compaction workgroup (256 threads x 16)

__host__ __device__ inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

__host__ __device__ inline Ws ws_layout(void* base, size_t plane) {
  char* p = static_cast<char*>(base);
  Ws w;
  w.hdr = reinterpret_cast<unsigned*>(p);
  p += 256;
  w.fb_list = reinterpret_cast<unsigned*>(p);
  p += al256(plane * 4);
  w.cont_list = reinterpret_cast<unsigned*>(p);
  p += al256(plane * 4);
  w.cont_state = reinterpret_cast<float4*>(p);
  p += al256(plane * 16);
  w.cont_it = reinterpret_cast<int*>(p);
  p += al256(plane * 4);
  w.alpha = reinterpret_cast<float*>(p);
  p += al256(plane * 4);
  w.conv = reinterpret_cast<unsigned char*>(p);
  p += al256(plane);
  w.best = reinterpret_cast<float4*>(p);
  p += al256(plane * 16);
  w.status = reinterpret_cast<unsigned char*>(p);
  p += al256(plane);
  w.blocksum = reinterpret_cast<unsigned*>(p);
  p += al256(((plane + kCompactBlock - 1) / kCompactBlock) * 4);
  w.res = reinterpret_cast<float4*>(p);
  p += (size_t)kStartBlock * plane * 16;
  w.stage = reinterpret_cast<float4*>(p);
  return w;
}

// float4 slots of one staged voxel: the K normalised components, then ||C||_F.
__host__ __device__ constexpr int stage_slots(int K) { return (K + 1 + 3) / 4; }

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

// Tangent model of max <C, u^n> on the unit sphere at u with (g, lambda) =
// (C u^{n-1}, <C, u^n>): tangent basis e1 = a x u/|a x u| (a = axis of the
// smallest |u_i|), e2 = u x e1 (e = {e1, e2}); the tangent Hessian
// A = (n-1) E^T H E - lambda I (H = C u^{n-2}) and the tangent gradient t = E^T g.
template <int N>
__device__ __forceinline__ void tangent_model(const float (&c)[ncomp3(N)], float ux, float uy,
                                              float uz, float g0, float g1, float g2, float lam,
                                              float (&e)[6], float& a00, float& a01, float& a11,
                                              float& t0, float& t1) {
  const float fx = fabsf(ux), fy = fabsf(uy), fz = fabsf(uz);
  float e1x, e1y, e1z;
  if (fx <= fy && fx <= fz) {        // a = e_x: a x u = (0, -uz, uy)
    e1x = 0.0f; e1y = -uz; e1z = uy;
  } else if (fy <= fz) {             // a = e_y: (uz, 0, -ux)
    e1x = uz; e1y = 0.0f; e1z = -ux;
  } else {                           // a = e_z: (-uy, ux, 0)
    e1x = -uy; e1y = ux; e1z = 0.0f;
  }
  const float r1 = rsqrtf(e1x * e1x + e1y * e1y + e1z * e1z);
  e1x *= r1; e1y *= r1; e1z *= r1;
  const float e2x = uy * e1z - uz * e1y, e2y = uz * e1x - ux * e1z, e2z = ux * e1y - uy * e1x;
  float h[6];
  contract2<N>(c, ux, uy, uz, h);
  const float hx1 = h[0] * e1x + h[1] * e1y + h[2] * e1z;
  const float hy1 = h[1] * e1x + h[3] * e1y + h[4] * e1z;
  const float hz1 = h[2] * e1x + h[4] * e1y + h[5] * e1z;
  const float hx2 = h[0] * e2x + h[1] * e2y + h[2] * e2z;
  const float hy2 = h[1] * e2x + h[3] * e2y + h[4] * e2z;
  const float hz2 = h[2] * e2x + h[4] * e2y + h[5] * e2z;
  constexpr float nm1 = (float)(N - 1);
  a00 = nm1 * (e1x * hx1 + e1y * hy1 + e1z * hz1) - lam;
  a01 = nm1 * (e1x * hx2 + e1y * hy2 + e1z * hz2);
  a11 = nm1 * (e2x * hx2 + e2y * hy2 + e2z * hz2) - lam;
  t0 = e1x * g0 + e1y * g1 + e1z * g2;
  t1 = e2x * g0 + e2y * g1 + e2z * g2;
  e[0] = e1x; e[1] = e1y; e[2] = e1z; e[3] = e2x; e[4] = e2y; e[5] = e2z;
}

// Newton direction of a tangent model: d = E eta with eta = -A^{-1} t, where A
// must be negative definite (false otherwise: no step).
__device__ __forceinline__ bool tangent_step(const float (&e)[6], float a00, float a01, float a11,
                                             float t0, float t1, float& dx, float& dy, float& dz) {
  const float det = a00 * a11 - a01 * a01;
  if (!(det > 0.0f && a00 + a11 < 0.0f)) return false;
  const float inv = 1.0f / det;
  const float eta0 = -(a11 * t0 - a01 * t1) * inv;
  const float eta1 = -(a00 * t1 - a01 * t0) * inv;
  dx = eta0 * e[0] + eta1 * e[3];
  dy = eta0 * e[1] + eta1 * e[4];
  dz = eta0 * e[2] + eta1 * e[5];
  return true;
}

// Riemannian Newton direction for max <C, u^n> on the unit sphere at u (false
// where the tangent Hessian is not negative definite: no step).
template <int N>
__device__ __forceinline__ bool newton_dir(const float (&c)[ncomp3(N)], float ux, float uy,
                                           float uz, float g0, float g1, float g2, float lam,
                                           float& dx, float& dy, float& dz) {
  float e[6], a00, a01, a11, t0, t1;
  tangent_model<N>(c, ux, uy, uz, g0, g1, g2, lam, e, a00, a01, a11, t0, t1);
  return tangent_step(e, a00, a01, a11, t0, t1, dx, dy, dz);
}

// v = (u + t d) / |u + t d| and (q, lambda_v) = (C v^{n-1}, <C, v^n>).
template <int N>
__device__ __forceinline__ void newton_move(const float (&c)[ncomp3(N)], float ux, float uy,
                                            float uz, float dx, float dy, float dz, float t,
                                            float& vx, float& vy, float& vz, float& q0, float& q1,
                                            float& q2, float& lam_v) {
  vx = ux + t * dx;
  vy = uy + t * dy;
  vz = uz + t * dz;
  const float rv = rsqrtf(vx * vx + vy * vy + vz * vz);
  vx *= rv; vy *= rv; vz *= rv;
  contract<N>(c, vx, vy, vz, q0, q1, q2);
  lam_v = q0 * vx + q1 * vy + q2 * vz;
}

// One full Newton step (false if the tangent Hessian is not negative definite).
template <int N>
__device__ __forceinline__ bool newton_step(const float (&c)[ncomp3(N)], float ux, float uy,
                                            float uz, float g0, float g1, float g2, float lam,
                                            float& vx, float& vy, float& vz, float& q0, float& q1,
                                            float& q2, float& lam_v) {
  float dx, dy, dz;
  if (!newton_dir<N>(c, ux, uy, uz, g0, g1, g2, lam, dx, dy, dz)) return false;
  newton_move<N>(c, ux, uy, uz, dx, dy, dz, 1.0f, vx, vy, vz, q0, q1, q2, lam_v);
  return true;
}

// Up to `steps` Newton steps from a converged SS-HOPM point; a step is kept
// unless lambda drops by more than 1e-7.  (g, lambda) must hold C u^{n-1} and
// <C, u^n> at u on entry and are kept current.  Returns the steps computed.
template <int N>
__device__ __forceinline__ int newton_polish(const float (&c)[ncomp3(N)], float& ux, float& uy,
                                             float& uz, float& g0, float& g1, float& g2,
                                             float& lam, int steps) {
  int taken = 0;
  for (int s = 0; s < steps; ++s) {
    float vx, vy, vz, q0, q1, q2, lam_new;
    if (!newton_step<N>(c, ux, uy, uz, g0, g1, g2, lam, vx, vy, vz, q0, q1, q2, lam_new)) break;
    ++taken;
    if (lam_new < lam - 1e-7f) break;
    ux = vx; uy = vy; uz = vz;
    g0 = q0; g1 = q1; g2 = q2;
    lam = lam_new;
  }
  return taken;
}

// Newton iteration from a start: up to `steps` steps.  A step whose lambda
// falls by more than 1e-6 (lambda <= 1 for C / ||C||_F; a few FP32 ulps, so
// rounding near convergence is not taken for a fall) is halved, at most
// kHalvings times; the search stops without convergence when the tangent
// Hessian is not negative definite or the halved steps still fall.  Converged
// (ok) after a full step that changes lambda by at most tol.  Returns the
// Newton directions computed.
constexpr int kHalvings = 2;

template <int N>
__device__ __forceinline__ int newton_ascent(const float (&c)[ncomp3(N)], float& ux, float& uy,
                                             float& uz, float& g0, float& g1, float& g2,
                                             float& lam, int steps, float tol, bool& ok) {
  int taken = 0;
  ok = false;
  for (int s = 0; s < steps; ++s) {
    float dx, dy, dz;
    if (!newton_dir<N>(c, ux, uy, uz, g0, g1, g2, lam, dx, dy, dz)) break;
    ++taken;
    float vx, vy, vz, q0, q1, q2, lam_new;
    float t = 1.0f;
    bool up = false;
    for (int h = 0; h <= kHalvings; ++h) {
      newton_move<N>(c, ux, uy, uz, dx, dy, dz, t, vx, vy, vz, q0, q1, q2, lam_new);
      if (lam_new >= lam - 1e-6f) {
        up = true;
        break;
      }
      t *= 0.5f;
    }
    if (!up) break;
    const bool done = t == 1.0f && fabsf(lam_new - lam) <= tol;
    ux = vx; uy = vy; uz = vz;
    g0 = q0; g1 = q1; g2 = q2;
    lam = lam_new;
    if (done) {
      ok = true;
      break;
    }
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
// |b| = |g| = n/2.  The Gershgorin discs give lo <= lambda_min and the
// smallest diagonal entry hi >= lambda_min; STEPS bisection steps then keep
// lo where B - lo I passes a Cholesky factorisation (positive definite, so
// lambda_min > lo).  The result lo - kShiftMargin stays below lambda_min under
// FP32 rounding of the 10 x 10 factorisation (backward error a few 1e-6 for
// entries of C / ||C||_F), so the shift -lo is never smaller than the
// unfolding rule's, and exceeds it by at most (hi - lo) / 2^STEPS + margin.
constexpr float kShiftMargin = 1e-5f;

template <int N>
__device__ __forceinline__ float unfolding_entry(const float (&c)[ncomp3(N)], int p, int q) {
  constexpr int H = N / 2;
  constexpr Sym3<H> hs{};
  return sqrtf(hs.mu[p] * hs.mu[q]) * c[comp_index3(N, hs.ax[p] + hs.ax[q], hs.ay[p] + hs.ay[q])];
}

template <int N, int STEPS>
__device__ __forceinline__ float unfolding_lambda_min(const float (&c)[ncomp3(N)]) {
  constexpr int M = ncomp3(N / 2);
  float lo = INFINITY, hi = INFINITY;
#pragma unroll
  for (int p = 0; p < M; ++p) {
    float rad = 0.0f;
#pragma unroll
    for (int q = 0; q < M; ++q)
      if (q != p) rad += fabsf(unfolding_entry<N>(c, p, q));
    const float d = unfolding_entry<N>(c, p, p);
    lo = fminf(lo, d - rad);
    hi = fminf(hi, d);
  }
  for (int step = 0; step < STEPS; ++step) {
    const float mid = 0.5f * (lo + hi);
    // Cholesky of W = B - mid I (upper triangle R, packed); pd stays true while
    // every pivot is positive
    float R[M * (M + 1) / 2];
    bool pd = true;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      float d = unfolding_entry<N>(c, j, j) - mid;
#pragma unroll
      for (int k = 0; k < j; ++k) d = fmaf(-R[tri(M, k, j)], R[tri(M, k, j)], d);
      pd = pd && d > 0.0f;
      const float r = pd ? rsqrtf(d) : 0.0f;
      R[tri(M, j, j)] = d * r;
#pragma unroll
      for (int i = j + 1; i < M; ++i) {
        float e = unfolding_entry<N>(c, j, i);
#pragma unroll
        for (int k = 0; k < j; ++k) e = fmaf(-R[tri(M, k, j)], R[tri(M, k, i)], e);
        R[tri(M, j, i)] = e * r;
      }
    }
    if (pd) lo = mid; else hi = mid;
  }
  return lo - kShiftMargin;
}

// Bisection steps of the shift bound for the multistart search and for the
// learned start.
constexpr int kShiftSteps = 12;

__device__ __forceinline__ void canonical(float& x, float& y, float& z) {
  // u and -u are the same answer: make the last non-zero coordinate positive
  const float sg = (z != 0.0f) ? z : ((y != 0.0f) ? y : x);
  if (sg < 0.0f) {
    x = -x; y = -y; z = -z;
  }
}

using Vox = VoxelRef;
__device__ __forceinline__ Vox vox(const ExtractArgs& a, size_t v) { return voxel_ref(a, v); }

// The K components of a voxel, as stored (no arithmetic, so a lane can
// issue them for its next voxel and keep working on the current one).
template <int N>
__device__ __forceinline__ void load_raw_at(const ExtractArgs& a, const Vox& r, float (&c)[ncomp3(N)]) {
  constexpr int K = ncomp3(N);
  if (a.in_dtype == 1) {
    const unsigned short* p = reinterpret_cast<const unsigned short*>(r.C);
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = bf16_to_f32(p[k * r.stride + r.lv]);
  } else {
    const float* p = reinterpret_cast<const float*>(r.C);
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = p[k * r.stride + r.lv];
  }
}

template <int N>
__device__ __forceinline__ void load_raw(const ExtractArgs& a, size_t v, float (&c)[ncomp3(N)]) {
  load_raw_at<N>(a, vox(a, v), c);
}

// Load the K components of a voxel, return ||C||_F.
template <int N>
__device__ __forceinline__ float load_tensor_at(const ExtractArgs& a, const Vox& r,
                                                float (&c)[ncomp3(N)]) {
  constexpr int K = ncomp3(N);
  constexpr Sym3<N> sy{};
  load_raw_at<N>(a, r, c);
  float f2 = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) f2 = fmaf(sy.mu[k] * c[k], c[k], f2);
  return sqrtf(f2);
}

template <int N>
__device__ __forceinline__ float load_tensor(const ExtractArgs& a, size_t v, float (&c)[ncomp3(N)]) {
  return load_tensor_at<N>(a, vox(a, v), c);
}

// ||C||_F of loaded components (the same sum load_tensor forms).
template <int N>
__device__ __forceinline__ float frob(const float (&c)[ncomp3(N)]) {
  constexpr Sym3<N> sy{};
  float f2 = 0.0f;
#pragma unroll
  for (int k = 0; k < ncomp3(N); ++k) f2 = fmaf(sy.mu[k] * c[k], c[k], f2);
  return sqrtf(f2);
}

template <int N>
__device__ __forceinline__ void scale(float (&c)[ncomp3(N)], float inv) {
#pragma unroll
  for (int k = 0; k < ncomp3(N); ++k) c[k] *= inv;
}

__device__ __forceinline__ void write_answer(const Vox& r, float lam, float x, float y, float z) {
  if (r.lam) r.lam[r.o] = lam;
  if (r.dir) {
    r.dir[3 * r.o + 0] = x;
    r.dir[3 * r.o + 1] = y;
    r.dir[3 * r.o + 2] = z;
  }
}

// <C, s^n> for every fixed start s as a dot product with the start's weighted
// monomials mono[s][k] = mu_k s^alpha_k (s normalised), built once per block.
template <int N>
__device__ __forceinline__ void build_monomials(const float* st, int n_starts, float* mono) {
  constexpr int K = ncomp3(N);
  constexpr Sym3<N> sy{};
  for (int i = threadIdx.x; i < n_starts * K; i += blockDim.x) {
    const int s = i / K, k = i % K;
    const float sx = st[3 * s], sy_ = st[3 * s + 1], sz = st[3 * s + 2];
    const float r = 1.0f / sqrtf(sx * sx + sy_ * sy_ + sz * sz);
    float m = sy.mu[k];
    for (int e = 0; e < sy.ax[k]; ++e) m *= sx * r;
    for (int e = 0; e < sy.ay[k]; ++e) m *= sy_ * r;
    for (int e = 0; e < sy.az[k]; ++e) m *= sz * r;
    mono[i] = m;
  }
}

// ---------------------------------------------------------------------------
// score only
// ---------------------------------------------------------------------------

template <int N>
__global__ __launch_bounds__(256) void k_score(ExtractArgs a) {
  const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= a.plane) return;
  float c[ncomp3(N)];
  const Vox r = vox(a, v);
  const float cn = load_tensor_at<N>(a, r, c);
  if (r.score) r.score[r.o] = cn;
}

// ---------------------------------------------------------------------------
// multistart: shift per voxel, pooled runs, reduction
// ---------------------------------------------------------------------------

// Work list: `list` (box voxel per item, length *count) or all box voxels.
// Items of a run: the voxels of a device-side list (or every box voxel).
// stage: where the learned start left the listed voxels' normalised tensors
// (one contiguous piece per voxel), else they are read from the K planes.
struct Items {
  const unsigned* list;
  const unsigned* count;
  const float4* stage;
  __device__ __forceinline__ unsigned n(const ExtractArgs& a) const {
    return list ? *count : (unsigned)a.plane;
  }
  __device__ __forceinline__ size_t voxel(unsigned j) const { return list ? list[j] : j; }
};

// Normalised tensor of box voxel v staged by the learned start; returns ||C||_F.
template <int N>
__device__ __forceinline__ float load_staged(const float4* stage, size_t v, float (&c)[ncomp3(N)]) {
  constexpr int K = ncomp3(N), SQ = stage_slots(K);
  float f[4 * SQ];
  const float4* p = stage + v * SQ;
#pragma unroll
  for (int i = 0; i < SQ; ++i) {
    const float4 q = p[i];
    f[4 * i] = q.x; f[4 * i + 1] = q.y; f[4 * i + 2] = q.z; f[4 * i + 3] = q.w;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) c[k] = f[k];
  return f[K];
}

template <int N>
__device__ __forceinline__ void store_staged(float4* stage, size_t v, const float (&c)[ncomp3(N)],
                                             float cn) {
  constexpr int K = ncomp3(N), SQ = stage_slots(K);
  float f[4 * SQ];
#pragma unroll
  for (int k = 0; k < 4 * SQ; ++k) f[k] = k < K ? c[k] : (k == K ? cn : 0.0f);
  float4* p = stage + v * SQ;
#pragma unroll
  for (int i = 0; i < SQ; ++i) p[i] = make_float4(f[4 * i], f[4 * i + 1], f[4 * i + 2], f[4 * i + 3]);
}

// Shift (and optionally the score) per item.  `add_total`: add the item
// count to the caller's fallback counter.
template <int N>
__global__ __launch_bounds__(256) void k_prepare(ExtractArgs a, Items it, int write_score,
                                                 int add_total) {
  const Ws w = ws_layout(a.ws, a.plane);
  const unsigned n = it.n(a);
  if (add_total && a.fb_total && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.fb_total, (int)n);
  unsigned long long n_shift = 0;
  for (unsigned j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const size_t v = it.voxel(j);
    float c[ncomp3(N)];
    const float cn = it.stage ? load_staged<N>(it.stage, v, c) : load_tensor<N>(a, v, c);
    if (write_score) {
      const Vox r = vox(a, v);
      if (r.score) r.score[r.o] = cn;
    }
    float alpha = 0.0f;
    if (cn > 0.0f) {
      if (!it.stage) scale<N>(c, 1.0f / cn);
      alpha = fmaxf(0.0f, -unfolding_lambda_min<N, kShiftSteps>(c));
      n_shift += 1;
    }
    w.alpha[j] = alpha;
  }
  if (a.counters) count_add(a.counters + 3, n_shift);
}

// Persistent pooled SS-HOPM runs.  Run q of a chunk is item q / R, start
// s0 + q % R (multistart) or the item's saved iterate (cont).  A wavefront
// takes up to 64 items at a time from a global counter and stages their normalised
// tensors (and shifts, saved iterates) in LDS; lanes whose run has ended take
// the chunk's next runs as soon as kRefill of them wait.  Each run ends at
// |delta lambda| <= tol or max_iter updates; its (u, lambda) is written to
// res[(q % R) * plane + item] (and, for cont, conv[item]).
struct RunArgs {
  Items items;
  int per_item;   // R
  int s0;         // first start of this block
  unsigned long long* ctr;
};

template <int N, bool CONT>
__global__ __launch_bounds__(64) void k_runs(ExtractArgs a, RunArgs r) {
  constexpr int K = ncomp3(N);
  __shared__ float st[64 * 3];
  __shared__ float cs[K][64];     // chunk tensors, [component][item]
  __shared__ float ca[64];        // shift per item
  __shared__ float cz[64];        // ||C||_F per item (0: nothing to run)
  __shared__ float4 cu[CONT ? 64 : 1];
  __shared__ int ci[CONT ? 64 : 1];
  const int lane = threadIdx.x;
  for (int i = lane; i < a.n_starts * 3; i += 64) st[i] = a.starts[i];
  __syncthreads();
  const Ws w = ws_layout(a.ws, a.plane);
  const unsigned n_items = r.items.n(a);
  const int R = r.per_item;
  // items per chunk: up to 64, fewer when the list is short, so that every
  // wavefront of the grid gets several chunks
  const unsigned per_wave = (n_items + 4 * gridDim.x - 1) / (4 * gridDim.x);
  const unsigned chunk = per_wave < 1 ? 1 : (per_wave > 64 ? 64 : per_wave);
  // chunk state (uniform across the wavefront)
  unsigned chunk_base = 0;
  int chunk_runs = 0, next_q = 0;
  bool exhausted = n_items == 0;
  // lane state
  float c[K];
#pragma unroll
  for (int k = 0; k < K; ++k) c[k] = 0.0f;
  float alpha = 0.0f, ux = 0.0f, uy = 0.0f, uz = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, lam = 0.0f;
  int iters = 0, s = 0;
  unsigned j = 0;
  bool first = false, busy = false;
  unsigned long long n_steps = 0, n_runs = 0;
  while (true) {
    unsigned long long waiting = __ballot(!busy);
    int n_wait = __popcll(waiting);
    if (n_wait == 64 && exhausted && next_q == chunk_runs) break;
    if (n_wait >= kRefill || n_wait == 64) {
      while (n_wait > 0) {
        if (next_q == chunk_runs) {
          if (exhausted) break;
          // next chunk of items
          unsigned long long base = 0;
          if (lane == 0) base = atomicAdd(r.ctr, (unsigned long long)chunk);
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
          __syncthreads();   // earlier LDS reads of the previous chunk are complete
          if (lane < cnt) {
            const unsigned jj = chunk_base + lane;
            const size_t v = r.items.voxel(jj);
            if (r.items.stage) {
              // normalised already
              float cv[K];
              const float cn = load_staged<N>(r.items.stage, v, cv);
#pragma unroll
              for (int k = 0; k < K; ++k) cs[k][lane] = cv[k];
              cz[lane] = cn;
            } else {
              float cv[K];
              const float cn = load_tensor<N>(a, v, cv);
#pragma unroll
              for (int k = 0; k < K; ++k) cs[k][lane] = cv[k];
              const float inv = cn > 0.0f ? 1.0f / cn : 0.0f;
#pragma unroll
              for (int k = 0; k < K; ++k) cs[k][lane] *= inv;
              cz[lane] = cn;
            }
            ca[lane] = w.alpha[jj];
            if constexpr (CONT) {
              cu[lane] = w.cont_state[v];
              ci[lane] = w.cont_it[v] & ((1 << 30) - 1);
            }
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
              if constexpr (CONT) {
                const float4 sv = cu[jl];
                ux = sv.x; uy = sv.y; uz = sv.z;
                iters = ci[jl];
              } else {
                const float sx = st[3 * (r.s0 + s)], sy_ = st[3 * (r.s0 + s) + 1],
                            sz = st[3 * (r.s0 + s) + 2];
                const float rs = 1.0f / sqrtf(sx * sx + sy_ * sy_ + sz * sz);
                ux = sx * rs; uy = sy_ * rs; uz = sz * rs;
                iters = 0;
              }
              first = true;
              busy = true;
              ++n_runs;
            } else {
              w.res[(size_t)s * a.plane + j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
              if constexpr (CONT) w.conv[j] = 1;
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
        const float wx = fmaf(alpha, ux, g0), wy = fmaf(alpha, uy, g1), wz = fmaf(alpha, uz, g2);
        const float rn = rsqrtf(wx * wx + wy * wy + wz * wz);
        ux = wx * rn; uy = wy * rn; uz = wz * rn;
      }
      contract<N>(c, ux, uy, uz, g0, g1, g2);
      const float lam_new = g0 * ux + g1 * uy + g2 * uz;
      bool conv = false, end = false;
      if (first) {
        first = false;
      } else {
        ++iters;
        ++n_steps;
        conv = fabsf(lam_new - lam) <= a.tol;
        end = conv || iters >= a.max_iter;
      }
      lam = lam_new;
      if (end) {
        w.res[(size_t)s * a.plane + j] = make_float4(ux, uy, uz, lam);
        if constexpr (CONT) w.conv[j] = conv ? 1 : 0;
        busy = false;
      }
    }
  }
  if (a.counters) {
    count_add(a.counters + 0, n_steps);
    count_add(a.counters + 4, n_runs);
  }
}

// Per item: every run of one start block takes the Newton polish, and the
// largest polished lambda wins (first in start order on ties), carried across
// blocks; after the last block the winner is written (merge: only where it
// beats the answer already in the maps).
template <int N>
__global__ __launch_bounds__(256) void k_reduce(ExtractArgs a, Items it, int nsb, int first_block,
                                                int last_block, int merge) {
  constexpr int K = ncomp3(N);
  const Ws w = ws_layout(a.ws, a.plane);
  const unsigned n = it.n(a);
  unsigned long long n_newton = 0, n_oriented = 0;
  for (unsigned j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const size_t v = it.voxel(j);
    float c[K];
    const float cn = it.stage ? load_staged<N>(it.stage, v, c) : load_tensor<N>(a, v, c);
    float4 b = first_block ? make_float4(0.0f, 0.0f, 0.0f, -INFINITY) : w.best[j];
    if (cn > 0.0f) {
      if (!it.stage) scale<N>(c, 1.0f / cn);
      for (int s = 0; s < nsb; ++s) {
        const float4 r = w.res[(size_t)s * a.plane + j];
        float ux = r.x, uy = r.y, uz = r.z, g0, g1, g2;
        contract<N>(c, ux, uy, uz, g0, g1, g2);
        float lam = g0 * ux + g1 * uy + g2 * uz;
        n_newton += newton_polish<N>(c, ux, uy, uz, g0, g1, g2, lam, a.newton);
        if (lam > b.w) b = make_float4(ux, uy, uz, lam);
      }
    }
    if (!last_block) {
      w.best[j] = b;
    } else {
      float lam = 0.0f, ux = 0.0f, uy = 0.0f, uz = 0.0f;
      if (cn > 0.0f) {
        ux = b.x; uy = b.y; uz = b.z;
        canonical(ux, uy, uz);
        lam = b.w * cn;
        n_oriented += merge ? 0 : 1;
      }
      const Vox r = vox(a, v);
      if (!merge || lam > r.lam[r.o]) write_answer(r, lam, ux, uy, uz);
    }
  }
  if (a.counters) {
    count_add(a.counters + 1, n_newton);
    count_add(a.counters + 2, n_oriented);
  }
}

// ---------------------------------------------------------------------------
// learned start
// ---------------------------------------------------------------------------

// Polish, screen and write a learned-start answer; mark the voxel for the
// multistart search (status 2) when the run did not converge, the answer is
// not certified near a local maximum, lambda / ||C||_F < kappa, the network
// gave no direction, or some fixed start s already has <C, s^n> above lambda
// (SS-HOPM never lowers lambda, so the multistart answer is then higher).
// Certified: the tangent gradient |g - lambda u| is at most kCertifyGrad and
// the tangent Hessian's largest eigenvalue at most kCertifyCurv (a critical
// point to rounding level that is not a minimum or a clear saddle: degenerate
// maxima pass), or the tangent Hessian is negative definite and the next
// Newton step is at most kCertify long (a slow SS-HOPM run on a flat, curved
// ridge can meet its stopping rule far from the maximum); otherwise up to
// kCertifySteps Newton steps are taken (halved while lambda falls, as in the
// Newton search) and the test repeats.
constexpr float kCertify = 1e-2f;
constexpr float kCertifyGrad = 3e-5f;
constexpr float kCertifyCurv = 1e-3f;
constexpr int kCertifySteps = 4;

template <int N>
__device__ __forceinline__ unsigned long long learned_finish(
    const ExtractArgs& a, const Ws& w, const float (&c)[ncomp3(N)], float cn, size_t v,
    const float* mono, float ux, float uy, float uz, float g0, float g1, float g2, float lam,
    bool conv, bool forced, int polish, bool& fell) {
  constexpr int K = ncomp3(N);
  unsigned long long taken = newton_polish<N>(c, ux, uy, uz, g0, g1, g2, lam, polish);
  bool certified = false;
  for (int k = 0; k <= kCertifySteps; ++k) {
    float e[6], a00, a01, a11, t0, t1;
    ++taken;
    tangent_model<N>(c, ux, uy, uz, g0, g1, g2, lam, e, a00, a01, a11, t0, t1);
    const float amax = 0.5f * (a00 + a11) + 0.5f * sqrtf((a00 - a11) * (a00 - a11) + 4.0f * a01 * a01);
    if (t0 * t0 + t1 * t1 <= kCertifyGrad * kCertifyGrad && amax <= kCertifyCurv) {
      certified = true;
      break;
    }
    float dx, dy, dz;
    if (!tangent_step(e, a00, a01, a11, t0, t1, dx, dy, dz)) break;
    if (dx * dx + dy * dy + dz * dz <= kCertify * kCertify) {
      certified = true;
      break;
    }
    if (k == kCertifySteps) break;
    float vx, vy, vz, q0, q1, q2, lam_new, t = 1.0f;
    bool up = false;
    for (int h = 0; h <= kHalvings; ++h) {
      newton_move<N>(c, ux, uy, uz, dx, dy, dz, t, vx, vy, vz, q0, q1, q2, lam_new);
      if (lam_new >= lam - 1e-6f) {
        up = true;
        break;
      }
      t *= 0.5f;
    }
    if (!up) break;
    ux = vx; uy = vy; uz = vz;
    g0 = q0; g1 = q1; g2 = q2;
    lam = lam_new;
  }
  bool beaten = false;
  if (a.screen) {
    for (int s = 0; s < a.n_starts; ++s) {
      float f = 0.0f;
#pragma unroll
      for (int k = 0; k < K; ++k) f = fmaf(mono[s * K + k], c[k], f);
      beaten = beaten || f > lam;
    }
  }
  const bool fallback = forced || !conv || !certified || !(lam >= a.kappa) || beaten;
  canonical(ux, uy, uz);
  write_answer(vox(a, v), lam * cn, ux, uy, uz);
  w.status[v] = fallback ? 2 : 0;
  fell = fallback;
  return taken;
}

// Learned start directions alone (start_only): persistent wavefronts (one per
// workgroup) hold the network in registers and run it on 64 voxels at a time;
// writes the score and u0 = y / |y| (start 0 where the network gives no
// direction) into the direction maps.
constexpr int kMlpGroups = 2048;

template <int N>
__global__ __launch_bounds__(64) void k_mlp_start(ExtractArgs a) {
  constexpr int K = ncomp3(N);
  constexpr Sym3<N> sy{};
  __shared__ unsigned short xs[64 * kMlpIn];
  const int lane = threadIdx.x;
  MlpRegs net;
  load_mlp_regs(a.mlp, lane, net);
  const float s0x = a.starts[0], s0y = a.starts[1], s0z = a.starts[2];
  const size_t n_groups = (a.plane + 63) / 64;
  float c[K];
  if (blockIdx.x < n_groups) {
    const size_t v0 = (size_t)blockIdx.x * 64 + lane;
    load_raw<N>(a, v0 < a.plane ? v0 : a.plane - 1, c);
  }
  for (size_t gi = blockIdx.x; gi < n_groups; gi += gridDim.x) {
    const size_t v0 = gi * 64 + lane;
    const bool active = v0 < a.plane;
    const size_t v = active ? v0 : a.plane - 1;
    // the next group's tensors are loaded while this group runs through the network
    float cx[K];
    const size_t gn = gi + gridDim.x;
    if (gn < n_groups) {
      const size_t vn = gn * 64 + lane;
      load_raw<N>(a, vn < a.plane ? vn : a.plane - 1, cx);
    }
    const float cn = frob<N>(c);
    const Vox vr = vox(a, v);
    if ((a.mode & 1) && active && vr.score) vr.score[vr.o] = cn;
    const float inv = cn > 0.0f ? 1.0f / cn : 0.0f;
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k)
      xs[lane * kMlpIn + k] = k < K ? bf16_bits(sqrtf(sy.mu[k]) * c[k] * inv) : (unsigned short)0;
    float y0, y1, y2;
    mlp_forward(xs, net, lane, y0, y1, y2);
    const float ny = sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
    const bool forced = !(ny > 0.0f);
    float ux = forced ? s0x : y0, uy = forced ? s0y : y1, uz = forced ? s0z : y2;
    const float r = 1.0f / sqrtf(ux * ux + uy * uy + uz * uz);
    ux *= r; uy *= r; uz *= r;
    if (active) write_answer(vr, 0.0f, ux, uy, uz);
    __syncthreads();   // xs is rewritten by the next group
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = cx[k];
  }
}

// Learned start and Newton search in one pass over the field: persistent
// workgroups of kLearnedWaves wavefronts, each taking 64 voxels at a time
// (voxel = lane).  The network, read from an LDS copy shared by the
// workgroup, gives u0 = y / |y| on the matrix cores (start 0 if y = 0, which
// also forces the fallback); each lane then takes up to kNewtonFirst Newton
// steps from u0.  Converged voxels are screened and written (status 0 or 2),
// the others marked for SS-HOPM from u0 (status 1, with u0 and its lambda
// kept per voxel).  Each lane loads its next voxel's tensor before working on
// the current one, and nothing in the loop waits on a memory result, so the
// loads' latency hides behind the network and the Newton steps.
constexpr int kLearnedGroups = 1024;
constexpr int kLearnedWaves = 4;

template <int N>
__global__ __launch_bounds__(64 * kLearnedWaves) void k_learned(ExtractArgs a) {
  constexpr int K = ncomp3(N);
  constexpr Sym3<N> sy{};
  __shared__ float st[64 * 3];
  __shared__ float mono[64 * K];
  __shared__ __align__(16) unsigned char pk[kMlpPackedBytes];
  __shared__ unsigned short xs_all[kLearnedWaves][64 * kMlpIn];
  static_assert(kMlpPackedBytes % 16 == 0, "packed network copied in 16-byte pieces");
  for (int i = threadIdx.x; i < a.n_starts * 3; i += blockDim.x) st[i] = a.starts[i];
  for (int i = threadIdx.x; i < kMlpPackedBytes / 16; i += blockDim.x)
    reinterpret_cast<uint4*>(pk)[i] = reinterpret_cast<const uint4*>(a.mlp)[i];
  __syncthreads();
  if (a.screen) build_monomials<N>(st, a.n_starts, mono);
  __syncthreads();
  const Ws w = ws_layout(a.ws, a.plane);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned short* xs = xs_all[wave];
  const MlpLds net{pk, lane};
  const float s0x = st[0], s0y = st[1], s0z = st[2];
  const size_t n_groups = (a.plane + 63) / 64;
  const size_t gstride = (size_t)gridDim.x * kLearnedWaves;
  size_t gi = (size_t)blockIdx.x * kLearnedWaves + wave;
  unsigned long long n_newton = 0, n_oriented = 0;
  float c[K];
  if (gi < n_groups) {
    const size_t v0 = gi * 64 + lane;
    load_raw<N>(a, v0 < a.plane ? v0 : a.plane - 1, c);
  }
  for (; gi < n_groups; gi += gstride) {
    const size_t v0 = gi * 64 + lane;
    const bool active = v0 < a.plane;
    const size_t v = active ? v0 : a.plane - 1;
    float cx[K];
    const size_t gn = gi + gstride;
    if (gn < n_groups) {
      const size_t vn = gn * 64 + lane;
      load_raw<N>(a, vn < a.plane ? vn : a.plane - 1, cx);
    }
    const float cn = frob<N>(c);
    const Vox vr = vox(a, v);
    if ((a.mode & 1) && active && vr.score) vr.score[vr.o] = cn;
    const float inv = cn > 0.0f ? 1.0f / cn : 0.0f;
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k)
      xs[lane * kMlpIn + k] = k < K ? bf16_bits(sqrtf(sy.mu[k]) * c[k] * inv) : (unsigned short)0;
    wave_lds_sync();
    float y0, y1, y2;
    mlp_forward_w(xs, net, lane, y0, y1, y2);
    const float ny = sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
    const bool forced = !(ny > 0.0f);
    float ux = forced ? s0x : y0, uy = forced ? s0y : y1, uz = forced ? s0z : y2;
    const float r = 1.0f / sqrtf(ux * ux + uy * uy + uz * uz);
    ux *= r; uy *= r; uz *= r;
    if (active) {
      if (cn > 0.0f) {
        scale<N>(c, inv);
        const float u0x = ux, u0y = uy, u0z = uz;
        float g0, g1, g2;
        contract<N>(c, ux, uy, uz, g0, g1, g2);
        float lam = g0 * ux + g1 * uy + g2 * uz;
        const float lam0 = lam;
        bool ok;
        n_newton += newton_ascent<N>(c, ux, uy, uz, g0, g1, g2, lam, kNewtonFirst, a.tol, ok);
        n_oriented += 1;
        bool fell = true;
        if (ok) {
          n_newton += learned_finish<N>(a, w, c, cn, v, mono, ux, uy, uz, g0, g1, g2, lam, true,
                                        forced, 0, fell);
        } else {
          // SS-HOPM from the learned start, run by the pooled kernel
          w.status[v] = 1;
          w.cont_state[v] = make_float4(u0x, u0y, u0z, lam0);
          w.cont_it[v] = forced ? (1 << 30) : 0;
        }
        // the voxels handed on read their tensor from here, in one piece
        if (fell) store_staged<N>(w.stage, v, c, cn);
      } else {
        write_answer(vr, 0.0f, 0.0f, 0.0f, 0.0f);
        w.status[v] = 0;
      }
    }
    wave_lds_sync();   // xs is rewritten by the next group
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = cx[k];
  }
  if (a.counters) {
    count_add(a.counters + 1, n_newton);
    count_add(a.counters + 2, n_oriented);
  }
}

// Finish the continued learned-start runs (k_runs with cont) as k_learned does.
template <int N>
__global__ __launch_bounds__(256) void k_learned_post(ExtractArgs a) {
  constexpr int K = ncomp3(N);
  __shared__ float st[64 * 3];
  __shared__ float mono[64 * K];
  for (int i = threadIdx.x; i < a.n_starts * 3; i += blockDim.x) st[i] = a.starts[i];
  __syncthreads();
  if (a.screen) build_monomials<N>(st, a.n_starts, mono);
  __syncthreads();
  const Ws w = ws_layout(a.ws, a.plane);
  const unsigned n = w.hdr[kHdrContinue];
  unsigned long long n_newton = 0;
  for (unsigned j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const size_t v = w.cont_list[j];
    float c[K];
    const float cn = load_staged<N>(w.stage, v, c);
    const float4 r = w.res[j];
    float ux = r.x, uy = r.y, uz = r.z;
    float g0, g1, g2;
    contract<N>(c, ux, uy, uz, g0, g1, g2);
    const float lam = g0 * ux + g1 * uy + g2 * uz;
    const bool forced = (w.cont_it[v] >> 30) & 1;
    bool fell;
    n_newton += learned_finish<N>(a, w, c, cn, v, mono, ux, uy, uz, g0, g1, g2, lam,
                                  w.conv[j] != 0, forced, a.newton, fell);
  }
  if (a.counters) count_add(a.counters + 1, n_newton);
}

// ---------------------------------------------------------------------------
// list compaction: the box voxels whose status equals `value`, in voxel order
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned block_count(const unsigned char* status, size_t plane,
                                                size_t base, unsigned char value,
                                                unsigned& mine_mask) {
  // thread t of the workgroup owns voxels base + t * 16 ... + 15
  mine_mask = 0;
  const size_t v0 = base + (size_t)threadIdx.x * 16;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const size_t v = v0 + i;
    if (v < plane && status[v] == value) mine_mask |= 1u << i;
  }
  return __popc(mine_mask);
}

__global__ __launch_bounds__(256) void k_flag_count(const unsigned char* status, size_t plane,
                                                    unsigned char value, unsigned* blocksum) {
  __shared__ unsigned part[4];
  unsigned mask;
  unsigned cnt = block_count(status, plane, (size_t)blockIdx.x * kCompactBlock, value, mask);
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) blocksum[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Exclusive scan of the block counts (one workgroup); total -> *count.
__global__ __launch_bounds__(1024) void k_flag_scan(unsigned* blocksum, int nblk, unsigned* count) {
  __shared__ unsigned sums[1024];
  unsigned carry = 0;
  for (int base = 0; base < nblk; base += 1024) {
    const int i = base + (int)threadIdx.x;
    const unsigned x = i < nblk ? blocksum[i] : 0u;
    sums[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const unsigned y = threadIdx.x >= (unsigned)off ? sums[threadIdx.x - off] : 0u;
      __syncthreads();
      sums[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < nblk) blocksum[i] = carry + sums[threadIdx.x] - x;
    const unsigned tot = sums[1023];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) *count = carry;
}

__global__ __launch_bounds__(256) void k_flag_scatter(const unsigned char* status, size_t plane,
                                                      unsigned char value,
                                                      const unsigned* blocksum, unsigned* list) {
  __shared__ unsigned part[4];
  unsigned mask;
  const size_t base = (size_t)blockIdx.x * kCompactBlock;
  const unsigned cnt = block_count(status, plane, base, value, mask);
  // inclusive scan over the workgroup's threads (in thread order = voxel order)
  unsigned incl = cnt;
  const int lane = threadIdx.x & 63;
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) part[threadIdx.x >> 6] = incl;
  __syncthreads();
  unsigned wave_off = 0;
  for (int wv = 0; wv < (int)(threadIdx.x >> 6); ++wv) wave_off += part[wv];
  unsigned pos = blocksum[blockIdx.x] + wave_off + incl - cnt;
  const size_t v0 = base + (size_t)threadIdx.x * 16;
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (mask & (1u << i)) list[pos++] = (unsigned)(v0 + i);
}

void compact(const Ws& w, size_t plane, unsigned char value, unsigned* list, unsigned* count,
             hipStream_t s) {
  const int nblk = (int)((plane + kCompactBlock - 1) / kCompactBlock);
  hipLaunchKernelGGL(k_flag_count, dim3(nblk), dim3(256), 0, s, w.status, plane, value, w.blocksum);
  hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, s, w.blocksum, nblk, count);
  hipLaunchKernelGGL(k_flag_scatter, dim3(nblk), dim3(256), 0, s, w.status, plane, value,
                     w.blocksum, list);
}

}  // namespace

size_t extract_workspace(size_t plane, int degree) {
  const int K = (degree + 1) * (degree + 2) / 2;
  return 256 + al256(plane * 4) * 2 + al256(plane * 16) + al256(plane * 4) * 2 + al256(plane) +
         al256(plane * 16) + al256(plane) + al256(((plane + kCompactBlock - 1) / kCompactBlock) * 4) +
         (size_t)kStartBlock * plane * 16 + plane * 16 * (size_t)stage_slots(K);
}

// Workgroups of the per-item kernels (k_prepare, k_reduce, k_learned_post):
// they loop over their items, so a list whose length only the device knows
// costs no launch of hundreds of thousands of empty workgroups.
constexpr unsigned kItemGroups = 1024;

template <int N>
int launch_multistart(const ExtractArgs& a, Items it, unsigned long long* ctr_base, int merge,
                      hipStream_t s) {
  const unsigned nb0 = (unsigned)((a.plane + 255) / 256);
  const unsigned nb = nb0 < kItemGroups ? nb0 : kItemGroups;
  const int n_blocks = (a.n_starts + kStartBlock - 1) / kStartBlock;
  hipLaunchKernelGGL((k_prepare<N>), dim3(nb), dim3(256), 0, s, a, it,
                     merge ? 0 : (a.mode & 1), merge);
  for (int b = 0; b < n_blocks; ++b) {
    const int nsb = (a.n_starts - b * kStartBlock) < kStartBlock ? (a.n_starts - b * kStartBlock)
                                                                 : kStartBlock;
    RunArgs r{it, nsb, b * kStartBlock, ctr_base + b};
    hipLaunchKernelGGL((k_runs<N, false>), dim3(kPoolGroups), dim3(64), 0, s, a, r);
    hipLaunchKernelGGL(k_reduce<N>, dim3(nb), dim3(256), 0, s, a, it, nsb, b == 0 ? 1 : 0,
                       b == n_blocks - 1 ? 1 : 0, merge);
  }
  return 0;
}

template <int N>
int launch_n(const ExtractArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)((a.plane + 255) / 256);
  if constexpr (N >= 2) {
    if (a.mode & 2) {
      const Ws w = ws_layout(a.ws, a.plane);
      fill_zero(w.hdr, 256, s);
      unsigned long long* ctr = reinterpret_cast<unsigned long long*>(w.hdr);
      if ((a.mode & 4) == 0) {
        launch_multistart<N>(a, Items{nullptr, nullptr, nullptr}, ctr + kHdrPoolDense / 2, 0, s);
      } else {
        const size_t n_groups = (a.plane + 63) / 64;
        if (a.start_only) {
          const unsigned mg = (unsigned)(n_groups < (size_t)kMlpGroups ? n_groups : kMlpGroups);
          hipLaunchKernelGGL((k_mlp_start<N>), dim3(mg), dim3(64), 0, s, a);
        } else {
          const size_t wg = (n_groups + kLearnedWaves - 1) / kLearnedWaves;
          const unsigned lg = (unsigned)(wg < (size_t)kLearnedGroups ? wg : kLearnedGroups);
          hipLaunchKernelGGL((k_learned<N>), dim3(lg), dim3(64 * kLearnedWaves), 0, s, a);
          compact(w, a.plane, 1, w.cont_list, &w.hdr[kHdrContinue], s);
          const Items cont{w.cont_list, &w.hdr[kHdrContinue], w.stage};
          const unsigned ib = nb < kItemGroups ? nb : kItemGroups;
          hipLaunchKernelGGL((k_prepare<N>), dim3(ib), dim3(256), 0, s, a, cont, 0, 0);
          RunArgs r{cont, 1, 0, ctr + kHdrPoolCont / 2};
          hipLaunchKernelGGL((k_runs<N, true>), dim3(kPoolGroups), dim3(64), 0, s, a, r);
          hipLaunchKernelGGL(k_learned_post<N>, dim3(ib), dim3(256), 0, s, a);
          compact(w, a.plane, 2, w.fb_list, &w.hdr[kHdrFallbacks], s);
          launch_multistart<N>(a, Items{w.fb_list, &w.hdr[kHdrFallbacks], w.stage}, ctr + kHdrPoolFb / 2,
                               1, s);
        }
      }
      hipError_t e = hipGetLastError();
      return e == hipSuccess ? 0 : hip_status(e, "extract launch");
    }
  }
  hipLaunchKernelGGL(k_score<N>, dim3(nb), dim3(256), 0, s, a);
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
