// refine.hip -- position refinement TTM-ref (Sec. 3.3, Alg. 3) and the tensor
// field at listed voxels by real-space sums (gfx950).
//
// For each peak x^i of the score map the search visits the sphere of voxels
// |x - x^i| <= r_s (the peak first, then the other offsets in lexicographic
// (dz, dy, dx) order, skipping voxels outside the valid region), takes at
// each voxel the optimal rotation of its tensor C(x) (the dominant
// eigenvector on S^3, d' = 4, Sec. 3.1) and the LNCC at that single rotation,
//   c(x, R) = w(x) sum_p g(x + p - c) t'(c + R^T (p - c))      (Eq. lncc),
// computed in real space from the template window, and keeps the voxel with
// the largest LNCC (a later voxel only on a strictly larger value, so ties
// keep the earlier one and the peak itself stays unless beaten).
//
// Kernels: k_offsets (the sphere's offsets), k_candidates (peak x offset ->
// voxel, or invalid), k_field_at (C at every candidate: a workgroup per peak
// and candidate block, the template components staged through LDS in chunks
// of template voxels, one candidate per thread with its K sums in registers),
// the d' = 4 multistart extraction (extract4.hip) on those tensors,
// k_lncc (a workgroup per candidate, only template voxels within r + 2 of the
// centre, where the rotated t' can be non-zero), k_best (one thread per peak).
#include "internal.hpp"

namespace ttm {

namespace {

constexpr int kFieldThreads = 128;   // candidates per k_field_at workgroup
constexpr int kFieldChunk = 256;     // template voxels staged per LDS chunk
// Template voxels per LDS chunk for K components: kFieldChunk, or half of it
// where that many would take more than 48 KB (K = 84 at degree 6: 128 voxels).
__host__ __device__ constexpr int field_chunk(int K) {
  return ((K + 3) / 4 * 4) * kFieldChunk * 4 <= 48 * 1024 ? kFieldChunk : kFieldChunk / 2;
}
constexpr int kMaxRefineRadius = 8;

struct RefineWs {
  int4* offs;       // sphere offsets (dz, dy, dx, 0), the zero offset first
  int* n_offs;
  int4* cand;       // candidate voxel (z, y, x, valid)
  float* C;         // K x (n_peaks * V) tensors
  float* lam;       // n_peaks * V
  float* quat;      // n_peaks * V x 4
  float* lncc;      // n_peaks * V
  void* ext;        // d' = 4 extraction workspace
};

__host__ __device__ inline size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// Offsets of the sphere of radius r_s as the device kernels enumerate them.
int sphere_count(float rs) {
  const int R = (int)floorf(rs);
  int n = 0;
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx)
        if ((float)(dz * dz + dy * dy + dx * dx) <= rs * rs) ++n;
  return n;
}

namespace {

RefineWs refine_layout(void* base, int K, size_t n_cand) {
  char* p = static_cast<char*>(base);
  RefineWs w;
  w.offs = reinterpret_cast<int4*>(p);
  p += a256((size_t)(2 * kMaxRefineRadius + 1) * (2 * kMaxRefineRadius + 1) * (2 * kMaxRefineRadius + 1) * 16);
  w.n_offs = reinterpret_cast<int*>(p);
  p += 256;
  w.cand = reinterpret_cast<int4*>(p);
  p += a256(n_cand * 16);
  w.C = reinterpret_cast<float*>(p);
  p += a256((size_t)K * n_cand * 4);
  w.lam = reinterpret_cast<float*>(p);
  p += a256(n_cand * 4);
  w.quat = reinterpret_cast<float*>(p);
  p += a256(n_cand * 16);
  w.lncc = reinterpret_cast<float*>(p);
  p += a256(n_cand * 4);
  w.ext = p;
  return w;
}

__global__ void k_offsets(float rs, int4* offs, int* n_offs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int R = (int)floorf(rs);
  int n = 0;
  offs[n++] = make_int4(0, 0, 0, 0);
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx)
        if ((dz | dy | dx) != 0 && (float)(dz * dz + dy * dy + dx * dx) <= rs * rs)
          offs[n++] = make_int4(dz, dy, dx, 0);
  *n_offs = n;
}

// Candidate i * V + j = peak i + offset j, valid when its template window lies
// inside the volume (lo <= voxel <= hi on every axis).
__global__ void k_candidates(const int32_t* __restrict__ peaks, int n_peaks, const int4* __restrict__ offs,
                             int V, int4 lo, int4 hi, int4* __restrict__ cand) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)n_peaks * V) return;
  const int i = (int)(k / V), j = (int)(k % V);
  const int4 o = offs[j];
  const int z = peaks[3 * i] + o.x, y = peaks[3 * i + 1] + o.y, x = peaks[3 * i + 2] + o.z;
  const bool ok = z >= lo.x && z <= hi.x && y >= lo.y && y <= hi.y && x >= lo.z && x <= hi.z;
  cand[k] = make_int4(z, y, x, ok ? 1 : 0);
}

// C_k(x) = w(x) sum_p g(x + p - c) T_k(p) at every candidate x (Eq. tcc at
// single voxels).  Workgroup (peak, block of kFieldThreads candidates); the
// template components of field_chunk(K) template voxels at a time sit in LDS as
// [p][K] (every thread reads the same entry: a broadcast).
template <int K>
__global__ __launch_bounds__(kFieldThreads) void k_field_at(const float* __restrict__ g,
                                                            const float* __restrict__ w, int ny, int nx,
                                                            const float* __restrict__ T, int L,
                                                            const int4* __restrict__ cand, int V,
                                                            size_t n_cand, float* __restrict__ C) {
  constexpr int KP = (K + 3) / 4 * 4;
  constexpr int CH = field_chunk(K);
  __shared__ __align__(16) float tl[CH * KP];
  const int j = blockIdx.y * kFieldThreads + threadIdx.x;
  const size_t k = (size_t)blockIdx.x * V + j;
  const bool live = j < V && cand[k].w != 0;
  const int4 cv = live ? cand[k] : make_int4(0, 0, 0, 0);
  const int c = L / 2;
  const size_t base = live ? ((size_t)(cv.x - c) * ny + (cv.y - c)) * nx + (cv.z - c) : 0;
  float acc[K];
#pragma unroll
  for (int a = 0; a < K; ++a) acc[a] = 0.0f;
  const int np = L * L * L;
  for (int p0 = 0; p0 < np; p0 += CH) {
    const int cnt = min(CH, np - p0);
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * K; e += kFieldThreads) {
      const int a = e / cnt, pp = e % cnt;   // read each component's run of voxels in order
      tl[pp * KP + a] = T[(size_t)a * np + p0 + pp];
    }
    __syncthreads();
    if (live) {
      int pz = p0 / (L * L), py = (p0 / L) % L, px = p0 % L;
      for (int pp = 0; pp < cnt; ++pp) {
        const float gv = g[base + ((size_t)pz * ny + py) * nx + px];
        const float4* t4 = reinterpret_cast<const float4*>(&tl[pp * KP]);
#pragma unroll
        for (int a4 = 0; a4 < KP / 4; ++a4) {
          const float4 t = t4[a4];
          if (4 * a4 + 0 < K) acc[4 * a4 + 0] = fmaf(t.x, gv, acc[4 * a4 + 0]);
          if (4 * a4 + 1 < K) acc[4 * a4 + 1] = fmaf(t.y, gv, acc[4 * a4 + 1]);
          if (4 * a4 + 2 < K) acc[4 * a4 + 2] = fmaf(t.z, gv, acc[4 * a4 + 2]);
          if (4 * a4 + 3 < K) acc[4 * a4 + 3] = fmaf(t.w, gv, acc[4 * a4 + 3]);
        }
        if (++px == L) {
          px = 0;
          if (++py == L) {
            py = 0;
            ++pz;
          }
        }
      }
    }
  }
  if (j < V) {
    const float wv = live ? w[((size_t)cv.x * ny + cv.y) * nx + cv.z] : 0.0f;
#pragma unroll
    for (int a = 0; a < K; ++a) C[(size_t)a * n_cand + k] = live ? wv * acc[a] : 0.0f;
  }
}

// LNCC of every candidate at its own rotation (Eq. lncc), in real space.
__global__ __launch_bounds__(256) void k_lncc(const float* __restrict__ g, const float* __restrict__ w,
                                              int ny, int nx, const float* __restrict__ tn, int L,
                                              float r, const int4* __restrict__ cand,
                                              const float* __restrict__ quat, float* __restrict__ lncc) {
  __shared__ float red[4];
  const size_t k = blockIdx.x;
  const int4 cv = cand[k];
  if (cv.w == 0) {
    if (threadIdx.x == 0) lncc[k] = -INFINITY;
    return;
  }
  float qw = quat[4 * k], qx = quat[4 * k + 1], qy = quat[4 * k + 2], qz = quat[4 * k + 3];
  const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  if (!(qn > 0.0f)) {     // zero tensor: no rotation, the identity stands in
    qw = 1.0f; qx = qy = qz = 0.0f;
  } else {
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
  }
  const float R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                      2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                      2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
  const int c = L / 2;
  const float cf = (float)c;
  const float lim = (r + 2.0f) * (r + 2.0f);
  const size_t base = ((size_t)(cv.x - c) * ny + (cv.y - c)) * nx + (cv.z - c);
  float acc = 0.0f;
  const int np = L * L * L;
  for (int p = threadIdx.x; p < np; p += 256) {
    const int pz = p / (L * L), py = (p / L) % L, px = p % L;
    const float dx = (float)(px - c), dy = (float)(py - c), dz = (float)(pz - c);
    if (dx * dx + dy * dy + dz * dz > lim) continue;
    // source point c + R^T (p - c), (x, y, z)
    const float sx = cf + R[0] * dx + R[3] * dy + R[6] * dz;
    const float sy = cf + R[1] * dx + R[4] * dy + R[7] * dz;
    const float sz = cf + R[2] * dx + R[5] * dy + R[8] * dz;
    const float fx = floorf(sx), fy = floorf(sy), fz = floorf(sz);
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    const float tx = sx - fx, ty = sy - fy, tz = sz - fz;
    float val = 0.0f;
#pragma unroll
    for (int oz = 0; oz < 2; ++oz) {
      const int zz = iz + oz;
      if (zz < 0 || zz >= L) continue;
      const float wz = oz ? tz : 1.0f - tz;
#pragma unroll
      for (int oy = 0; oy < 2; ++oy) {
        const int yy = iy + oy;
        if (yy < 0 || yy >= L) continue;
        const float wy = oy ? ty : 1.0f - ty;
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
          const int xx = ix + ox;
          if (xx < 0 || xx >= L) continue;
          const float wx = ox ? tx : 1.0f - tx;
          val += wz * wy * wx * tn[((size_t)zz * L + yy) * L + xx];
        }
      }
    }
    acc = fmaf(val, g[base + ((size_t)pz * ny + py) * nx + px], acc);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float s = (red[0] + red[1]) + (red[2] + red[3]);
    lncc[k] = w[((size_t)cv.x * ny + cv.y) * nx + cv.z] * s;
  }
}

// Per peak: the candidate with the largest LNCC, the peak itself first and a
// later candidate only on a strictly larger value.
__global__ void k_best(const int4* __restrict__ cand, const float* __restrict__ quat,
                       const float* __restrict__ lncc, int n_peaks, int V, int32_t* __restrict__ pos_out,
                       float* __restrict__ quat_out, float* __restrict__ lncc_out,
                       float* __restrict__ quat_peak, float* __restrict__ lncc_peak) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_peaks) return;
  const size_t k0 = (size_t)i * V;
  size_t best = k0;
  float bv = lncc[k0];
  for (int j = 1; j < V; ++j) {
    const float v = lncc[k0 + j];
    if (v > bv) {
      bv = v;
      best = k0 + j;
    }
  }
  pos_out[3 * i] = cand[best].x;
  pos_out[3 * i + 1] = cand[best].y;
  pos_out[3 * i + 2] = cand[best].z;
  lncc_out[i] = bv;
#pragma unroll
  for (int d = 0; d < 4; ++d) quat_out[4 * i + d] = quat[4 * best + d];
  if (quat_peak) {
#pragma unroll
    for (int d = 0; d < 4; ++d) quat_peak[4 * i + d] = quat[4 * k0 + d];
  }
  if (lncc_peak) lncc_peak[i] = lncc[k0];
}

template <int K>
void launch_field_at(const float* g, const float* w, int ny, int nx, const float* T, int L,
                     const int4* cand, int n_groups, int V, size_t n_cand, float* C, hipStream_t s) {
  const dim3 grid(n_groups, (V + kFieldThreads - 1) / kFieldThreads);
  hipLaunchKernelGGL(k_field_at<K>, grid, dim3(kFieldThreads), 0, s, g, w, ny, nx, T, L, cand, V,
                     n_cand, C);
}

}  // namespace

size_t refine_workspace(int K, int n_peaks, float rs) {
  const size_t n_cand = (size_t)n_peaks * sphere_count(rs);
  return a256((size_t)(2 * kMaxRefineRadius + 1) * (2 * kMaxRefineRadius + 1) * (2 * kMaxRefineRadius + 1) * 16) +
         256 + a256(n_cand * 16) + a256((size_t)K * n_cand * 4) + a256(n_cand * 4) + a256(n_cand * 16) +
         a256(n_cand * 4) + extract_workspace4(n_cand);
}

int max_refine_radius() { return kMaxRefineRadius; }

// Field at listed candidates; K must be one of the built component counts.
int field_at(int K, const float* g, const float* w, int ny, int nx, const float* T, int L,
             const int4* cand, int n_groups, int V, size_t n_cand, float* C, hipStream_t s) {
  switch (K) {
    case 1: launch_field_at<1>(g, w, ny, nx, T, L, cand, n_groups, V, n_cand, C, s); break;
    case 4: launch_field_at<4>(g, w, ny, nx, T, L, cand, n_groups, V, n_cand, C, s); break;
    case 6: launch_field_at<6>(g, w, ny, nx, T, L, cand, n_groups, V, n_cand, C, s); break;
    case 10: launch_field_at<10>(g, w, ny, nx, T, L, cand, n_groups, V, n_cand, C, s); break;
    case 15: launch_field_at<15>(g, w, ny, nx, T, L, cand, n_groups, V, n_cand, C, s); break;
    case 28: launch_field_at<28>(g, w, ny, nx, T, L, cand, n_groups, V, n_cand, C, s); break;
    case 35: launch_field_at<35>(g, w, ny, nx, T, L, cand, n_groups, V, n_cand, C, s); break;
    case 84: launch_field_at<84>(g, w, ny, nx, T, L, cand, n_groups, V, n_cand, C, s); break;
    default: set_error("field at listed voxels: %d components not built", K); return -4;
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : hip_status(e, "field_at launch");
}

int refine(int degree, int K, const float* g, const float* w, int nz, int ny, int nx, const float* T,
           const float* tn, int L, float r, const int32_t* peaks, int n_peaks, float rs,
           const ExtractArgs& opts, int32_t* pos_out, float* quat_out, float* lncc_out,
           float* quat_peak, float* lncc_peak, void* ws, hipStream_t s) {
  const int V = sphere_count(rs);
  const size_t n_cand = (size_t)n_peaks * V;
  const RefineWs rw = refine_layout(ws, K, n_cand);
  hipLaunchKernelGGL(k_offsets, dim3(1), dim3(64), 0, s, rs, rw.offs, rw.n_offs);
  const int c = L / 2;
  const int4 lo = make_int4(c, c, c, 0), hi = make_int4(nz - L + c, ny - L + c, nx - L + c, 0);
  hipLaunchKernelGGL(k_candidates, dim3((unsigned)((n_cand + 255) / 256)), dim3(256), 0, s, peaks,
                     n_peaks, rw.offs, V, lo, hi, rw.cand);
  int rc = field_at(K, g, w, ny, nx, T, L, rw.cand, n_peaks, V, n_cand, rw.C, s);
  if (rc) return rc;
  ExtractArgs a = opts;
  a.items = nullptr;
  a.n_items = 0;
  a.C = rw.C;
  a.in_dtype = 0;
  a.plane = n_cand;
  a.by = 1;
  a.bx = (int)n_cand;
  a.score = nullptr;
  a.lam = rw.lam;
  a.dir = rw.quat;
  a.oz = a.oy = a.ox = 0;
  a.dy = 1;
  a.dx = (int)n_cand;
  a.mode = 2;
  a.ws = rw.ext;
  rc = launch_extract4(degree, a, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_lncc, dim3((unsigned)n_cand), dim3(256), 0, s, g, w, ny, nx, tn, L, r, rw.cand,
                     rw.quat, rw.lncc);
  hipLaunchKernelGGL(k_best, dim3((n_peaks + 63) / 64), dim3(64), 0, s, rw.cand, rw.quat, rw.lncc,
                     n_peaks, V, pos_out, quat_out, lncc_out, quat_peak, lncc_peak);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : hip_status(e, "refine launch");
}

}  // namespace ttm
