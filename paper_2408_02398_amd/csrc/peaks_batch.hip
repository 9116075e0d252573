// peaks_batch.hip -- exact greedy Find Peaks for many score maps in one
// launch (gfx950), for batches of subtomograms that each want few peaks.
//
// The rule (Sec. 3.4) keeps, again and again, the first voxel in visiting
// order (descending score, ties by ascending linear index z*ny*nx + y*nx + x)
// that lies at least D from every peak kept so far, until P peaks are kept or
// none is left.  With the 64-bit key (~score_bits << 32 | linear index) the
// visiting order is ascending key order, so each step takes the smallest key
// among the voxels not yet excluded; after a peak is kept, the voxels of its
// exclusion ball (distance < D) are excluded.  That is the greedy result
// itself, with no sort of the map:
//   k_block_keys  the smallest key of every 8^3 block of every item's valid
//                 region (one workgroup per block)
//   k_nms         one workgroup per item: P times, the smallest block key is
//                 the next peak (or none is left); the ball's voxels are set
//                 in the item's exclusion bitmask, and the blocks the ball
//                 touches are updated: emptied when they lie inside it,
//                 rescanned without the excluded voxels when their smallest
//                 key's voxel was excluded, and otherwise left as they are.
// Every item's work is independent, so one launch serves the whole batch.
#include "../../include/ttm.h"
#include "internal.hpp"

namespace ttm {

namespace {

constexpr int kBlk = 8;                 // block edge (voxels)
constexpr int kNmsThreads = 1024;
constexpr int kMaxBatchPeaks = 4096;

__device__ __forceinline__ unsigned sbits(float s) { return (s > 0.0f) ? __float_as_uint(s) : 0u; }

struct ItemGeo {
  int vz, vy, vx;       // valid box extent
  int bz, by, bx;       // blocks per axis
  size_t words;         // bitmask words
};

__host__ __device__ inline ItemGeo geo(const int32_t lo[3], const int32_t hi[3]) {
  ItemGeo g;
  g.vz = hi[0] - lo[0] + 1;
  g.vy = hi[1] - lo[1] + 1;
  g.vx = hi[2] - lo[2] + 1;
  g.bz = (g.vz + kBlk - 1) / kBlk;
  g.by = (g.vy + kBlk - 1) / kBlk;
  g.bx = (g.vx + kBlk - 1) / kBlk;
  g.words = ((size_t)g.vz * g.vy * g.vx + 31) / 32;
  return g;
}

__host__ __device__ inline size_t a256b(size_t b) { return (b + 255) & ~(size_t)255; }

// An item the kernels can serve: its valid box inside its map, at least one
// peak wanted, a map of fewer than 2^32 voxels (linear indices fit the key).
__device__ __forceinline__ bool item_ok(const ttm_peak_item& it) {
  for (int a = 0; a < 3; ++a)
    if (it.valid_lo[a] < 0 || it.valid_hi[a] >= it.dims[a] || it.valid_lo[a] > it.valid_hi[a]) return false;
  return it.top_p >= 1 && it.top_p <= kMaxBatchPeaks && it.min_dist >= 0.0f && it.score && it.peaks && it.vals && it.n_found &&
         it.scratch && (unsigned long long)it.dims[0] * it.dims[1] * it.dims[2] < (1ull << 32);
}

// scratch of one item: block keys, then the exclusion bitmask (one bit per
// valid voxel, x fastest)
__host__ __device__ inline void scratch_layout(void* base, const ItemGeo& g,
                                               unsigned long long** keys, unsigned** bits) {
  char* p = static_cast<char*>(base);
  *keys = reinterpret_cast<unsigned long long*>(p);
  *bits = reinterpret_cast<unsigned*>(p + a256b((size_t)g.bz * g.by * g.bx * 8));
}

__device__ __forceinline__ unsigned long long voxel_key(const ttm_peak_item& it, const ItemGeo& g,
                                                        const unsigned* bits, int vz, int vy, int vx) {
  const size_t vi = ((size_t)vz * g.vy + vy) * g.vx + vx;
  if ((bits[vi >> 5] >> (vi & 31)) & 1u) return ~0ull;
  const int z = it.valid_lo[0] + vz, y = it.valid_lo[1] + vy, x = it.valid_lo[2] + vx;
  const size_t lin = ((size_t)z * it.dims[1] + y) * it.dims[2] + x;
  return ((unsigned long long)(~sbits(it.score[lin])) << 32) | (unsigned long long)lin;
}

__device__ __forceinline__ unsigned long long wave_min(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off);
    v = o < v ? o : v;
  }
  return v;
}

// Smallest key of one 8^3 block (512 threads, one voxel each), or ~0 when
// every voxel of the block is excluded or outside the valid box.
__device__ __forceinline__ unsigned long long block_min(const ttm_peak_item& it, const ItemGeo& g,
                                                        const unsigned* bits, int b, int t,
                                                        int nthreads) {
  const int bxx = b % g.bx, byy = (b / g.bx) % g.by, bzz = b / (g.bx * g.by);
  unsigned long long m = ~0ull;
  for (int i = t; i < kBlk * kBlk * kBlk; i += nthreads) {
    const int vx = bxx * kBlk + i % kBlk, vy = byy * kBlk + (i / kBlk) % kBlk,
              vz = bzz * kBlk + i / (kBlk * kBlk);
    if (vx < g.vx && vy < g.vy && vz < g.vz) {
      const unsigned long long k = voxel_key(it, g, bits, vz, vy, vx);
      m = k < m ? k : m;
    }
  }
  return m;
}

__global__ __launch_bounds__(512) void k_block_keys(const ttm_peak_item* __restrict__ items) {
  __shared__ unsigned long long red[8];
  const ttm_peak_item it = items[blockIdx.y];
  if (!item_ok(it)) return;
  const ItemGeo g = geo(it.valid_lo, it.valid_hi);
  const int b = blockIdx.x;
  if (b >= g.bz * g.by * g.bx) return;            // uniform per workgroup
  unsigned long long* keys;
  unsigned* bits;
  scratch_layout(it.scratch, g, &keys, &bits);
  unsigned long long m = block_min(it, g, bits, b, threadIdx.x, 512);
  m = wave_min(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long r = red[0];
    for (int i = 1; i < 8; ++i) r = red[i] < r ? red[i] : r;
    keys[b] = r;
  }
}

__global__ __launch_bounds__(256) void k_clear_bits(const ttm_peak_item* __restrict__ items) {
  const ttm_peak_item it = items[blockIdx.y];
  if (!item_ok(it)) return;
  const ItemGeo g = geo(it.valid_lo, it.valid_hi);
  unsigned long long* keys;
  unsigned* bits;
  scratch_layout(it.scratch, g, &keys, &bits);
  for (size_t w = (size_t)blockIdx.x * 256 + threadIdx.x; w < g.words; w += (size_t)gridDim.x * 256)
    bits[w] = 0u;
}

__global__ __launch_bounds__(kNmsThreads) void k_nms(const ttm_peak_item* __restrict__ items) {
  __shared__ unsigned long long red_k[kNmsThreads / 64];
  __shared__ unsigned long long s_best;
  const ttm_peak_item it = items[blockIdx.x];
  if (!item_ok(it)) {
    if (threadIdx.x == 0 && it.n_found) *it.n_found = -1;
    return;
  }
  const ItemGeo g = geo(it.valid_lo, it.valid_hi);
  unsigned long long* keys;
  unsigned* bits;
  scratch_layout(it.scratch, g, &keys, &bits);
  const int nb = g.bz * g.by * g.bx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float D = it.min_dist, D2 = D * D;
  const int R = (int)ceilf(D);
  const int P = it.top_p < kMaxBatchPeaks ? it.top_p : kMaxBatchPeaks;
  int found = 0;
  for (int p = 0; p < P; ++p) {
    // 1. the smallest block key: the next voxel in visiting order not excluded
    unsigned long long m = ~0ull;
    for (int b = threadIdx.x; b < nb; b += kNmsThreads) {
      const unsigned long long k = keys[b];
      m = k < m ? k : m;
    }
    m = wave_min(m);
    if (lane == 0) red_k[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long r = red_k[0];
      for (int i = 1; i < kNmsThreads / 64; ++i) r = red_k[i] < r ? red_k[i] : r;
      s_best = r;
    }
    __syncthreads();
    const unsigned long long best = s_best;
    if (best == ~0ull) break;                    // uniform: nothing left
    const unsigned lin = (unsigned)(best & 0xFFFFFFFFull);
    const int x = (int)(lin % (unsigned)it.dims[2]);
    const int y = (int)((lin / (unsigned)it.dims[2]) % (unsigned)it.dims[1]);
    const int z = (int)(lin / ((unsigned)it.dims[2] * (unsigned)it.dims[1]));
    if (threadIdx.x == 0) {
      it.peaks[3 * p] = z;
      it.peaks[3 * p + 1] = y;
      it.peaks[3 * p + 2] = x;
      it.vals[p] = it.score[lin];
    }
    ++found;
    // 2. exclude the ball: every (z, y) row of it is an x range of the bitmask
    const int vz0 = z - it.valid_lo[0], vy0 = y - it.valid_lo[1], vx0 = x - it.valid_lo[2];
    const int rows = (2 * R + 1) * (2 * R + 1);
    for (int rr = threadIdx.x; rr < rows; rr += kNmsThreads) {
      const int dz = rr / (2 * R + 1) - R, dy = rr % (2 * R + 1) - R;
      const int vz = vz0 + dz, vy = vy0 + dy;
      if (vz < 0 || vz >= g.vz || vy < 0 || vy >= g.vy) continue;
      const float rem = D2 - (float)(dz * dz + dy * dy);
      if (!(rem > 0.0f)) continue;
      // |dx| with dx^2 < rem
      int h = (int)sqrtf(rem);
      while ((float)(h * h) >= rem) --h;
      while ((float)((h + 1) * (h + 1)) < rem) ++h;
      const int xa = max(vx0 - h, 0), xb = min(vx0 + h, g.vx - 1);
      if (xa > xb) continue;
      const size_t base = ((size_t)vz * g.vy + vy) * g.vx;
      size_t i0 = base + xa;
      const size_t i1 = base + xb;
      while (i0 <= i1) {
        const size_t w = i0 >> 5;
        const unsigned s0 = (unsigned)(i0 & 31);
        const size_t wend = (w << 5) + 31;
        const unsigned s1 = (unsigned)((i1 < wend ? i1 : wend) & 31);
        const unsigned mask = (s1 == 31 ? 0xFFFFFFFFu : ((1u << (s1 + 1)) - 1u)) & ~((1u << s0) - 1u);
        atomicOr(&bits[w], mask);
        i0 = (w << 5) + 32;
      }
    }
    if (threadIdx.x == 0) {                      // the peak itself is visited (D = 0 too)
      const size_t vi = ((size_t)vz0 * g.vy + vy0) * g.vx + vx0;
      atomicOr(&bits[vi >> 5], 1u << (vi & 31));
    }
    __threadfence_block();
    __syncthreads();
    // 3. the keys of the blocks the ball touches, without the excluded voxels.
    // Exclusion only removes voxels, so a block whose smallest key belongs to
    // a voxel outside the ball keeps it; a block inside the ball is emptied;
    // only a block whose smallest-key voxel was just excluded is rescanned.
    const int bz0 = max(vz0 - R, 0) / kBlk, bz1 = min(vz0 + R, g.vz - 1) / kBlk;
    const int by0 = max(vy0 - R, 0) / kBlk, by1 = min(vy0 + R, g.vy - 1) / kBlk;
    const int bx0 = max(vx0 - R, 0) / kBlk, bx1 = min(vx0 + R, g.vx - 1) / kBlk;
    const int nbz = bz1 - bz0 + 1, nby = by1 - by0 + 1, nbx = bx1 - bx0 + 1;
    for (int q = wave; q < nbz * nby * nbx; q += kNmsThreads / 64) {
      const int qz = bz0 + q / (nby * nbx), qy = by0 + (q / nbx) % nby, qx = bx0 + q % nbx;
      const int b = (qz * g.by + qy) * g.bx + qx;
      const unsigned long long kb = keys[b];     // the same value in every lane
      if (kb == ~0ull) continue;                 // already empty
      // farthest corner of the block's valid part from the peak
      const int cz0 = qz * kBlk - vz0, cz1 = min(qz * kBlk + kBlk, g.vz) - 1 - vz0;
      const int cy0 = qy * kBlk - vy0, cy1 = min(qy * kBlk + kBlk, g.vy) - 1 - vy0;
      const int cx0 = qx * kBlk - vx0, cx1 = min(qx * kBlk + kBlk, g.vx) - 1 - vx0;
      const int fz = max(cz0 * cz0, cz1 * cz1), fy = max(cy0 * cy0, cy1 * cy1), fx = max(cx0 * cx0, cx1 * cx1);
      if ((float)(fz + fy + fx) < D2) {
        if (lane == 0) keys[b] = ~0ull;          // every voxel of the block is excluded
        continue;
      }
      const unsigned kl = (unsigned)(kb & 0xFFFFFFFFull);
      const int mx = (int)(kl % (unsigned)it.dims[2]) - x;
      const int my = (int)((kl / (unsigned)it.dims[2]) % (unsigned)it.dims[1]) - y;
      const int mz = (int)(kl / ((unsigned)it.dims[2] * (unsigned)it.dims[1])) - z;
      const bool gone = (mx | my | mz) == 0 || (float)(mx * mx + my * my + mz * mz) < D2;
      if (!gone) continue;                       // its smallest key is still there
      unsigned long long mm = block_min(it, g, bits, b, lane, 64);
      mm = wave_min(mm);
      if (lane == 0) keys[b] = mm;
    }
    __threadfence_block();
    __syncthreads();
  }
  if (threadIdx.x == 0) *it.n_found = found;
}

}  // namespace

size_t peaks_batch_scratch(const int32_t lo[3], const int32_t hi[3]) {
  const ItemGeo g = geo(lo, hi);
  return a256b((size_t)g.bz * g.by * g.bx * 8) + a256b(g.words * 4);
}

int peaks_batch_max_peaks() { return kMaxBatchPeaks; }

int find_peaks_batch(const ttm_peak_item* items, int n_items, const int32_t max_valid[3],
                     hipStream_t s) {
  const int32_t zero[3] = {0, 0, 0};
  const int32_t hi[3] = {max_valid[0] - 1, max_valid[1] - 1, max_valid[2] - 1};
  const ItemGeo g = geo(zero, hi);
  const int max_blocks = g.bz * g.by * g.bx;
  const size_t max_words = g.words;
  const unsigned cw = (unsigned)((max_words + 255) / 256);
  hipLaunchKernelGGL(k_clear_bits, dim3(cw < 4096 ? cw : 4096, n_items), dim3(256), 0, s, items);
  hipLaunchKernelGGL(k_block_keys, dim3(max_blocks, n_items), dim3(512), 0, s, items);
  hipLaunchKernelGGL(k_nms, dim3(n_items), dim3(kNmsThreads), 0, s, items);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : hip_status(e, "find peaks batch launch");
}

}  // namespace ttm
