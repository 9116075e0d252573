// peaks.hip -- exact greedy Find Peaks on the GPU (gfx950).
//
// The rule (Sec. 3.4): visit voxels by descending score, ties by ascending
// linear index, keep a voxel when every kept peak is at least D away, stop
// at P.  A voxel's fate depends only on higher-ranked voxels, so the first P
// kept peaks are decided by the voxels ranked above the P-th of them.  The
// search therefore runs on the top-ranked candidates only:
//   1. 16-bit histogram of the score bit patterns (scores are >= 0, so the
//      bit pattern is monotone in the value),
//   2. the host picks the histogram bin above which at least `want`
//      candidates lie and the kernels compact them as 64-bit keys
//      (~score_bits << 32 | linear index), so ascending key order is exactly
//      the visiting order,
//   3. LSD radix sort of the keys (8-bit digits, stable ranks from wavefront
//      ballots),
//   4. one workgroup walks the sorted keys in chunks of 1024: every lane
//      tests its candidate against the kept peaks through a spatial hash of
//      cell size D; the survivors, compacted in rank order, are settled 64 at
//      a time by one wavefront (pairwise conflict bitmasks, then a 64-step
//      in-order acceptance on those masks).
// If fewer than P peaks are found while lower-ranked voxels remain, the host
// doubles `want` and repeats.
#include <climits>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace ttm {

size_t peaks_workspace(int64_t n_voxels);

namespace {

constexpr int kHistBins = 4096;   // per level: bits [31:20], then [19:8]
constexpr int kSortIPT = 16;           // keys per thread per sort block
constexpr int kSortBlock = 256;        // threads per sort block
constexpr int kSortTile = kSortIPT * kSortBlock;

__device__ __forceinline__ unsigned score_bits(float s) {
  // scores are norms (>= 0); clamp anything else to 0 so the order is monotone
  return (s > 0.0f) ? __float_as_uint(s) : 0u;
}

struct Region {
  int nz, ny, nx;
  int z0, y0, x0, z1, y1, x1;  // inclusive valid box
};

// Histogram of one 12-bit field of the score bit patterns over the region,
// privatised in LDS per workgroup.  level 0: bits [31:20] of every voxel;
// level 1: bits [19:8] of the voxels whose bits [31:20] equal `top`.
// Each workgroup covers kHistRows rows (y) of one z slice, in groups of 8, so
// clearing and flushing its 16 KB of bins is spread over enough voxels.
constexpr int kHistRows = 32;
__global__ __launch_bounds__(256) void k_hist(const float* __restrict__ score, Region r, int level,
                                              unsigned top, unsigned* __restrict__ hist) {
  __shared__ unsigned h[kHistBins];
  for (int i = threadIdx.x; i < kHistBins; i += 256) h[i] = 0;
  __syncthreads();
  const int z = r.z0 + blockIdx.z;
  const int nxv = r.x1 - r.x0 + 1;
  // scores crowd into few bins: a thread counts a run of equal bins in a
  // register and adds it at once, instead of one contended LDS atomic each.
  // A thread takes one column x of 8 rows at a time, its 8 loads in flight
  // together.
  unsigned cur = 0xFFFFFFFFu, run = 0;
  for (int y8 = r.y0 + (int)blockIdx.y * kHistRows;
       y8 < min(r.y0 + ((int)blockIdx.y + 1) * kHistRows, r.y1 + 1); y8 += 8) {
    const int nyv = min(8, r.y1 - y8 + 1);
    const float* col0 = score + ((size_t)z * r.ny + y8) * r.nx + r.x0;
    for (int x = blockIdx.x * 256 + threadIdx.x; x < nxv; x += 256 * gridDim.x) {
      float v[8];
#pragma unroll
      for (int yy = 0; yy < 8; ++yy) v[yy] = yy < nyv ? col0[(size_t)yy * r.nx + x] : 0.0f;
#pragma unroll
      for (int yy = 0; yy < 8; ++yy) {
        if (yy >= nyv) break;
        const unsigned b = score_bits(v[yy]);
        unsigned bin = 0xFFFFFFFFu;
        if (level == 0) {
          bin = b >> 20;
        } else if ((b >> 20) == top) {
          bin = (b >> 8) & 0xFFFu;
        }
        if (bin == 0xFFFFFFFFu) continue;
        if (bin != cur) {
          if (run) atomicAdd(&h[cur], run);
          cur = bin;
          run = 0;
        }
        ++run;
      }
    }
  }
  if (run) atomicAdd(&h[cur], run);
  __syncthreads();
  for (int i = threadIdx.x; i < kHistBins; i += 256)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Keys of the voxels whose score bits are >= key_lo, in any order (they are
// sorted next).  A workgroup takes kCompactRows rows of one z slice and 1024
// columns of each, 4 loads per thread in flight; a wavefront reserves the
// slots of all its keys with one atomic.
constexpr int kCompactRows = 4;
__global__ __launch_bounds__(256) void k_compact(const float* __restrict__ score, Region r,
                                                 unsigned key_lo,
                                                 unsigned long long* __restrict__ keys,
                                                 unsigned* __restrict__ counter) {
  const int z = r.z0 + blockIdx.z, y0 = r.y0 + blockIdx.y * kCompactRows;
  const int xb = r.x0 + blockIdx.x * 1024 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const int nrows = min(kCompactRows, r.y1 - y0 + 1);
  for (int yy = 0; yy < nrows; ++yy) {
    const size_t row = ((size_t)z * r.ny + y0 + yy) * r.nx;
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = xb + 256 * k <= r.x1 ? score[row + xb + 256 * k] : 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int x = xb + 256 * k;
      const unsigned bits = score_bits(v[k]);
      const bool take = x <= r.x1 && bits >= key_lo;
      const unsigned long long bal = __ballot(take);
      if (bal == 0ull) continue;  // uniform across the wavefront
      const int leader = __ffsll((long long)bal) - 1;
      unsigned base = 0;
      if (lane == leader) base = atomicAdd(counter, (unsigned)__popcll(bal));
      base = (unsigned)__shfl((int)base, leader);
      if (take)
        keys[base + __popcll(bal & lt)] = ((unsigned long long)(~bits) << 32) |
                                          (unsigned long long)(row + x);
    }
  }
}

__global__ void k_fill(unsigned long long* __restrict__ keys, size_t from, size_t to) {
  const size_t i = from + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < to) keys[i] = ~0ull;
}

// ---------------------------------------------------------------- radix sort
__global__ __launch_bounds__(kSortBlock) void k_rs_hist(const unsigned long long* __restrict__ keys,
                                                        int shift, unsigned* __restrict__ hist,
                                                        int nblocks) {
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kSortTile;
  for (int i = 0; i < kSortIPT; ++i) {
    const unsigned d = (unsigned)(keys[base + i * kSortBlock + threadIdx.x] >> shift) & 255u;
    atomicAdd(&h[d], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of n values by one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void k_scan(unsigned* __restrict__ a, int n) {
  __shared__ unsigned part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  // each thread's segment in batches of 8 loads in flight
  unsigned s = 0;
  int i = lo;
  for (; i + 8 <= hi; i += 8) {
    unsigned v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = a[i + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  for (; i < hi; ++i) s += a[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    unsigned v = (t >= off) ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned run = (t == 0) ? 0u : part[t - 1];
  for (i = lo; i + 8 <= hi; i += 8) {
    unsigned v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = a[i + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a[i + k] = run;
      run += v[k];
    }
  }
  for (; i < hi; ++i) {
    const unsigned v = a[i];
    a[i] = run;
    run += v;
  }
}

__global__ __launch_bounds__(kSortBlock) void k_rs_scatter(
    const unsigned long long* __restrict__ in, unsigned long long* __restrict__ out, int shift,
    const unsigned* __restrict__ offs, int nblocks) {
  constexpr int NW = kSortBlock / 64;
  __shared__ unsigned run[256];
  __shared__ unsigned wcnt[NW][256];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  run[tid] = offs[(size_t)tid * nblocks + blockIdx.x];
  const size_t base = (size_t)blockIdx.x * kSortTile;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int i = 0; i < kSortIPT; ++i) {
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const unsigned long long key = in[base + i * kSortBlock + tid];
    const unsigned d = (unsigned)(key >> shift) & 255u;
    unsigned long long same = ~0ull;
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const unsigned long long bal = __ballot((d >> bit) & 1u);
      same &= ((d >> bit) & 1u) ? bal : ~bal;
    }
    const unsigned rank = __popcll(same & lt);
    if (rank == 0) wcnt[wv][d] = __popcll(same);
    __syncthreads();
    unsigned before = 0;
    for (int w = 0; w < wv; ++w) before += wcnt[w][d];
    out[run[d] + before + rank] = key;
    __syncthreads();
    unsigned tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += wcnt[w][tid];
    run[tid] += tot;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- greedy walk
constexpr int kGreedyThreads = 1024;
constexpr int kMaxPeaks = 2048;
constexpr int kMaxCells = 16384;

// The kept peaks' spatial hash as the greedy leaves it in global memory for
// the filter and for the next walk: head[kMaxCells], then next, pz, py, px
// (kMaxPeaks each), all 16-bit.
constexpr int kHashShorts = kMaxCells + 4 * kMaxPeaks;

struct GreedyArgs {
  const unsigned long long* keys;
  int m;                  // number of candidate keys (sorted ascending)
  const int* m_dev;       // if set, the number of keys is read here instead
  int limit;              // walk at most this many keys (a multiple of the chunk)
  int resume;             // 1: continue from the peaks (and hash) already kept
  int nz, ny, nx;
  float d2;               // squared exclusion distance
  float cell;             // hash cell edge (>= exclusion distance)
  int gz, gy, gx;         // hash grid extent
  int top_p;
  int* peaks;             // top_p x 3
  float* vals;
  int* n_found;           // device
  short* hash;            // kHashShorts, device
};

// Candidates per thread and chunk.  More than one lets a thread issue its
// hash lookups together and a chunk's barriers serve more keys, but then more
// keys reach the serial settle before the hash learns of the peaks kept in
// their chunk; with many peaks (thousands at 2r apart) one per thread is
// faster.
constexpr int kGreedyPer = 1;
constexpr int kGreedyChunk = kGreedyThreads * kGreedyPer;

__global__ __launch_bounds__(kGreedyThreads) void k_greedy(GreedyArgs g) {
  constexpr int NW = kGreedyThreads / 64;
  __shared__ short head[kMaxCells];
  __shared__ short next[kMaxPeaks];
  __shared__ short pz[kMaxPeaks], py[kMaxPeaks], px[kMaxPeaks];
  __shared__ short sz[kGreedyChunk], sy[kGreedyChunk], sx[kGreedyChunk];
  __shared__ int srank[kGreedyChunk];   // rank within the chunk of each survivor
  __shared__ int wsum[kGreedyPer * NW];
  __shared__ int nkept, stop, mlen;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ncell = g.gz * g.gy * g.gx;
  short* gnext = g.hash + kMaxCells;
  short* gpz = gnext + kMaxPeaks;
  short* gpy = gpz + kMaxPeaks;
  short* gpx = gpy + kMaxPeaks;
  if (tid == 0) {
    nkept = g.resume ? *g.n_found : 0;
    stop = nkept >= g.top_p ? 1 : 0;
    mlen = g.m_dev ? *g.m_dev : g.m;
  }
  __syncthreads();
  if (stop) return;  // uniform: the peaks are complete
  if (g.resume) {
    for (int i = tid; i < ncell; i += kGreedyThreads) head[i] = g.hash[i];
    for (int k = tid; k < nkept; k += kGreedyThreads) {
      next[k] = gnext[k];
      pz[k] = gpz[k];
      py[k] = gpy[k];
      px[k] = gpx[k];
    }
  } else {
    for (int i = tid; i < ncell; i += kGreedyThreads) head[i] = (short)-1;
  }
  __syncthreads();
  const int mm = min(mlen, g.limit);
  // linear indices fit the key's low 32 bits and ny * nx < 2^30 (edges are
  // below 2^15), so the decode divides in 32 bits
  const unsigned yx = (unsigned)g.ny * (unsigned)g.nx, nxu = (unsigned)g.nx;
  const unsigned long long lt = (1ull << lane) - 1ull;
  // candidate k of a thread in a chunk has rank k * kGreedyThreads + tid; its
  // key is loaded one chunk ahead
  unsigned long long key_next[kGreedyPer];
#pragma unroll
  for (int k = 0; k < kGreedyPer; ++k) {
    const int i = k * kGreedyThreads + tid;
    key_next[k] = i < mm ? g.keys[i] : 0ull;
  }
  for (int base = 0; base < mm; base += kGreedyChunk) {
    int cz[kGreedyPer], cy[kGreedyPer], cxx[kGreedyPer], hz[kGreedyPer], hy[kGreedyPer],
        hx[kGreedyPer];
    bool alive[kGreedyPer];
#pragma unroll
    for (int k = 0; k < kGreedyPer; ++k) {
      const int idx = base + k * kGreedyThreads + tid;
      alive[k] = idx < mm;
      const unsigned lin = (unsigned)(key_next[k] & 0xffffffffull);
      const unsigned qz = lin / yx, rz = lin - qz * yx, qy = rz / nxu;
      cz[k] = alive[k] ? (int)qz : 0;
      cy[k] = alive[k] ? (int)qy : 0;
      cxx[k] = alive[k] ? (int)(rz - qy * nxu) : 0;
      hz[k] = (int)(cz[k] / g.cell);
      hy[k] = (int)(cy[k] / g.cell);
      hx[k] = (int)(cxx[k] / g.cell);
      if (idx + kGreedyChunk < mm) key_next[k] = g.keys[idx + kGreedyChunk];
    }
    // a candidate dies when a peak kept in an earlier chunk lies within D;
    // such a peak sits in one of the 27 hash cells around the candidate's
    for (int c = 0; c < 27; ++c) {
      bool any = false;
#pragma unroll
      for (int k = 0; k < kGreedyPer; ++k) any = any || alive[k];
      if (!any) break;
      const int dz = c / 9 - 1, dy = (c / 3) % 3 - 1, dx = c % 3 - 1;
      int p[kGreedyPer];
#pragma unroll
      for (int k = 0; k < kGreedyPer; ++k) {
        const int z2 = hz[k] + dz, y2 = hy[k] + dy, x2 = hx[k] + dx;
        const bool in = alive[k] && z2 >= 0 && z2 < g.gz && y2 >= 0 && y2 < g.gy && x2 >= 0 &&
                        x2 < g.gx;
        p[k] = in ? head[(z2 * g.gy + y2) * g.gx + x2] : -1;
      }
#pragma unroll
      for (int k = 0; k < kGreedyPer; ++k) {
        for (int q = p[k]; q >= 0; q = next[q]) {
          const float ddz = (float)(cz[k] - pz[q]), ddy = (float)(cy[k] - py[q]),
                      ddx = (float)(cxx[k] - px[q]);
          if (ddz * ddz + ddy * ddy + ddx * ddx < g.d2) {
            alive[k] = false;
            break;
          }
        }
      }
    }
    // survivors in rank order (k, then thread): wavefront ballots, then the
    // offsets of the sub-chunks and waves ahead
    unsigned long long bal[kGreedyPer];
#pragma unroll
    for (int k = 0; k < kGreedyPer; ++k) {
      bal[k] = __ballot(alive[k]);
      if (lane == 0) wsum[k * NW + wv] = __popcll(bal[k]);
    }
    __syncthreads();
    int ns = 0;
#pragma unroll
    for (int k = 0; k < kGreedyPer; ++k) {
      int before = 0, tot = 0;
      for (int w = 0; w < NW; ++w) {
        const int v = wsum[k * NW + w];
        before += w < wv ? v : 0;
        tot += v;
      }
      if (alive[k]) {
        const int pos = ns + before + __popcll(bal[k] & lt);
        sz[pos] = (short)cz[k];
        sy[pos] = (short)cy[k];
        sx[pos] = (short)cxx[k];
        srank[pos] = k * kGreedyThreads + tid;
      }
      ns += tot;
    }
    __syncthreads();
    // settle the survivors in order, 64 at a time on wavefront 0: a survivor
    // is kept when no peak kept earlier in this chunk and no kept survivor
    // ahead of it in its group lies within D
    if (wv == 0) {
      const int first_new = nkept;
      for (int g0 = 0; g0 < ns; g0 += 64) {
        if (nkept >= g.top_p) break;
        const int i = g0 + lane;
        bool cand = i < ns;
        int z = 0, y = 0, x = 0;
        if (cand) {
          z = sz[i];
          y = sy[i];
          x = sx[i];
          for (int p = first_new; p < nkept && cand; ++p) {
            const float ddz = (float)(z - pz[p]), ddy = (float)(y - py[p]), ddx = (float)(x - px[p]);
            if (ddz * ddz + ddy * ddy + ddx * ddx < g.d2) cand = false;
          }
        }
        // conflicts with the group's survivors ahead of this one, whose
        // coordinates are read from the lanes that hold them (gn and j are
        // the same on every lane, so these are plain lane reads)
        const int gn = min(64, ns - g0);
        unsigned long long conf = 0;
        for (int j = 0; j < gn; ++j) {
          const int zj = __builtin_amdgcn_readlane(z, j), yj = __builtin_amdgcn_readlane(y, j),
                    xj = __builtin_amdgcn_readlane(x, j);
          const float ddz = (float)(z - zj), ddy = (float)(y - yj), ddx = (float)(x - xj);
          if (j < lane && ddz * ddz + ddy * ddy + ddx * ddx < g.d2) conf |= 1ull << j;
        }
        const unsigned long long cands = __ballot(cand);
        const unsigned conf_lo = (unsigned)conf, conf_hi = (unsigned)(conf >> 32);
        unsigned long long kept = 0;
        int room = g.top_p - nkept;
        for (int l = 0; l < gn && room > 0; ++l) {
          const unsigned long long cl =
              ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)conf_hi, l) << 32) |
              (unsigned)__builtin_amdgcn_readlane((int)conf_lo, l);
          if (((cands >> l) & 1ull) && !(cl & kept)) {
            kept |= 1ull << l;
            --room;
          }
        }
        if ((kept >> lane) & 1ull) {
          const int k = nkept + __popcll(kept & ((1ull << lane) - 1ull));
          pz[k] = (short)z;
          py[k] = (short)y;
          px[k] = (short)x;
          const unsigned long long key = g.keys[base + srank[i]];
          g.peaks[3 * k + 0] = z;
          g.peaks[3 * k + 1] = y;
          g.peaks[3 * k + 2] = x;
          g.vals[k] = __uint_as_float(~(unsigned)(key >> 32));
        }
        wave_lds_sync();
        if (lane == 0) {
          // hash insertion in rank order
          const int nk = __popcll(kept);
          for (int t = 0; t < nk; ++t) {
            const int k = nkept + t;
            const int cell =
                ((int)(pz[k] / g.cell) * g.gy + (int)(py[k] / g.cell)) * g.gx + (int)(px[k] / g.cell);
            next[k] = head[cell];
            head[cell] = (short)k;
          }
          nkept += nk;
          if (nkept >= g.top_p) stop = 1;
        }
        wave_lds_sync();
      }
    }
    __syncthreads();
    if (stop) break;
  }
  // the hash and the count for the filter and the next walk
  const int nk = nkept;
  for (int i = tid; i < ncell; i += kGreedyThreads) g.hash[i] = head[i];
  for (int k = tid; k < nk; k += kGreedyThreads) {
    gnext[k] = next[k];
    gpz[k] = pz[k];
    gpy[k] = py[k];
    gpx[k] = px[k];
  }
  if (tid == 0) *g.n_found = nk;
}

// ---------------------------------------------------------------- filter
// Between two walks the rest of the sorted list is filtered on the whole
// GPU: a key dies when a peak kept so far lies within D (it could never be
// kept later, and only kept peaks decide anything), and the survivors are
// written in their order.  k_filter<false> counts the survivors of each
// block of kSortTile keys, k_scan turns the counts into offsets (the extra
// last entry becomes the total), k_filter<true> writes the survivors and the
// new list length.
struct FilterArgs {
  const unsigned long long* keys;
  int from;               // first key to filter (the walk took the keys before)
  int m;                  // list length, or
  const int* m_dev;       // read here when set
  int ny, nx;
  float d2, cell;
  int gz, gy, gx;
  int top_p;
  const int* n_found;
  const short* hash;      // as the greedy leaves it
  unsigned* counts;       // nb + 1 entries
  int nb;
  unsigned long long* out;
  int* m_next;
};

template <bool SCATTER>
__global__ __launch_bounds__(kSortBlock) void k_filter(FilterArgs f) {
  constexpr int NW = kSortBlock / 64;
  __shared__ short head[kMaxCells];
  __shared__ short next[kMaxPeaks], pz[kMaxPeaks], py[kMaxPeaks], px[kMaxPeaks];
  __shared__ unsigned wcnt[kSortIPT][NW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int np = *f.n_found;
  const int m = f.m_dev ? *f.m_dev : f.m;
  const bool done = np >= f.top_p;
  const int base = f.from + (int)blockIdx.x * kSortTile;
  if (blockIdx.x == 0 && tid == 0) {
    if (SCATTER) {
      *f.m_next = done ? 0 : (int)f.counts[f.nb];
    } else {
      f.counts[f.nb] = 0u;
    }
  }
  if (done || base >= m) {  // uniform per workgroup
    if (!SCATTER && tid == 0) f.counts[blockIdx.x] = 0u;
    return;
  }
  const int ncell = f.gz * f.gy * f.gx;
  for (int i = tid; i < ncell; i += kSortBlock) head[i] = f.hash[i];
  for (int k = tid; k < np; k += kSortBlock) {
    next[k] = f.hash[kMaxCells + k];
    pz[k] = f.hash[kMaxCells + kMaxPeaks + k];
    py[k] = f.hash[kMaxCells + 2 * kMaxPeaks + k];
    px[k] = f.hash[kMaxCells + 3 * kMaxPeaks + k];
  }
  __syncthreads();
  const unsigned yx = (unsigned)f.ny * (unsigned)f.nx, nxu = (unsigned)f.nx;
  unsigned long long key[kSortIPT];
  bool alive[kSortIPT];
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    const int i = base + j * kSortBlock + tid;
    alive[j] = i < m;
    key[j] = alive[j] ? f.keys[i] : 0ull;
  }
  for (int j = 0; j < kSortIPT; ++j) {
    if (!alive[j]) continue;
    const unsigned lin = (unsigned)(key[j] & 0xffffffffull);
    const unsigned qz = lin / yx, rz = lin - qz * yx, qy = rz / nxu;
    const int cz = (int)qz, cy = (int)qy, cxx = (int)(rz - qy * nxu);
    const int hz = (int)(cz / f.cell), hy = (int)(cy / f.cell), hx = (int)(cxx / f.cell);
    bool al = true;
    for (int c = 0; c < 27 && al; ++c) {
      const int z2 = hz + c / 9 - 1, y2 = hy + (c / 3) % 3 - 1, x2 = hx + c % 3 - 1;
      if (z2 < 0 || z2 >= f.gz || y2 < 0 || y2 >= f.gy || x2 < 0 || x2 >= f.gx) continue;
      for (int q = head[(z2 * f.gy + y2) * f.gx + x2]; q >= 0; q = next[q]) {
        const float ddz = (float)(cz - pz[q]), ddy = (float)(cy - py[q]), ddx = (float)(cxx - px[q]);
        if (ddz * ddz + ddy * ddy + ddx * ddx < f.d2) {
          al = false;
          break;
        }
      }
    }
    alive[j] = al;
  }
  // survivors of each slice j, per wavefront; ranks follow (j, thread)
  unsigned long long bal[kSortIPT];
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    bal[j] = __ballot(alive[j]);
    if (lane == 0) wcnt[j][wv] = __popcll(bal[j]);
  }
  __syncthreads();
  if (!SCATTER) {
    if (tid == 0) {
      unsigned t = 0;
      for (int j = 0; j < kSortIPT; ++j)
        for (int w = 0; w < NW; ++w) t += wcnt[j][w];
      f.counts[blockIdx.x] = t;
    }
    return;
  }
  unsigned run = f.counts[blockIdx.x];
  const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    unsigned before = 0, tot = 0;
    for (int w = 0; w < NW; ++w) {
      const unsigned v = wcnt[j][w];
      before += w < wv ? v : 0u;
      tot += v;
    }
    if (alive[j]) f.out[run + before + __popcll(bal[j] & lt)] = key[j];
    run += tot;
  }
}

// Index bytes of the keys (their low 32 bits) that are zero for every linear
// index of the map need no radix pass: the pass would keep the order.  The
// padding keys (all ones) still sort after every real key, because the real
// keys' index bytes that are sorted already stay below theirs or, at equality,
// stable passes keep the real keys (placed first) ahead.
bool index_byte_constant(int shift, const Region& r) {
  const unsigned long long total = (unsigned long long)r.nz * r.ny * r.nx;
  return shift < 32 && total <= (1ull << shift);
}

constexpr int kWalkRounds = 3;                // short walks, each followed by a filter
constexpr int kWalkKeys = 8 * kGreedyChunk;    // keys per short walk

// Bytes of the workspace before its tail (keys, histograms, counters,
// sort counts), and the tail: the kept peaks' hash and the list lengths.
size_t peaks_head_bytes(int64_t n_voxels) {
  const size_t cand = (size_t)n_voxels + kSortTile;
  const size_t nblk = (cand + kSortTile - 1) / kSortTile;
  const size_t b = 2 * cand * 8 + kHistBins * 4 + 256 * nblk * 4 + 256 + 1024;
  return (b + 255) / 256 * 256;
}
constexpr size_t kPeaksTailBytes = kHashShorts * 2 + 256;

// The greedy walk over m sorted keys in `srt` (`spare` holds as many):
// `rounds` times a walk over the first kWalkKeys keys of the list and the
// filter of the rest into the other buffer, then a walk over what is left.
// The result equals one walk over all m keys: a filtered key was within D of
// a peak kept before it, and the survivors keep their order.  The rounds pay
// when most keys die (every voxel a candidate, few peaks); over the top
// candidates alone one walk is as fast.
void greedy_walks(unsigned long long* srt, unsigned long long* spare, size_t m, const Region& r,
                  float min_dist, float cell, int gz, int gy, int gx, int top_p, int32_t* peaks,
                  float* vals, int32_t* n_found, unsigned* counts, char* tail, int rounds,
                  hipStream_t s) {
  short* hash = reinterpret_cast<short*>(tail);
  int* mdev = reinterpret_cast<int*>(tail + kHashShorts * 2);
  const int nb = m > (size_t)kWalkKeys ? (int)((m - kWalkKeys + kSortTile - 1) / kSortTile) : 0;
  unsigned long long* cur = srt;
  unsigned long long* other = spare;
  const int* mcur = nullptr;
  const float d2 = min_dist * min_dist;
  for (int round = 0;; ++round) {
    const bool last = round == rounds || nb == 0;
    GreedyArgs ga{cur, (int)m, mcur, last ? INT_MAX : kWalkKeys, round > 0 ? 1 : 0, r.nz, r.ny,
                  r.nx, d2, cell, gz, gy, gx, top_p, peaks, vals, n_found, hash};
    hipLaunchKernelGGL(k_greedy, dim3(1), dim3(kGreedyThreads), 0, s, ga);
    if (last) break;
    FilterArgs fa{cur, kWalkKeys, (int)m, mcur, r.ny, r.nx, d2, cell, gz, gy, gx, top_p, n_found,
                  hash, counts, nb, other, mdev + round};
    hipLaunchKernelGGL(k_filter<false>, dim3(nb), dim3(kSortBlock), 0, s, fa);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, nb + 1);
    hipLaunchKernelGGL(k_filter<true>, dim3(nb), dim3(kSortBlock), 0, s, fa);
    mcur = mdev + round;
    std::swap(cur, other);
  }
}

}  // namespace

// Exact Find Peaks with every valid voxel as a candidate and no host
// synchronisation (the count stays on the device), for graph capture.
int find_peaks_async(const float* score, int nz, int ny, int nx, const int32_t lo[3],
                     const int32_t hi[3], int top_p, float min_dist, int32_t* peaks_out,
                     float* vals_out, int32_t* n_found_dev, void* ws, size_t ws_bytes,
                     hipStream_t s) {
  Region r{nz, ny, nx, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
  const int64_t nvalid = (int64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
  const size_t need = peaks_workspace(nvalid);
  if (ws_bytes < need) {
    set_error("ttm_find_peaks_async: workspace %zu < %zu bytes", ws_bytes, need);
    return -5;
  }
  const float cell = fmaxf(min_dist, 1.0f);
  const int gz = (int)(nz / cell) + 1, gy = (int)(ny / cell) + 1, gx = (int)(nx / cell) + 1;
  if ((int64_t)gz * gy * gx > kMaxCells || top_p > kMaxPeaks || nz > 32767 || ny > 32767 ||
      nx > 32767) {
    set_error("ttm_find_peaks_async: exclusion grid %dx%dx%d or top_p %d too large", gz, gy, gx,
              top_p);
    return -4;
  }
  char* w = static_cast<char*>(ws);
  const size_t cand_cap = (size_t)nvalid + kSortTile;
  unsigned long long* keys_a = reinterpret_cast<unsigned long long*>(w);
  unsigned long long* keys_b = keys_a + cand_cap;
  unsigned* hist = reinterpret_cast<unsigned*>(keys_b + cand_cap);
  unsigned* counter = hist + kHistBins;
  unsigned* shist = reinterpret_cast<unsigned*>(counter + 128);
  const dim3 cgrid((hi[2] - lo[2] + 1 + 1023) / 1024, (hi[1] - lo[1] + kCompactRows) / kCompactRows,
                   hi[0] - lo[0] + 1);
  const size_t m = (size_t)nvalid;
  const size_t mpad = (m + kSortTile - 1) / kSortTile * kSortTile;
  const int nblk = (int)(mpad / kSortTile);
  fill_zero(counter, 4, s);
  hipLaunchKernelGGL(k_compact, cgrid, dim3(256), 0, s, score, r, 0u, keys_a, counter);
  if (mpad > m) {
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((mpad - m + 255) / 256)), dim3(256), 0, s, keys_a, m,
                       mpad);
  }
  unsigned long long* src = keys_a;
  unsigned long long* dst = keys_b;
  for (int shift = 0; shift < 64; shift += 8) {
    if (index_byte_constant(shift, r)) continue;
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kSortBlock), 0, s, src, shift, shist, nblk);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, shist, 256 * nblk);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kSortBlock), 0, s, src, dst, shift, shist,
                       nblk);
    std::swap(src, dst);
  }
  greedy_walks(src, dst, m, r, min_dist, cell, gz, gy, gx, top_p, peaks_out, vals_out,
               n_found_dev, shist, w + peaks_head_bytes(nvalid), kWalkRounds, s);
  TTM_HIP(hipGetLastError());
  return 0;
}

size_t peaks_workspace(int64_t n_voxels) {
  return peaks_head_bytes(n_voxels) + kPeaksTailBytes;
}

int find_peaks(const float* score, int nz, int ny, int nx, const int32_t lo[3],
               const int32_t hi[3], int top_p, float min_dist, int32_t* peaks_out,
               float* vals_out, int32_t* n_found_host, void* ws, size_t ws_bytes,
               hipStream_t s) {
  Region r{nz, ny, nx, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
  const int64_t nvalid = (int64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
  const size_t need = peaks_workspace(nvalid);
  if (ws_bytes < need) {
    set_error("ttm_find_peaks: workspace %zu < %zu bytes", ws_bytes, need);
    return -5;
  }
  const float cell = fmaxf(min_dist, 1.0f);
  const int gz = (int)(nz / cell) + 1, gy = (int)(ny / cell) + 1, gx = (int)(nx / cell) + 1;
  if ((int64_t)gz * gy * gx > kMaxCells || top_p > kMaxPeaks || nz > 32767 || ny > 32767 ||
      nx > 32767) {
    set_error("ttm_find_peaks: exclusion grid %dx%dx%d or top_p %d too large", gz, gy, gx, top_p);
    return -4;
  }
  char* w = static_cast<char*>(ws);
  const size_t cand_cap = (size_t)nvalid + kSortTile;
  unsigned long long* keys_a = reinterpret_cast<unsigned long long*>(w);
  unsigned long long* keys_b = keys_a + cand_cap;
  unsigned* hist = reinterpret_cast<unsigned*>(keys_b + cand_cap);
  unsigned* counter = hist + kHistBins;
  int* nfound_dev = reinterpret_cast<int*>(counter + 64);
  unsigned* shist = reinterpret_cast<unsigned*>(nfound_dev + 64);

  const dim3 cgrid((hi[2] - lo[2] + 1 + 1023) / 1024, (hi[1] - lo[1] + kCompactRows) / kCompactRows,
                   hi[0] - lo[0] + 1);
  const dim3 hgrid(1, (hi[1] - lo[1] + kHistRows) / kHistRows, hi[0] - lo[0] + 1);
  std::vector<unsigned> h0(kHistBins), h1(kHistBins);
  fill_zero(hist, kHistBins * 4, s);
  hipLaunchKernelGGL(k_hist, hgrid, dim3(256), 0, s, score, r, 0, 0u, hist);
  TTM_HIP(hipMemcpyAsync(h0.data(), hist, kHistBins * 4, hipMemcpyDeviceToHost, s));
  TTM_HIP(hipStreamSynchronize(s));
  int top_cached = -1;

  int64_t want = std::max<int64_t>(64 * (int64_t)top_p, 1 << 16);
  while (true) {
    // coarse bin (bits 31:20) such that it and the bins above hold >= want voxels
    int64_t above = 0;
    int b0 = kHistBins - 1;
    for (; b0 >= 0; --b0) {
      if (above + h0[b0] >= want) break;
      above += h0[b0];
    }
    unsigned key_lo = 0;
    int64_t acc = 0;
    if (b0 < 0) {
      key_lo = 0;             // every voxel
      acc = above;
    } else {
      if (top_cached != b0) {
        fill_zero(hist, kHistBins * 4, s);
        hipLaunchKernelGGL(k_hist, hgrid, dim3(256), 0, s, score, r, 1, (unsigned)b0, hist);
        TTM_HIP(hipMemcpyAsync(h1.data(), hist, kHistBins * 4, hipMemcpyDeviceToHost, s));
        TTM_HIP(hipStreamSynchronize(s));
        top_cached = b0;
      }
      int64_t in = 0;
      int b1 = kHistBins - 1;
      for (; b1 > 0; --b1) {
        if (above + in + h1[b1] >= want) break;
        in += h1[b1];
      }
      in += h1[b1];
      key_lo = ((unsigned)b0 << 20) | ((unsigned)b1 << 8);
      acc = above + in;
    }
    const bool all = (acc >= nvalid) || key_lo == 0;
    const int64_t m = acc;
    const size_t mpad = ((size_t)m + kSortTile - 1) / kSortTile * kSortTile;
    const int nblk = (int)(mpad / kSortTile);
    fill_zero(counter, 4, s);
    hipLaunchKernelGGL(k_compact, cgrid, dim3(256), 0, s, score, r, key_lo, keys_a, counter);
    if (mpad > (size_t)m) {
      hipLaunchKernelGGL(k_fill, dim3((unsigned)((mpad - m + 255) / 256)), dim3(256), 0, s, keys_a,
                         (size_t)m, mpad);
    }
    unsigned long long* src = keys_a;
    unsigned long long* dst = keys_b;
    for (int shift = 0; shift < 64; shift += 8) {
      if (index_byte_constant(shift, r)) continue;
      hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kSortBlock), 0, s, src, shift, shist, nblk);
      hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, shist, 256 * nblk);
      hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kSortBlock), 0, s, src, dst, shift, shist,
                         nblk);
      std::swap(src, dst);
    }
    greedy_walks(src, dst, (size_t)m, r, min_dist, cell, gz, gy, gx, top_p, peaks_out, vals_out,
                 nfound_dev, shist, w + peaks_head_bytes(nvalid), 0, s);
    TTM_HIP(hipGetLastError());
    int nf = 0;
    TTM_HIP(hipMemcpyAsync(&nf, nfound_dev, 4, hipMemcpyDeviceToHost, s));
    TTM_HIP(hipStreamSynchronize(s));
    if (nf >= top_p || all) {
      *n_found_host = nf;
      return 0;
    }
    want *= 4;
  }
}

}  // namespace ttm
