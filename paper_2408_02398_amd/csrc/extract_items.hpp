// extract_items.hpp -- where a voxel of an extraction call reads its tensor
// field and writes its answer, for one box or a batch of boxes (shared by the
// axis-form and quaternion-form extraction kernels).
#pragma once

#include "internal.hpp"

namespace ttm {

// Output-map index of voxel v of a single-box call: the box voxel (z, y, x)
// lands at (oz + z, oy + y, ox + x) of a dz x dy x dx map (only dy, dx enter).
__device__ __forceinline__ size_t box_map_index(const ExtractArgs& a, size_t v) {
  const int vx = (int)(v % a.bx), vy = (int)((v / a.bx) % a.by), vz = (int)(v / ((size_t)a.bx * a.by));
  return ((size_t)(a.oz + vz) * a.dy + (a.oy + vy)) * a.dx + (a.ox + vx);
}

// The single box, or in a batched call the item holding v (the last whose
// first voxel is <= v, by binary search over the items' first voxels), with
// v's place inside it.
struct VoxelRef {
  const void* C;
  size_t stride;     // voxels per component plane
  size_t lv;         // v within the planes
  size_t o;          // index in the output maps
  float* score;
  float* lam;
  float* dir;        // d' floats per map voxel
};

__device__ __forceinline__ VoxelRef voxel_ref(const ExtractArgs& a, size_t v) {
  if (!a.items) return VoxelRef{a.C, a.plane, v, box_map_index(a, v), a.score, a.lam, a.dir};
  int lo = 0, hi = a.n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.items[mid].first <= v) lo = mid; else hi = mid - 1;
  }
  const ExtractItem& it = a.items[lo];
  const size_t lv = v - it.first;
  const int by = it.box[1], bx = it.box[2];
  const int vx = (int)(lv % bx), vy = (int)((lv / bx) % by), vz = (int)(lv / ((size_t)bx * by));
  const size_t o = ((size_t)(it.out_lo[0] + vz) * it.out_dims[1] + (it.out_lo[1] + vy)) * it.out_dims[2] +
                   (it.out_lo[2] + vx);
  return VoxelRef{it.C, (size_t)it.box[0] * by * bx, lv, o, it.score, it.lambda, it.dir};
}

}  // namespace ttm
