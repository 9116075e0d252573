// internal.hpp -- declarations shared by the HIP translation units of libttm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/ttm.h"
#include "fft_core.hpp"

namespace ttm {

// ----------------------------------------------------------------------------
// error reporting (thread-local message behind ttm_last_error)
// ----------------------------------------------------------------------------
void set_error(const char* fmt, ...);
int hip_status(hipError_t e, const char* what);

#define TTM_HIP(call)                                          \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return ::ttm::hip_status(e_, #call); \
  } while (0)

// ----------------------------------------------------------------------------
// real-space tile source / destination descriptors for the FFT passes
// ----------------------------------------------------------------------------

// Tile element (z, y, x) of batch b is src[b][oz + z][oy + y][ox + x] when that
// voxel lies inside the dz x dy x dx source, else 0.  If `center` is set the
// value is (v - center[0]); if `square` it is then squared, and with
// `square_odd` so are the odd batch entries (batch_stride 0: a tile and its
// square from one source in one launch).
struct RealSrc {
  const float* p;
  size_t batch_stride;
  int dz, dy, dx;
  int oz, oy, ox;
  const double* center;
  int square;
  int square_odd;
};

// Tile output (z, y, x) with z < sz, y < sy, x < sx lands at
// dst[b][vz0 + z][vy0 + y][vx0 + x] in a bz x by x bx array, multiplied by
// `scale` and, when `w` is set, by w[woz + z][woy + y][wox + x] of a
// wz x wy x wx map.  dtype: 0 = float32, 1 = bfloat16.
struct RealDst {
  void* p;
  int dtype;
  size_t batch_stride;
  int by, bx;
  int vz0, vy0, vx0;
  int sz, sy, sx;
  const float* w;
  int wy, wx;
  int woz, woy, wox;
  float scale;
};

// Twiddle table for edge N inside the context table.
int twiddle_offset(int N);
constexpr int kTwiddleTotal = 32 + 64 + 128 + 256 + 512 + 96 + 160 + 192;

// Forward 3D R2C of `batch` N^3 tiles into half spectra [kz][kx][ky]
// (spec_stride complex elements apart).
int fft3d_forward(int N, const RealSrc& src, int batch, cf* spec, size_t spec_stride,
                  const cf* tw_all, hipStream_t s);

// The X and Y passes of fft3d_forward alone, for tiles whose z planes from
// `planes` on are zero: out[b] = [z < planes][kx][ky] (out_stride complex
// elements apart), the z transform left to fft3d_inverse_mul.
int fft3d_forward_planes(int N, const RealSrc& src, int batch, int planes, cf* out,
                         size_t out_stride, const cf* tw_all, hipStream_t s);

// Inverse: for every a < A, spectrum_a = G * conj(S_a) (+ DC term
// center * N^3 * Re S_a(0) when center is set) is inverse-transformed and the
// cropped, scaled real output written through `dst` (batch index a).
// S holds, s_stride complex elements apart, the first s_planes z planes of
// each x/y-transformed template from fft3d_forward_planes; S_a is its z
// transform, formed column by column inside the kernel.
// `work` holds A spectra.  If S is null, G itself (A = 1) is inverted.
// With gb > 1 (A = 1 only), gb spectra G + i g_stride are each multiplied by
// the same S in one launch: work spectrum i and dst batch entry i are theirs.
int fft3d_inverse_mul(int N, const cf* G, const cf* S, size_t s_stride, int s_planes, int A,
                      const double* center, cf* work, size_t work_stride, const RealDst& dst,
                      const cf* tw_all, hipStream_t s, int gb = 1, size_t g_stride = 0);

int init_twiddles(cf* tw_all, hipStream_t s);

// One box of a batched extraction: the ABI's device table entry.
using ExtractItem = ttm_extract_item;

// Per-voxel extraction launch (extract.hip).
struct ExtractArgs {
  const void* C;       // K planes of `plane` voxels (float32 or bfloat16)
  int in_dtype;
  size_t plane;        // bz * by * bx
  int by, bx;
  float* score;
  float* lam;
  float* dir;
  int oz, oy, ox;      // map position of box voxel (0,0,0)
  int dy, dx;          // map extent along y and x
  int mode;
  const float* starts;
  int n_starts;
  int max_iter;
  float tol;
  int newton;          // Newton polishing steps of the selected answer
  unsigned long long* counters;  // optional: {SS-HOPM steps, Newton steps, oriented voxels}
  // learned start
  const unsigned char* mlp;      // packed BF16 parameters
  float kappa;                   // fall back when lambda / ||C||_F < kappa
  int start_only;                // write the network's start direction only
  int screen;                    // fall back when a fixed start beats the learned lambda
  void* ws;                      // work queues and run results (extract_workspace bytes)
  int* fb_total;                 // optional caller counter of fallbacks
  // batched call: `plane` voxels over n_items boxes of a device table (C, the
  // box geometry and the maps above are then unused)
  const ExtractItem* items;
  int n_items;
};
// Workspace bytes of an orientation extraction over `plane` voxels.
size_t extract_workspace(size_t plane, int degree);
int launch_extract(int degree, const ExtractArgs& a, hipStream_t s);
// The quaternion form (d' = 4, extract4.hip): score at degree 0..6,
// multistart orientation at degree 2 and 4; directions are 4 floats per voxel.
size_t extract_workspace4(size_t plane);
int launch_extract4(int degree, const ExtractArgs& a, hipStream_t s);

// Position refinement TTM-ref (refine.hip): voxels of the sphere |d| <= r_s,
// workspace of a refinement of n_peaks peaks, and the refinement itself
// (opts supplies the multistart options of the d' = 4 orientation).
int sphere_count(float rs);
int max_refine_radius();
size_t refine_workspace(int K, int n_peaks, float rs);
int refine(int degree, int K, const float* g, const float* w, int nz, int ny, int nx, const float* T,
           const float* tn, int L, float r, const int32_t* peaks, int n_peaks, float rs,
           const ExtractArgs& opts, int32_t* pos_out, float* quat_out, float* lncc_out,
           float* quat_peak, float* lncc_peak, void* ws, hipStream_t s);

// Find Peaks over many maps in one launch (peaks_batch.hip); items is a
// device array of ttm_peak_item (include/ttm.h).
size_t peaks_batch_scratch(const int32_t lo[3], const int32_t hi[3]);
int peaks_batch_max_peaks();

// Find Peaks (peaks.hip).
size_t peaks_workspace(int64_t n_voxels);
int find_peaks(const float* score, int nz, int ny, int nx, const int32_t lo[3],
               const int32_t hi[3], int top_p, float min_dist, int32_t* peaks_out,
               float* vals_out, int32_t* n_found_host, void* ws, size_t ws_bytes, hipStream_t s);
int find_peaks_async(const float* score, int nz, int ny, int nx, const int32_t lo[3],
                     const int32_t hi[3], int top_p, float min_dist, int32_t* peaks_out,
                     float* vals_out, int32_t* n_found_dev, void* ws, size_t ws_bytes,
                     hipStream_t s);

// Learned start training (mlp.hip).
size_t mlp_train_workspace(int B);
int mlp_train_step(int degree, int dprime, const float* Cin, const float* T, int B, float* params,
                   float* adam_m, float* adam_v, int step, float lr, unsigned char* packed,
                   float* loss_out, float* grads_out, void* ws, hipStream_t s);
int mlp_pack(int K, const float* params, unsigned char* packed, hipStream_t s);

// Zero-fill with a kernel (graph-capture friendly, unlike memset nodes).
void fill_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace ttm
