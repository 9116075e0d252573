// fft.hip -- batched 3D real FFTs for the tensor-field correlations (gfx950).
//
// Spectrum layout: [kz][kx][ky], ky fastest, kx in 0..N/2 (the R2C half).
// Forward = X pass (two real rows packed as one complex row, R2C split on
// the way out, transposed store so ky becomes contiguous), Y pass (contiguous
// rows), Z pass (strided columns, 16 columns per workgroup so every global
// access is a 128-byte segment).  Templates, which are nonzero only in their
// first L z planes, stop after the Y pass and keep just those planes.
// Inverse = Z pass with the spectral product fused in (one read of G per tile
// for all components; each template column's z transform formed in registers
// from its L stored values), Y pass, X pass with the C2R merge, 1/N^3 scale,
// weight map, crop and dtype conversion fused into the store.
#include "internal.hpp"

namespace ttm {

namespace {

constexpr int kRowsX = 16;  // real rows per workgroup in the X passes (packed in pairs)
constexpr int kRowsC = 32;  // the same in the inverse X pass: its input columns are read in 256-byte pieces

__device__ __forceinline__ float load_src(const RealSrc& s, int b, int z, int y, int x) {
  const int gz = s.oz + z, gy = s.oy + y, gx = s.ox + x;
  if (gz < 0 || gz >= s.dz || gy < 0 || gy >= s.dy || gx < 0 || gx >= s.dx) return 0.0f;
  float v = s.p[b * s.batch_stride + ((size_t)gz * s.dy + gy) * s.dx + gx];
  if (s.center) v = (float)((double)v - s.center[0]);
  if (s.square || (s.square_odd && (b & 1))) v = v * v;
  return v;
}

// Workgroups go to the 8 XCDs in turn (workgroup i to XCD i mod 8), and each
// XCD has its own L2.  This renumbering hands every XCD one contiguous range
// of work items, so neighbouring items -- the two halves of a 128-byte line,
// the components that share a crop's weight-map rows -- meet in one L2.
__device__ __forceinline__ unsigned xcd_item(unsigned bid, unsigned n) {
  constexpr unsigned kXcd = 8;
  return n % kXcd ? bid : (bid % kXcd) * (n / kXcd) + bid / kXcd;
}

__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}

// ---------------------------------------------------------------- X forward
template <int N>
__global__ __launch_bounds__(kRowsX / 2 * Plan<N>::T) void k_r2c_x(RealSrc src, cf* __restrict__ spec,
                                                          size_t spec_stride,
                                                          const cf* __restrict__ tw) {
  constexpr int T = Plan<N>::T, E = N / T, NP = kRowsX / 2, NH = N / 2 + 1;
  constexpr int S = lds_stride<N>();
  constexpr int RS = N + 8;  // padded real row
  constexpr int BYTES_A = kRowsX * RS * 4, BYTES_B = NP * S * 8;
  __shared__ __align__(16) unsigned char smem[BYTES_A > BYTES_B ? BYTES_A : BYTES_B];
  float* rows = reinterpret_cast<float*>(smem);
  cf* xl = reinterpret_cast<cf*>(smem);
  const int tid = threadIdx.x;
  const int y0 = blockIdx.x * kRowsX, z = blockIdx.y, b = blockIdx.z;
  const int p = tid / T, t = tid % T;
  FftTw<N> twr;
  twr.load(tw, t);
  {
    constexpr int NTH = NP * T, IT = kRowsX * N / NTH;
    static_assert(kRowsX * N % NTH == 0, "tile rows");
    float ld[IT];  // all loads in flight, then the LDS stores
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = tid + i * NTH;
      ld[i] = load_src(src, b, z, y0 + e / N, e % N);
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = tid + i * NTH;
      rows[(e / N) * RS + e % N] = ld[i];
    }
  }
  __syncthreads();
  cf v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int n = t + T * j;
    v[j] = cf{rows[(2 * p) * RS + n], rows[(2 * p + 1) * RS + n]};
  }
  __syncthreads();  // rows and xl share memory
  fft_1d<N, false, true>(v, xl + p * S, twr, t);  // each pair's transform lies in one wavefront
#pragma unroll
  for (int j = 0; j < E; ++j) xl[p * S + lds_idx(t + T * j)] = v[j];
  __syncthreads();
  cf* out = spec + b * spec_stride + (size_t)z * NH * N + y0;
  for (int e = tid; e < NH * kRowsX; e += NP * T) {
    const int r = e % kRowsX, kx = e / kRowsX, pp = r >> 1;
    const cf zk = xl[pp * S + lds_idx(kx)];
    const cf zn = cconj(xl[pp * S + lds_idx((N - kx) % N)]);
    cf o;
    if ((r & 1) == 0) {
      o = cscale(cadd(zk, zn), 0.5f);              // (Z[k] + conj Z[N-k]) / 2
    } else {
      const cf d = csub(zk, zn);                   // (Z[k] - conj Z[N-k]) / 2i
      o = cf{0.5f * d.y, -0.5f * d.x};
    }
    out[(size_t)kx * N + r] = o;
  }
}

// ---------------------------------------------------------------- Y (rows)
template <int N, bool INV>
__global__ __launch_bounds__((128 / Plan<N>::T > 0 ? 128 / Plan<N>::T : 1) * Plan<N>::T) void
k_c2c_rows(cf* __restrict__ data, size_t batch_stride, int row_limit, int out_limit,
           const cf* __restrict__ tw) {
  constexpr int T = Plan<N>::T, E = N / T, RB = (128 / T > 0 ? 128 / T : 1);
  constexpr int S = lds_stride<N>();
  __shared__ cf xl[RB * S];
  const int tid = threadIdx.x;
  const int r = tid / T, t = tid % T;
  const int row = blockIdx.x * RB + r;
  FftTw<N> twr;
  twr.load(tw, t);
  // rows are (z, kx): z = row / (N/2+1); rows with z >= row_limit are not
  // needed and may lie past the end of the buffer, so they are not touched.
  // Only the first out_limit outputs of a row are stored (the inverse pass
  // keeps the crop's rows; the X pass reads no others).
  if ((int)(blockIdx.x * RB) / (N / 2 + 1) >= row_limit) return;  // uniform per workgroup
  const bool live = row / (N / 2 + 1) < row_limit;
  cf* base = data + blockIdx.y * batch_stride + (size_t)row * N;
  cf v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = live ? base[t + T * j] : cf{0.0f, 0.0f};
  fft_1d<N, INV, true>(v, xl + r * S, twr, t);  // each row's transform lies in one wavefront
  if (live) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if (t + T * j < out_limit) base[t + T * j] = v[j];
    }
  }
}

// ---------------------------------------------------------------- Z (columns)
template <int N> struct ColBlock { static constexpr int CB = 16; };
// Columns per Z-inverse workgroup: 16 (128-byte row segments), 8 at N = 512
// with more than 2 plane slots (templates over 128 planes, beyond the edge
// the descriptor accepts today), where 16 would not fit the LDS.
template <int N, int JP> struct ZinvBlock { static constexpr int CB = (N >= 512 && JP > 2) ? 8 : 16; };

template <int N, bool INV>
__global__ __launch_bounds__(ColBlock<N>::CB * Plan<N>::T) void k_c2c_cols(
    cf* __restrict__ data, size_t batch_stride, const cf* __restrict__ tw) {
  constexpr int T = Plan<N>::T, E = N / T, CB = ColBlock<N>::CB, NC = (N / 2 + 1) * N;
  constexpr int S = lds_stride_cols<N>();
  __shared__ cf xl[CB * S];
  const int tid = threadIdx.x;
  const int c = tid % CB, t = tid / CB;
  const int col = blockIdx.x * CB + c;
  FftTw<N> twr;
  twr.load(tw, t);
  cf* base = data + blockIdx.y * batch_stride + col;
  cf v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = base[(size_t)(t + T * j) * NC];
  fft_1d<N, INV>(v, xl + c * S, twr, t);
#pragma unroll
  for (int j = 0; j < E; ++j) base[(size_t)(t + T * j) * NC] = v[j];
}

// Element at byte offset `off` from `base`.  A 32-bit offset from a pointer
// that is the same for the whole workgroup lets the compiler address through
// a scalar base and one 32-bit register per access.
__device__ __forceinline__ const cf& at_byte(const cf* base, unsigned off) {
  return *reinterpret_cast<const cf*>(reinterpret_cast<const char*>(base) + off);
}

// Raw buffer accesses (a resource of `bytes` bytes from its base; the
// offset is in bytes).  kBufferWord3 is the gfx9 resource word that selects
// 32-bit elements, the format raw byte-offset accesses take.
constexpr int kBufferWord3 = 0x00020000;
typedef int int2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cf buffer_load_cf(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(cf, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buffer_store_cf(cf v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(int2v, v), r, (int)off, 0, 0);
}

// Inverse Z pass with the spectral product: out_a = Z^-1( G conj(S_a) ).
// P holds only the sp nonzero z planes of each template after its X and Y
// passes; each column of S_a is their z transform, formed here in registers,
// which reads sp/N of the bytes a stored S_a would cost.  JP >= ceil(sp / T)
// plane slots per thread are kept (JP = 0: no template, G itself is
// inverted).  Each column's transforms run on T consecutive threads, inside
// one wavefront, so their exchanges need no workgroup barrier; global
// accesses go through LDS in the other order (column fastest), so that a
// wavefront reads and writes CB neighbouring columns of a z row together.
// Two workgroup barriers per component: after its planes are staged, and
// after its transformed columns are.  The planes of component a + 1 load
// while component a is transformed.  Grid y picks one of several G spectra
// (g_stride apart) for a one-component product: its output is work
// spectrum blockIdx.y.
template <int N, int JP>
__global__ __launch_bounds__((ZinvBlock<N, JP>::CB * Plan<N>::T)) void k_zinv_mul(
    const cf* __restrict__ G, const cf* __restrict__ P, size_t p_stride, int sp, int A,
    const double* __restrict__ center, cf* __restrict__ out, size_t out_stride, int z_limit,
    const cf* __restrict__ tw, size_t g_stride) {
  constexpr int T = Plan<N>::T, E = N / T, CB = ZinvBlock<N, JP>::CB, NC = (N / 2 + 1) * N;
  G += blockIdx.y * g_stride;
  out += blockIdx.y * out_stride;
  constexpr int S = lds_stride<N>();
  constexpr int SB = CB + 1;                // staging row: CB columns, one pad element
  constexpr int ZP = JP > 0 ? JP * T : 1;   // staged template planes
  // byte offsets inside one [z][kx][ky] spectrum stay below 2^32 for N <= 512
  constexpr unsigned ZSTEP = (unsigned)T * NC * 8u;
  static_assert((unsigned long long)N * NC * 8ull < (1ull << 32), "32-bit offsets");
  __shared__ cf xl[CB * S];
  __shared__ cf sb[N * SB];
  __shared__ cf pb[ZP * SB];
  const int tid = threadIdx.x;
  const int c = tid / T, t = tid % T;       // transforms: column c, element t + T j
  const int cc = tid % CB, tt = tid / CB;   // global accesses: column cc, z = tt + T k
  const unsigned col0 = xcd_item(blockIdx.x, gridDim.x) * CB;
  const unsigned offc = ((unsigned)tt * NC + col0 + cc) * 8u;
  FftTw<N> twr;
  twr.load(tw, t);
  {
    cf gl[E];
#pragma unroll
    for (int k = 0; k < E; ++k) gl[k] = at_byte(G, offc + k * ZSTEP);
#pragma unroll
    for (int k = 0; k < E; ++k) sb[(tt + T * k) * SB + cc] = gl[k];
  }
  // The template planes are read and the columns written through buffer
  // resources whose size ends at the sp stored planes and at the crop's
  // z_limit rows: the hardware returns 0 for a read past the end and drops a
  // write past it, so no lane needs a branch or a select for its row.
  cf qn[JP > 0 ? JP : 1];  // planes of the next component, global-access order
  auto load_planes = [&](int a) {
    const auto rp = __builtin_amdgcn_make_buffer_rsrc(const_cast<cf*>(P + (size_t)a * p_stride), (short)0,
                                                      sp * NC * 8, kBufferWord3);
#pragma unroll
    for (int k = 0; k < JP; ++k) qn[k] = buffer_load_cf(rp, offc + k * ZSTEP);
  };
  if constexpr (JP > 0) load_planes(0);
  __syncthreads();  // G staged
  cf g[E];
#pragma unroll
  for (int j = 0; j < E; ++j) g[j] = sb[(t + T * j) * SB + c];
  // DC bin (kz = kx = ky = 0) is element j = 0 of thread t = 0 in column 0:
  // restore the mean removed before the forward transform.
  if (JP > 0 && center && col0 + c == 0 && t == 0) {
    g[0].x += (float)(center[0] * (double)N * (double)N * (double)N);
  }
  if constexpr (JP > 0) {
#pragma unroll
    for (int k = 0; k < JP; ++k) pb[(tt + T * k) * SB + cc] = qn[k];
  }
  // Component a: its planes are in pb; the planes of a + 1 load during its
  // transforms and are staged right after its columns are, before its
  // stores are issued.  Waiting for a load also waits for every earlier
  // store (one counter covers both), so staging the planes there waits only
  // for stores issued a whole component earlier, which have drained, and
  // this component's stores drain during the next one's transforms.
  for (int a = 0; a < A; ++a) {
    cf v[E];
    __syncthreads();  // component a's planes staged; the previous columns read from sb
    if constexpr (JP > 0) {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = j < JP ? pb[(t + T * j) * SB + c] : cf{0.0f, 0.0f};
      if (a + 1 < A) load_planes(a + 1);
      fft_1d<N, false, true>(v, xl + c * S, twr, t);  // S_a along this column
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = cmulc(g[j], v[j]);
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = g[j];
    }
    fft_1d<N, true, true>(v, xl + c * S, twr, t);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if (t + T * j < z_limit) sb[(t + T * j) * SB + c] = v[j];
    }
    __syncthreads();  // columns staged; every wave has read component a's planes
    if constexpr (JP > 0) {
      if (a + 1 < A) {
#pragma unroll
        for (int k = 0; k < JP; ++k) pb[(tt + T * k) * SB + cc] = qn[k];
      }
    }
    const auto ro = __builtin_amdgcn_make_buffer_rsrc(out + (size_t)a * out_stride, (short)0,
                                                      z_limit * NC * 8, kBufferWord3);
#pragma unroll
    for (int k = 0; k < E; ++k) buffer_store_cf(sb[(tt + T * k) * SB + cc], ro, offc + k * ZSTEP);
  }
}

// ---------------------------------------------------------------- X inverse
template <int N>
__global__ __launch_bounds__(kRowsC / 2 * Plan<N>::T) __attribute__((amdgpu_waves_per_eu(N == 512 ? 8 : 1))) void k_c2r_x(const cf* __restrict__ spec,
                                                          size_t spec_stride, int A, RealDst dst,
                                                          const cf* __restrict__ tw) {
  constexpr int T = Plan<N>::T, E = N / T, NP = kRowsC / 2, NH = N / 2 + 1;
  constexpr int S = lds_stride<N>();
  constexpr int SPS = NH + 1;  // padded spectrum row
  constexpr int BYTES_A = kRowsC * SPS * 8, BYTES_B = NP * S * 8, BYTES_C = kRowsC * (N + 4) * 4;
  constexpr int BYTES = BYTES_A > BYTES_B ? (BYTES_A > BYTES_C ? BYTES_A : BYTES_C)
                                          : (BYTES_B > BYTES_C ? BYTES_B : BYTES_C);
  __shared__ __align__(16) unsigned char smem[BYTES];
  cf* sp = reinterpret_cast<cf*>(smem);
  cf* xl = reinterpret_cast<cf*>(smem);
  float* orow = reinterpret_cast<float*>(smem);
  const int tid = threadIdx.x;
  // work items: component fastest, then row block, then z plane, so the
  // workgroups that share a crop's weight-map rows run together in one XCD
  constexpr int NYB = N / kRowsC;
  const int item = (int)xcd_item(blockIdx.x, gridDim.x);
  const int b = item % A, y0 = (item / A) % NYB * kRowsC, z = item / A / NYB;
  if (z >= dst.sz || y0 >= dst.sy) return;  // uniform: nothing of this block is kept
  const int p = tid / T, t = tid % T;
  constexpr int NTH = NP * T, NIN = NH * kRowsC, IT = (NIN + NTH - 1) / NTH;
  const cf* in = spec + b * spec_stride + (size_t)z * NH * N + y0;
  {
    // all loads first (indices clamped, so every one is in bounds), then the
    // LDS stores: the loads are in flight together.  Rows past the crop were
    // not stored by the Y pass; they are read as zeros (each is paired with a
    // kept row in one complex transform, so it must be finite).
    const int nrows_in = min(kRowsC, dst.sy - y0);
    cf ld[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = min(tid + i * NTH, NIN - 1);
      ld[i] = e % kRowsC < nrows_in ? at_byte(in, (unsigned)((e / kRowsC) * N + e % kRowsC) * 8u)
                                    : cf{0.0f, 0.0f};
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = tid + i * NTH;
      if (e < NIN) sp[(e % kRowsC) * SPS + e / kRowsC] = ld[i];
    }
  }
  FftTw<N> twr;  // in flight across the barrier
  twr.load(tw, t);
  __syncthreads();
  cf v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int n = t + T * j;
    cf a, bb;
    if (n <= N / 2) {
      a = sp[(2 * p) * SPS + n];
      bb = sp[(2 * p + 1) * SPS + n];
      if (n == 0 || n == N / 2) {  // spectra of real rows: these bins are real
        a.y = 0.0f;
        bb.y = 0.0f;
      }
    } else {
      a = cconj(sp[(2 * p) * SPS + (N - n)]);
      bb = cconj(sp[(2 * p + 1) * SPS + (N - n)]);
    }
    v[j] = cf{a.x - bb.y, a.y + bb.x};  // A + iB
  }
  __syncthreads();
  fft_1d<N, true, true>(v, xl + p * S, twr, t);  // each pair's transform lies in one wavefront
  __syncthreads();  // the row buffer overlaps other pairs' exchange areas
  constexpr int RS = N + 4;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int n = t + T * j;
    orow[(2 * p) * RS + n] = v[j].x;
    orow[(2 * p + 1) * RS + n] = v[j].y;
  }
  __syncthreads();
  const int nrows = min(kRowsC, dst.sy - y0);
  const int sx = dst.sx;
  // row bases are the same for the whole workgroup, so each access takes a
  // scalar base and the lane's 32-bit byte offset
  const size_t o0 = b * dst.batch_stride +
                    ((size_t)(dst.vz0 + z) * dst.by + (dst.vy0 + y0)) * dst.bx + dst.vx0;
  const float* wr = dst.w ? dst.w + ((size_t)(dst.woz + z) * dst.wy + (dst.woy + y0)) * dst.wx + dst.wox
                          : nullptr;
  // one output column x of one group of RH rows per thread and pass: the
  // group's weight-map loads (row indices clamped into the crop) are in flight
  // together
  constexpr int RH = 16, NG = kRowsC / RH;
  for (int i = tid; i < sx * NG; i += NTH) {
    const int g = i / sx, x = i - g * sx, r0 = g * RH;
    float val[RH];
#pragma unroll
    for (int r = 0; r < RH; ++r) val[r] = orow[(r0 + r) * RS + x] * dst.scale;
    if (wr) {
      float wv[RH];
#pragma unroll
      for (int r = 0; r < RH; ++r) {
        const float* row = wr + (size_t)min(r0 + r, nrows - 1) * dst.wx;
        wv[r] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(row) + 4u * (unsigned)x);
      }
#pragma unroll
      for (int r = 0; r < RH; ++r) val[r] *= wv[r];
    }
    if (dst.dtype == 1) {
      unsigned short* out = reinterpret_cast<unsigned short*>(dst.p) + o0;
#pragma unroll
      for (int r = 0; r < RH; ++r) {
        if (r0 + r < nrows) {
          char* row = reinterpret_cast<char*>(out + (size_t)(r0 + r) * dst.bx);
          *reinterpret_cast<unsigned short*>(row + 2u * (unsigned)x) = f32_to_bf16(val[r]);
        }
      }
    } else {
      float* out = reinterpret_cast<float*>(dst.p) + o0;
#pragma unroll
      for (int r = 0; r < RH; ++r) {
        if (r0 + r < nrows) {
          char* row = reinterpret_cast<char*>(out + (size_t)(r0 + r) * dst.bx);
          *reinterpret_cast<float*>(row + 4u * (unsigned)x) = val[r];
        }
      }
    }
  }
}

__global__ void k_twiddles(cf* tw_all) {
  const int sizes[8] = {32, 64, 128, 256, 512, 96, 160, 192};
  int off = 0;
  for (int s = 0; s < 8; ++s) {
    const int N = sizes[s];
    for (int e = threadIdx.x; e < N; e += blockDim.x) {
      double sv, cv;
      sincospi(-2.0 * (double)e / (double)N, &sv, &cv);
      tw_all[off + e] = cf{(float)cv, (float)sv};
    }
    off += N;
  }
}

template <int N>
int forward_n(const RealSrc& src, int batch, cf* spec, size_t spec_stride, const cf* tw,
              hipStream_t s) {
  constexpr int T = Plan<N>::T;
  hipLaunchKernelGGL(k_r2c_x<N>, dim3(N / kRowsX, N, batch), dim3(kRowsX / 2 * T), 0, s, src, spec,
                     spec_stride, tw);
  constexpr int RB = (128 / T > 0 ? 128 / T : 1);
  constexpr int NROWS = N * (N / 2 + 1);
  hipLaunchKernelGGL((k_c2c_rows<N, false>), dim3(NROWS / RB, batch), dim3(RB * T), 0, s, spec,
                     spec_stride, N, N, tw);
  constexpr int CB = ColBlock<N>::CB;
  hipLaunchKernelGGL((k_c2c_cols<N, false>), dim3(NROWS / CB, batch), dim3(CB * T), 0, s, spec,
                     spec_stride, tw);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : hip_status(e, "fft forward launch");
}

template <int N>
int forward_planes_n(const RealSrc& src, int batch, int planes, cf* out, size_t out_stride,
                     const cf* tw, hipStream_t s) {
  constexpr int T = Plan<N>::T;
  hipLaunchKernelGGL(k_r2c_x<N>, dim3(N / kRowsX, planes, batch), dim3(kRowsX / 2 * T), 0, s, src,
                     out, out_stride, tw);
  constexpr int RB = (128 / T > 0 ? 128 / T : 1);
  const int rows = planes * (N / 2 + 1);
  hipLaunchKernelGGL((k_c2c_rows<N, false>), dim3((rows + RB - 1) / RB, batch), dim3(RB * T), 0, s,
                     out, out_stride, planes, N, tw);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : hip_status(e, "fft forward launch");
}

template <int N>
int inverse_n(const cf* G, const cf* Sp, size_t s_stride, int s_planes, int A, const double* center,
              cf* work, size_t work_stride, const RealDst& dst, const cf* tw, hipStream_t s,
              int gb, size_t g_stride) {
  constexpr int T = Plan<N>::T;
  constexpr int NROWS = N * (N / 2 + 1);
  const int zlim = dst.sz;
  constexpr int E = N / T;
  // template slots per thread: the next power of two >= ceil(s_planes / T),
  // and at least 2 at N = 512, whose one-slot variant the compiler keeps in
  // more registers (137 against 123)
  int jp = 0;
  if (Sp) {
    jp = N == 512 ? 2 : 1;
    while (jp < E && jp * T < s_planes) jp *= 2;
  }
  auto launch = [&](auto kern, int cb) {
    hipLaunchKernelGGL(kern, dim3(NROWS / cb, gb), dim3(cb * T), 0, s, G, Sp, s_stride, s_planes, A,
                       center, work, work_stride, zlim, tw, g_stride);
  };
  constexpr int J2 = 2 < E ? 2 : E, J4 = 4 < E ? 4 : E, J8 = 8 < E ? 8 : E;
  switch (jp) {
    case 0: launch(k_zinv_mul<N, 0>, ZinvBlock<N, 0>::CB); break;
    case 1: launch(k_zinv_mul<N, 1>, ZinvBlock<N, 1>::CB); break;
    case 2: launch(k_zinv_mul<N, J2>, ZinvBlock<N, J2>::CB); break;
    case 4: launch(k_zinv_mul<N, J4>, ZinvBlock<N, J4>::CB); break;
    case 8: launch(k_zinv_mul<N, J8>, ZinvBlock<N, J8>::CB); break;
    default: launch(k_zinv_mul<N, E>, ZinvBlock<N, E>::CB); break;
  }
  const int nb = A * gb;  // work spectra written by the Z pass
  constexpr int RB = (128 / T > 0 ? 128 / T : 1);
  hipLaunchKernelGGL((k_c2c_rows<N, true>), dim3(NROWS / RB, nb), dim3(RB * T), 0, s, work,
                     work_stride, zlim, dst.sy, tw);
  hipLaunchKernelGGL(k_c2r_x<N>, dim3(nb * (N / kRowsC) * N), dim3(kRowsC / 2 * T), 0, s, work,
                     work_stride, nb, dst, tw);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : hip_status(e, "fft inverse launch");
}

}  // namespace

int twiddle_offset(int N) {
  switch (N) {
    case 32: return 0;
    case 64: return 32;
    case 128: return 96;
    case 256: return 224;
    case 512: return 480;
    case 96: return 992;
    case 160: return 1088;
    case 192: return 1248;
    default: return -1;
  }
}

int init_twiddles(cf* tw_all, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3(1), dim3(256), 0, s, tw_all);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : hip_status(e, "twiddle init");
}

int fft3d_forward(int N, const RealSrc& src, int batch, cf* spec, size_t spec_stride,
                  const cf* tw_all, hipStream_t s) {
  const cf* tw = tw_all + twiddle_offset(N);
  switch (N) {
    case 32: return forward_n<32>(src, batch, spec, spec_stride, tw, s);
    case 64: return forward_n<64>(src, batch, spec, spec_stride, tw, s);
    case 128: return forward_n<128>(src, batch, spec, spec_stride, tw, s);
    case 256: return forward_n<256>(src, batch, spec, spec_stride, tw, s);
    case 512: return forward_n<512>(src, batch, spec, spec_stride, tw, s);
    case 96: return forward_n<96>(src, batch, spec, spec_stride, tw, s);
    case 160: return forward_n<160>(src, batch, spec, spec_stride, tw, s);
    case 192: return forward_n<192>(src, batch, spec, spec_stride, tw, s);
    default: set_error("unsupported FFT edge %d", N); return -4;
  }
}

int fft3d_forward_planes(int N, const RealSrc& src, int batch, int planes, cf* out,
                         size_t out_stride, const cf* tw_all, hipStream_t s) {
  const cf* tw = tw_all + twiddle_offset(N);
  switch (N) {
    case 32: return forward_planes_n<32>(src, batch, planes, out, out_stride, tw, s);
    case 64: return forward_planes_n<64>(src, batch, planes, out, out_stride, tw, s);
    case 128: return forward_planes_n<128>(src, batch, planes, out, out_stride, tw, s);
    case 256: return forward_planes_n<256>(src, batch, planes, out, out_stride, tw, s);
    case 512: return forward_planes_n<512>(src, batch, planes, out, out_stride, tw, s);
    case 96: return forward_planes_n<96>(src, batch, planes, out, out_stride, tw, s);
    case 160: return forward_planes_n<160>(src, batch, planes, out, out_stride, tw, s);
    case 192: return forward_planes_n<192>(src, batch, planes, out, out_stride, tw, s);
    default: set_error("unsupported FFT edge %d", N); return -4;
  }
}

int fft3d_inverse_mul(int N, const cf* G, const cf* Sp, size_t s_stride, int s_planes, int A,
                      const double* center, cf* work, size_t work_stride, const RealDst& dst,
                      const cf* tw_all, hipStream_t s, int gb, size_t g_stride) {
  if (gb < 1 || (gb > 1 && A != 1)) {
    set_error("fft inverse: a batch of %d G spectra needs one component (A = %d)", gb, A);
    return -1;
  }
  const cf* tw = tw_all + twiddle_offset(N);
  switch (N) {
    case 32: return inverse_n<32>(G, Sp, s_stride, s_planes, A, center, work, work_stride, dst, tw, s, gb, g_stride);
    case 64: return inverse_n<64>(G, Sp, s_stride, s_planes, A, center, work, work_stride, dst, tw, s, gb, g_stride);
    case 128: return inverse_n<128>(G, Sp, s_stride, s_planes, A, center, work, work_stride, dst, tw, s, gb, g_stride);
    case 256: return inverse_n<256>(G, Sp, s_stride, s_planes, A, center, work, work_stride, dst, tw, s, gb, g_stride);
    case 512: return inverse_n<512>(G, Sp, s_stride, s_planes, A, center, work, work_stride, dst, tw, s, gb, g_stride);
    case 96: return inverse_n<96>(G, Sp, s_stride, s_planes, A, center, work, work_stride, dst, tw, s, gb, g_stride);
    case 160: return inverse_n<160>(G, Sp, s_stride, s_planes, A, center, work, work_stride, dst, tw, s, gb, g_stride);
    case 192: return inverse_n<192>(G, Sp, s_stride, s_planes, A, center, work, work_stride, dst, tw, s, gb, g_stride);
    default: set_error("unsupported FFT edge %d", N); return -4;
  }
}

}  // namespace ttm
