// fft_core.hpp -- in-register / LDS building blocks of the batched 1D FFTs
// that make up the 3D transforms (gfx950, wave64).
//
// A length-N transform is spread over T threads; thread t owns the E = N/T
// elements with index t + T*j (j < E), before and after the transform.  The
// transform runs as a sequence of Stockham radix-R stages (N = R0*R1[*R2];
// R0 may be a composite 6, 10 or 12 for the edges 96, 160 and 192):
// butterfly i = t + T*b reads x[i + m*N/R] (m < R), twiddles by
// W_{P*R}^{(i mod P)*m}, applies a radix-R DFT in registers and writes
// x'[(i - i mod P)*R + i mod P + m*P], P being the product of the earlier
// radices.  The first stage reads from and the last stage writes to the
// registers directly; the stages in between exchange through LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace ttm {

struct cf {  // complex float, 8-byte aligned like float2
  float x, y;
};

__device__ __forceinline__ cf cmake(float a, float b) { return cf{a, b}; }
__device__ __forceinline__ cf cadd(cf a, cf b) { return cf{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return cf{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf cmul(cf a, cf b) {
  return cf{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
__device__ __forceinline__ cf cmulc(cf a, cf b) {
  return cf{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
__device__ __forceinline__ cf cconj(cf a) { return cf{a.x, -a.y}; }
__device__ __forceinline__ cf cscale(cf a, float s) { return cf{a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse) depending on INV
template <bool INV>
__device__ __forceinline__ cf rot_quarter(cf a) {
  return INV ? cf{-a.y, a.x} : cf{a.y, -a.x};
}

// cos(2 pi k / 16), k = 0..15
__device__ constexpr float kCos16[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};

// a * W_16^e with W = exp(-2 pi i / 16) (forward) or its conjugate (inverse);
// e is a compile-time constant so trivial factors cost nothing.
template <int E16, bool INV>
__device__ __forceinline__ cf twiddle16(cf a) {
  constexpr int e = ((E16 % 16) + 16) % 16;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (e == 4) {
    return rot_quarter<INV>(a);
  } else if constexpr (e == 8) {
    return cf{-a.x, -a.y};
  } else if constexpr (e == 12) {
    return rot_quarter<!INV>(a);
  } else {
    const float c = kCos16[e];
    const float s = INV ? kCos16[(e + 12) % 16] : -kCos16[(e + 12) % 16];  // +-sin(2 pi e/16)
    return cf{a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

template <bool INV>
__device__ __forceinline__ void dft2(cf& a0, cf& a1) {
  cf t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

template <bool INV>
__device__ __forceinline__ void dft4(cf& a0, cf& a1, cf& a2, cf& a3) {
  cf t0 = cadd(a0, a2), t1 = csub(a0, a2);
  cf t2 = cadd(a1, a3), t3 = rot_quarter<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// Radix-3 DFT: X1,2 = a0 - (a1 + a2)/2 -+ i (sqrt(3)/2)(a1 - a2) (forward; +- inverse).
template <bool INV>
__device__ __forceinline__ void dft3(cf& a0, cf& a1, cf& a2) {
  const cf t1 = cadd(a1, a2), t2 = csub(a1, a2);
  const cf m = cf{a0.x - 0.5f * t1.x, a0.y - 0.5f * t1.y};
  const cf r = rot_quarter<INV>(cscale(t2, 0.86602540378443865f));
  a0 = cadd(a0, t1);
  a1 = cadd(m, r);
  a2 = csub(m, r);
}

// Radix-5 DFT with c_k = cos(2 pi k/5), s_k = sin(2 pi k/5):
// X1,4 = a0 + c1 (a1 + a4) + c2 (a2 + a3) -+ i (s1 (a1 - a4) + s2 (a2 - a3)),
// X2,3 = a0 + c2 (a1 + a4) + c1 (a2 + a3) -+ i (s2 (a1 - a4) - s1 (a2 - a3))
// (forward; the signs of the i terms swap for the inverse).
template <bool INV>
__device__ __forceinline__ void dft5(cf& a0, cf& a1, cf& a2, cf& a3, cf& a4) {
  constexpr float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
  constexpr float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
  const cf t1 = cadd(a1, a4), t2 = cadd(a2, a3), t3 = csub(a1, a4), t4 = csub(a2, a3);
  const cf m1 = cf{a0.x + c1 * t1.x + c2 * t2.x, a0.y + c1 * t1.y + c2 * t2.y};
  const cf m2 = cf{a0.x + c2 * t1.x + c1 * t2.x, a0.y + c2 * t1.y + c1 * t2.y};
  const cf n1 = rot_quarter<INV>(cf{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
  const cf n2 = rot_quarter<INV>(cf{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
  a0 = cadd(a0, cadd(t1, t2));
  a1 = cadd(m1, n1);
  a4 = csub(m1, n1);
  a2 = cadd(m2, n2);
  a3 = csub(m2, n2);
}

// cos and sin of 2 pi e / R for the composite radices 6, 10, 12
template <int R> struct RootTable;
template <> struct RootTable<6> {
  static constexpr float c[6] = {1.0f, 0.5f, -0.5f, -1.0f, -0.5f, 0.5f};
  static constexpr float s[6] = {0.0f, 0.86602540378443865f, 0.86602540378443865f, 0.0f,
                                 -0.86602540378443865f, -0.86602540378443865f};
};
template <> struct RootTable<10> {
  static constexpr float c[10] = {1.0f, 0.80901699437494742f, 0.30901699437494742f,
                                  -0.30901699437494742f, -0.80901699437494742f, -1.0f,
                                  -0.80901699437494742f, -0.30901699437494742f,
                                  0.30901699437494742f, 0.80901699437494742f};
  static constexpr float s[10] = {0.0f, 0.58778525229247313f, 0.95105651629515357f,
                                  0.95105651629515357f, 0.58778525229247313f, 0.0f,
                                  -0.58778525229247313f, -0.95105651629515357f,
                                  -0.95105651629515357f, -0.58778525229247313f};
};
template <> struct RootTable<12> {
  static constexpr float c[12] = {1.0f, 0.86602540378443865f, 0.5f, 0.0f, -0.5f,
                                  -0.86602540378443865f, -1.0f, -0.86602540378443865f, -0.5f,
                                  0.0f, 0.5f, 0.86602540378443865f};
  static constexpr float s[12] = {0.0f, 0.5f, 0.86602540378443865f, 1.0f, 0.86602540378443865f,
                                  0.5f, 0.0f, -0.5f, -0.86602540378443865f, -1.0f,
                                  -0.86602540378443865f, -0.5f};
};

// a * W_R^e, W_R = exp(-2 pi i / R) (forward) or its conjugate (inverse)
template <int R, int E, bool INV>
__device__ __forceinline__ cf twiddle_r(cf a) {
  constexpr int e = ((E % R) + R) % R;
  if constexpr (e == 0) {
    return a;
  } else {
    const float c = RootTable<R>::c[e];
    const float s = INV ? RootTable<R>::s[e] : -RootTable<R>::s[e];
    return cf{a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

template <int R, bool INV> __device__ __forceinline__ void dft(cf* a);

// y[n1 R2 + k2] *= W_R^{n1 k2} for every n1, k2 (exponents fixed at compile time)
template <int R, int R2, bool INV, int I = 0>
__device__ __forceinline__ void twiddle_split(cf* y) {
  if constexpr (I < R) {
    y[I] = twiddle_r<R, (I / R2) * (I % R2), INV>(y[I]);
    twiddle_split<R, R2, INV, I + 1>(y);
  }
}

// Composite radix R = R1 * R2 by one four-step split: n = n1 + R1 n2,
// k = R2 k1 + k2: R1 transforms of length R2 over n2, twiddles W_R^{n1 k2},
// R2 transforms of length R1 over n1.
template <int R1, int R2, bool INV>
__device__ __forceinline__ void dft_split(cf* a) {
  constexpr int R = R1 * R2;
  cf y[R];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    cf b[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) b[n2] = a[n1 + R1 * n2];
    dft<R2, INV>(b);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[n1 * R2 + k2] = b[k2];
  }
  twiddle_split<R, R2, INV>(y);
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    cf b[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) b[n1] = y[n1 * R2 + k2];
    dft<R1, INV>(b);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) a[R2 * k1 + k2] = b[k1];
  }
}

// Radix-R DFT of a[0..R-1] in place, natural order in and out, R in
// {2, 3, 4, 5, 6, 8, 10, 12, 16}.  R = 8 and 16 use one four-step split:
// n = n1 + R1 n2, k = R2 k1 + k2; 6, 10 and 12 use dft_split.
template <int R, bool INV>
__device__ __forceinline__ void dft(cf* a) {
  if constexpr (R == 1) {
  } else if constexpr (R == 3) {
    dft3<INV>(a[0], a[1], a[2]);
  } else if constexpr (R == 5) {
    dft5<INV>(a[0], a[1], a[2], a[3], a[4]);
  } else if constexpr (R == 6) {
    dft_split<2, 3, INV>(a);
  } else if constexpr (R == 10) {
    dft_split<2, 5, INV>(a);
  } else if constexpr (R == 12) {
    dft_split<3, 4, INV>(a);
  } else if constexpr (R == 2) {
    dft2<INV>(a[0], a[1]);
  } else if constexpr (R == 4) {
    dft4<INV>(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 8) {
    // R1 = 2, R2 = 4
    dft4<INV>(a[0], a[2], a[4], a[6]);                 // n1 = 0
    dft4<INV>(a[1], a[3], a[5], a[7]);                 // n1 = 1
    // Y[1][k2] *= W_8^{k2}
    a[3] = twiddle16<2, INV>(a[3]);
    a[5] = twiddle16<4, INV>(a[5]);
    a[7] = twiddle16<6, INV>(a[7]);
    cf y[8] = {a[0], a[2], a[4], a[6], a[1], a[3], a[5], a[7]};  // y[n1*4 + k2]
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      cf u0 = y[k2], u1 = y[4 + k2];
      dft2<INV>(u0, u1);
      a[k2] = u0;       // k = 4*0 + k2
      a[4 + k2] = u1;   // k = 4*1 + k2
    }
  } else if constexpr (R == 16) {
    // R1 = 4, R2 = 4
    cf y[16];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
      cf b0 = a[n1], b1 = a[n1 + 4], b2 = a[n1 + 8], b3 = a[n1 + 12];
      dft4<INV>(b0, b1, b2, b3);
      y[n1 * 4 + 0] = b0;
      y[n1 * 4 + 1] = b1;
      y[n1 * 4 + 2] = b2;
      y[n1 * 4 + 3] = b3;
    }
    y[5] = twiddle16<1, INV>(y[5]);
    y[6] = twiddle16<2, INV>(y[6]);
    y[7] = twiddle16<3, INV>(y[7]);
    y[9] = twiddle16<2, INV>(y[9]);
    y[10] = twiddle16<4, INV>(y[10]);
    y[11] = twiddle16<6, INV>(y[11]);
    y[13] = twiddle16<3, INV>(y[13]);
    y[14] = twiddle16<6, INV>(y[14]);
    y[15] = twiddle16<9, INV>(y[15]);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      cf b0 = y[k2], b1 = y[4 + k2], b2 = y[8 + k2], b3 = y[12 + k2];
      dft4<INV>(b0, b1, b2, b3);
      a[k2] = b0;
      a[4 + k2] = b1;
      a[8 + k2] = b2;
      a[12 + k2] = b3;
    }
  } else {
    static_assert(R == 2, "unsupported radix");
  }
}

// Plans: threads per transform and stage radices for each supported edge.
template <int N> struct Plan;
template <> struct Plan<32> { static constexpr int T = 4, R0 = 4, R1 = 8, R2 = 1; };
template <> struct Plan<64> { static constexpr int T = 8, R0 = 8, R1 = 8, R2 = 1; };
template <> struct Plan<128> { static constexpr int T = 8, R0 = 8, R1 = 16, R2 = 1; };
template <> struct Plan<256> { static constexpr int T = 16, R0 = 16, R1 = 16, R2 = 1; };
template <> struct Plan<512> { static constexpr int T = 64, R0 = 8, R1 = 8, R2 = 8; };
// edges with a factor 3 or 5 (96 = 6 * 4 * 4, 160 = 10 * 4 * 4, 192 = 12 * 4 * 4)
template <> struct Plan<96> { static constexpr int T = 8, R0 = 6, R1 = 4, R2 = 4; };
template <> struct Plan<160> { static constexpr int T = 8, R0 = 10, R1 = 4, R2 = 4; };
template <> struct Plan<192> { static constexpr int T = 16, R0 = 12, R1 = 4, R2 = 4; };

// LDS footprint (complex elements) of one transform's exchange area.  Inside
// an area one padding element per 16 keeps stride-16 exchanges conflict-free.
// The areas of the transforms that share a wavefront are set apart by a
// stride chosen per edge and thread mapping (64 banks of 4 bytes, b64
// accesses): with one transform per T consecutive threads (rows) and with
// the transforms interleaved across consecutive threads (columns, thread
// c + CB*t), every exchange of the plan then touches each bank at most twice,
// the least a 64-lane b64 access can.
template <int N>
__host__ __device__ constexpr int lds_stride() {
  return N == 64 ? 76 : N == 128 ? 140 : N == 256 ? 280 : N + N / 16 + 1;
}
template <int N>
__host__ __device__ constexpr int lds_stride_cols() {
  return N == 64 ? 70 : N == 128 ? 138 : N == 256 ? 274 : N == 512 ? 548 : N + N / 16 + 1;
}
__device__ __forceinline__ int lds_idx(int i) { return i + (i >> 4); }

// Twiddles of one thread for the LDS stages of a length-N transform, held in
// registers: stage s (radix R, span P) needs W_{P*R}^{(i mod P)*m} for its
// butterflies i = t + T*b and m = 1..R-1, taken from the table
// tw[e] = exp(-2 pi i e / N) as entry (i mod P)*m*N/(P*R).  Loading them at
// kernel entry lets their latency overlap the data loads; the inverse uses
// the conjugates of the same values.
template <int N>
struct FftTw {
  using PL = Plan<N>;
  static constexpr int T = PL::T, E = N / T;
  static constexpr int N1 = E / PL::R1 * (PL::R1 - 1);
  static constexpr int N2 = PL::R2 > 1 ? E / PL::R2 * (PL::R2 - 1) : 1;
  cf w1[N1];
  cf w2[N2];

  template <int R, int P, int M>
  __device__ __forceinline__ static void fill(cf (&w)[M], const cf* __restrict__ tw, int t) {
    constexpr int NB = E / R, S = N / (P * R);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int k = (t + T * b) % P;
#pragma unroll
      for (int m = 1; m < R; ++m) w[b * (R - 1) + m - 1] = tw[k * m * S];
    }
  }
  __device__ __forceinline__ void load(const cf* __restrict__ tw, int t) {
    fill<PL::R1, PL::R0>(w1, tw, t);
    if constexpr (PL::R2 > 1) fill<PL::R2, PL::R0 * PL::R1>(w2, tw, t);
  }
};

// Orders one wavefront's LDS writes before its later reads by other lanes of
// the same wavefront (a wavefront's LDS instructions execute in order; the
// fence keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Exchange barrier of a transform: the whole workgroup, or (WAVE) only the
// wavefront, when every transform's T threads lie inside one wavefront and no
// other wavefront touches its LDS area.
template <bool WAVE>
__device__ __forceinline__ void fft_sync() {
  if constexpr (WAVE) {
    wave_lds_sync();
  } else {
    __syncthreads();
  }
}

// One Stockham stage from LDS to LDS (or registers for the last stage).
// span = P (product of earlier radices).  Reads x[i + m*N/R], writes
// x'[(i - k)*R + k + m*P] with k = i mod P.  wt: this stage's twiddles.
template <int N, int T, int R, int P, bool LAST, bool INV, bool WAVE>
__device__ __forceinline__ void stage_lds(cf (&v)[N / T], cf* lds, const cf* wt, int t) {
  constexpr int E = N / T;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "plan: radix must divide per-thread count");
  static_assert(P > 1, "LDS stages follow the first stage");
  cf u[E];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + T * b;
#pragma unroll
    for (int m = 0; m < R; ++m) u[b * R + m] = lds[lds_idx(i + m * (N / R))];
  }
  fft_sync<WAVE>();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + T * b;
    const int k = i % P;
    cf* w = &u[b * R];
#pragma unroll
    for (int m = 1; m < R; ++m) {
      const cf tw = wt[b * (R - 1) + m - 1];
      w[m] = cmul(w[m], INV ? cconj(tw) : tw);
    }
    dft<R, INV>(w);
    if constexpr (LAST) {
#pragma unroll
      for (int m = 0; m < R; ++m) v[b + m * NB] = w[m];      // index t + T*(b + m*NB)
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m) lds[lds_idx((i - k) * R + k + m * P)] = w[m];
    }
  }
  if constexpr (!LAST) fft_sync<WAVE>();
}

// Full transform.  On entry v[j] = x[t + T*j]; on exit v[j] = X[t + T*j].
// lds: this transform's exchange area (lds_stride<N>() elements).
// Every thread of the workgroup (WAVE: of the wavefront) must call it.
template <int N, bool INV, bool WAVE = false>
__device__ __forceinline__ void fft_1d(cf (&v)[N / Plan<N>::T], cf* lds, const FftTw<N>& tw,
                                       int t) {
  using PL = Plan<N>;
  constexpr int T = PL::T, E = N / T, R0 = PL::R0, R1 = PL::R1, R2 = PL::R2;
  constexpr int NB0 = E / R0;
  static_assert(E % R0 == 0, "plan");
  // stage 0 (P = 1): inputs of butterfly b are v[b + m*NB0]; no twiddles
#pragma unroll
  for (int b = 0; b < NB0; ++b) {
    cf w[R0];
#pragma unroll
    for (int m = 0; m < R0; ++m) w[m] = v[b + m * NB0];
    dft<R0, INV>(w);
    const int i = t + T * b;
#pragma unroll
    for (int m = 0; m < R0; ++m) lds[lds_idx(i * R0 + m)] = w[m];
  }
  fft_sync<WAVE>();
  if constexpr (R2 == 1) {
    stage_lds<N, T, R1, R0, true, INV, WAVE>(v, lds, tw.w1, t);
  } else {
    stage_lds<N, T, R1, R0, false, INV, WAVE>(v, lds, tw.w1, t);
    stage_lds<N, T, R2, R0 * R1, true, INV, WAVE>(v, lds, tw.w2, t);
  }
}

}  // namespace ttm
