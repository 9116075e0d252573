// sym_tables.hpp -- compile-time index tables of degree-n symmetric tensors
// over R^3 (the d' = 3 template-axis form).
//
// Components are the multi-indices alpha = (ax, ay, az), |alpha| = n, in
// graded-lex order: descending ax, then descending ay.  For s = n - ax the
// position of (ax, ay) is s(s+1)/2 + (s - ay).  Component alpha stores the
// full-tensor entry, so contractions carry the multinomial weight
// mu_alpha = n! / (ax! ay! az!).
#pragma once

namespace ttm {

__host__ __device__ constexpr int ncomp3(int n) { return (n + 1) * (n + 2) / 2; }

__host__ __device__ constexpr int comp_index3(int n, int ax, int ay) {
  return (n - ax) * (n - ax + 1) / 2 + (n - ax - ay);
}

__host__ __device__ constexpr int factorial(int k) { return k <= 1 ? 1 : k * factorial(k - 1); }

template <int N>
struct Sym3 {
  static constexpr int K = ncomp3(N);
  int ax[K], ay[K], az[K];
  float mu[K];
  constexpr Sym3() : ax(), ay(), az(), mu() {
    int i = 0;
    for (int a = N; a >= 0; --a) {
      for (int b = N - a; b >= 0; --b) {
        ax[i] = a;
        ay[i] = b;
        az[i] = N - a - b;
        mu[i] = (float)(factorial(N) / (factorial(a) * factorial(b) * factorial(N - a - b)));
        ++i;
      }
    }
  }
};

}  // namespace ttm
