// sym_tables.hpp -- compile-time index tables of degree-n symmetric tensors
// over R^3 (the d' = 3 template-axis form) and over R^4 (the quaternion form).
//
// d' = 3: components are the multi-indices alpha = (ax, ay, az), |alpha| = n,
// in graded-lex order: descending ax, then descending ay.  For s = n - ax the
// position of (ax, ay) is s(s+1)/2 + (s - ay).  Component alpha stores the
// full-tensor entry, so contractions carry the multinomial weight
// mu_alpha = n! / (ax! ay! az!).
// d' = 4: alpha = (aw, ax, ay, az) in graded-lex order (descending aw, then
// ax, then ay); K = binom(n + 3, 3); mu_alpha = n! / (aw! ax! ay! az!).
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

__host__ __device__ constexpr int ncomp4(int n) { return (n + 1) * (n + 2) * (n + 3) / 6; }

// Position of (a, b, c, n - a - b - c): the tuples with a larger first count
// come first (binom(n - a + 2, 3) of them), then those with the same a and a
// larger second count, then those with a larger third count.
__host__ __device__ constexpr int comp_index4(int n, int a, int b, int c) {
  return (n - a + 2) * (n - a + 1) * (n - a) / 6 + (n - a - b) * (n - a - b + 1) / 2 + (n - a - b - c);
}

__host__ __device__ constexpr int multinom4(int a, int b, int c, int d) {
  return factorial(a + b + c + d) / (factorial(a) * factorial(b) * factorial(c) * factorial(d));
}

template <int N>
struct Sym4 {
  static constexpr int K = ncomp4(N);
  int e[K > 0 ? K : 1][4];
  float mu[K > 0 ? K : 1];
  constexpr Sym4() : e(), mu() {
    int i = 0;
    for (int a = N; a >= 0; --a)
      for (int b = N - a; b >= 0; --b)
        for (int c = N - a - b; c >= 0; --c) {
          e[i][0] = a;
          e[i][1] = b;
          e[i][2] = c;
          e[i][3] = N - a - b - c;
          mu[i] = (float)multinom4(a, b, c, N - a - b - c);
          ++i;
        }
  }
};

}  // namespace ttm
