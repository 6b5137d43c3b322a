// Device-side index helpers and the arithmetic routines (reciprocal, square root, logarithm)
// shared by the libperk kernel files (gfx950).
#pragma once

#include "perk_internal.h"

namespace perk {
namespace {

// Reciprocal: hardware estimate refined by two Newton steps with FMA (within one ulp of 1/x for
// normal arguments away from the overflow range: densities, pressures, sums of them,
// wave-speed gaps, logarithms of ratios).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Square root of a non-negative argument (sound speeds): the hardware reciprocal-square-root
// estimate refined by two steps of Goldschmidt's coupled iteration for sqrt(x) and 1/(2 sqrt(x)),
// then one residual correction (correctly rounded in a host test over 2e7 arguments from
// estimates 2^-20 off).  The library square root scales the argument into range first, which
// positive normal sound-speed arguments do not need.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * y, g = x * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  return x == 0.0 ? 0.0 : g;
}

// Natural logarithm of a positive normal argument (node densities and inverse temperatures):
// x = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 artanh(f), f = (m - 1)/(m + 1), |f| <= 0.172,
// the artanh series through f^21 (truncation below 1e-18 relative), e ln 2 added with ln 2 split
// in two doubles.  Within 2 ulp of the correctly rounded logarithm in a host test over 2e7
// arguments; about half the instructions of the library logarithm.  Zero and negative
// arguments give NaN; subnormal ones are not expected here.
__device__ __forceinline__ double log_pos(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);   // [1/2, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0.70710678118654752440;
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double f = (m - 1.0) * rcp(m + 1.0), f2 = f * f;
  double s = 1.0 / 21;
  s = fma(s, f2, 1.0 / 19);
  s = fma(s, f2, 1.0 / 17);
  s = fma(s, f2, 1.0 / 15);
  s = fma(s, f2, 1.0 / 13);
  s = fma(s, f2, 1.0 / 11);
  s = fma(s, f2, 1.0 / 9);
  s = fma(s, f2, 1.0 / 7);
  s = fma(s, f2, 1.0 / 5);
  s = fma(s, f2, 1.0 / 3);
  const double t = 2.0 * f;
  const double lm = fma(t * f2, s, t);
  const double de = (double)e;
  const double r = fma(de, 0x1.62e42fefa39efp-1, fma(de, 0x1.abc9e3b39803fp-56, lm));
  return x > 0.0 ? r : __builtin_nan("");   // a non-physical state stays visible as NaN
}

template <int DIM, int N>
struct G {
  static constexpr int ND = DIM == 2 ? N * N : N * N * N;   // nodes per element
  static constexpr int NF = DIM == 2 ? N : N * N;           // nodes per face
  static constexpr int NFC = 2 * DIM;                       // faces per element
  static constexpr int NV = DIM + 2;                        // conserved variables
  static constexpr int NSUB = DIM == 2 ? 2 : 4;             // fine faces per mortar
  static constexpr int NQ = DIM + 5;                        // rho, v, p, ln rho, beta, ln beta
};

template <int DIM, int N>
__device__ __forceinline__ int node_index_dir(int nd, int d) {
  if (d == 0) return nd % N;
  if (d == 1) return (nd / N) % N;
  return nd / (N * N);
}

template <int DIM, int N>
__device__ __forceinline__ int stride_dir(int d) {
  return d == 0 ? 1 : (d == 1 ? N : N * N);
}

// volume node of face node j on face (d, side)
template <int DIM, int N>
__device__ __forceinline__ int face_node(int d, int side, int j) {
  const int sv = side ? N - 1 : 0;
  if (DIM == 2) return d == 0 ? sv + N * j : j + N * sv;
  const int a = j % N, b = j / N;
  if (d == 0) return sv + N * a + N * N * b;
  if (d == 1) return a + N * sv + N * N * b;
  return a + N * b + N * N * sv;
}

// face node index of volume node nd on a face normal to d
template <int DIM, int N>
__device__ __forceinline__ int face_index(int nd, int d) {
  const int i = nd % N, j = (nd / N) % N;
  if (DIM == 2) return d == 0 ? j : i;
  const int k = nd / (N * N);
  if (d == 0) return j + N * k;
  if (d == 1) return i + N * k;
  return i + N * j;
}

// index of the unordered pair (a, b), a < b, among the N(N-1)/2 pairs of a line
template <int N>
__device__ __forceinline__ int pair_index(int a, int b) {
  return a * (2 * N - a - 1) / 2 + (b - a - 1);
}

// line index of a node for direction d (the other coordinates) and its coordinate along d
template <int DIM, int N>
__device__ __forceinline__ void line_of(int nd, int d, int& line, int& pos) {
  const int i = nd % N, j = (nd / N) % N, k = DIM == 3 ? nd / (N * N) : 0;
  if (d == 0) { line = j + N * k; pos = i; }
  else if (d == 1) { line = i + N * k; pos = j; }
  else { line = i + N * j; pos = k; }
}

template <int DIM, int N>
__device__ __forceinline__ int node_on_line(int d, int line, int pos) {
  if (DIM == 2) return d == 0 ? pos + N * line : line + N * pos;
  const int a = line % N, b = line / N;
  if (d == 0) return pos + N * a + N * N * b;
  if (d == 1) return a + N * pos + N * N * b;
  return a + N * b + N * N * pos;
}

inline unsigned grid_for(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

}  // namespace
}  // namespace perk
