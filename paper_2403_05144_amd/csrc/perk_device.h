// Device-side index helpers and the reciprocal shared by the libperk kernel files (gfx950).
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
