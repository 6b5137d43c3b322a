// HIP kernels of libperk for gfx950 behind the spectrum estimation of Sec. 4.1 (the Arnoldi
// iteration on the Jacobian of the right-hand side at the real mesh, steps 3-4): the
// orthogonalisation of a new Krylov vector against the basis (classical Gram-Schmidt, two
// passes) and the directional derivative of the right-hand side by central differences.
// Vectors are state arrays in slot layout; bases are stored column after column at stride ldv.

#include "perk_device.h"

namespace perk {
namespace {

constexpr int kDotThreads = 256;
constexpr int kDotChunks = 256;      // blocks per vector in the first reduction pass

// partial[j][c] = sum over chunk c of V_j . w (deterministic two-pass reduction)
__global__ __launch_bounds__(kDotThreads) void k_multi_dot(int k, const double* __restrict__ V, int64_t ldv,
                                                           const double* __restrict__ w, int64_t n,
                                                           double* __restrict__ partial) {
  __shared__ double red[kDotThreads / 64];
  const int j = blockIdx.y;
  const int c = blockIdx.x;
  const int64_t per = (n + kDotChunks - 1) / kDotChunks;
  const int64_t lo = (int64_t)c * per, hi = lo + per < n ? lo + per : n;
  const double* v = V + (int64_t)j * ldv;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kDotThreads) acc = fma(v[i], w[i], acc);
  // wave reduction, then across the block's waves
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kDotThreads / 64; ++q) s += red[q];
    partial[(int64_t)j * kDotChunks + c] = s;
  }
  (void)k;
}

// out[j] = sum_c partial[j][c]
__global__ void k_sum_chunks(int k, const double* __restrict__ partial, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double s = 0.0;
  for (int c = 0; c < kDotChunks; ++c) s += partial[(int64_t)j * kDotChunks + c];
  out[j] = s;
}

// w -= sum_j h_j V_j  (h on the device)
__global__ void k_multi_axpy(int k, const double* __restrict__ V, int64_t ldv, const double* __restrict__ h,
                             double* __restrict__ w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = w[i];
  for (int j = 0; j < k; ++j) acc = fma(-h[j], V[(int64_t)j * ldv + i], acc);
  w[i] = acc;
}

// y = x + s v
__global__ void k_axpy_to(double* __restrict__ y, const double* __restrict__ x, double s,
                          const double* __restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = fma(s, v[i], x[i]);
}

// y = (a - b) * s
__global__ void k_diff_scale(double* __restrict__ y, const double* __restrict__ a, const double* __restrict__ b,
                             double s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (a[i] - b[i]) * s;
}

}  // namespace

int64_t multi_dot_scratch_doubles(int k) { return (int64_t)k * kDotChunks + k; }

hipError_t launch_multi_dot(int k, const double* V, int64_t ldv, const double* w, int64_t n, double* scratch,
                            double* out, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_multi_dot, dim3(kDotChunks, k), dim3(kDotThreads), 0, s, k, V, ldv, w, n, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_chunks, dim3((k + 63) / 64), dim3(64), 0, s, k, scratch, out);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(int k, const double* V, int64_t ldv, const double* h, double* w, int64_t n,
                             hipStream_t s) {
  if (k <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_multi_axpy, dim3(grid_for(n, 256)), dim3(256), 0, s, k, V, ldv, h, w, n);
  return hipGetLastError();
}

hipError_t launch_axpy_to(double* y, const double* x, double sc, const double* v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_to, dim3(grid_for(n, 256)), dim3(256), 0, s, y, x, sc, v, n);
  return hipGetLastError();
}

hipError_t launch_diff_scale(double* y, const double* a, const double* b, double sc, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diff_scale, dim3(grid_for(n, 256)), dim3(256), 0, s, y, a, b, sc, n);
  return hipGetLastError();
}

}  // namespace perk
