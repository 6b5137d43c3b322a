// HIP kernels of libperk for gfx950 around the stage kernel: re-partition (stable sort by
// member, connectivity remap, state permutation), leaf <-> slot layout changes, the AMR
// indicator and projection, the step-size bound and the evaluation counters.

#include <mutex>

#include "perk_device.h"

namespace perk {

// Scratch of the allocation-free step-size bound (pe_max_dt_noalloc): per-slot wave speeds in
// [0, kNoAllocMaxElements), per-level maxima in the kMaxLevels doubles after them.  Each device
// holds its own copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (noalloc_scratch).
static __device__ __align__(256) double scratch[kNoAllocMaxElements + kMaxLevels];

namespace {

// ------------------------------------------------------------------------------------------
// Re-partition (Sec. 6.2): member per leaf, stable counting sort by member (most stage
// evaluations first), one block of 1024 lanes; ranks inside a chunk from wave ballots.
// ------------------------------------------------------------------------------------------
constexpr int kSortThreads = 1024;

__global__ __launch_bounds__(kSortThreads) void k_partition_sort(PartitionArgs a) {
  __shared__ int s_count[kMaxMembers];
  __shared__ int s_base[kMaxMembers];
  __shared__ int s_wave[kMaxMembers][kSortThreads / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  if (tid < kMaxMembers) s_count[tid] = 0;
  __syncthreads();
  for (int i = tid; i < a.n; i += kSortThreads) {
    const int mem = a.member_of_level[a.lev_leaf[i]];
    a.mem_leaf[i] = mem;
    atomicAdd(&s_count[a.R - 1 - mem], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int k = 0; k < a.R; ++k) {
      s_base[k] = acc;
      acc += s_count[k];
      a.counts[a.R - 1 - k] = s_count[k];
    }
  }
  __syncthreads();
  for (int c0 = 0; c0 < a.n; c0 += kSortThreads) {
    const int i = c0 + tid;
    const int key = i < a.n ? a.R - 1 - a.mem_leaf[i] : -1;
    int my_rank = 0;
    for (int k = 0; k < a.R; ++k) {
      const unsigned long long mask = __ballot(key == k);
      if (lane == 0) s_wave[k][wave] = __popcll(mask);
      if (key == k) my_rank = __popcll(mask & ((1ull << lane) - 1ull));
    }
    __syncthreads();
    if (key >= 0) {
      int before = 0;
      for (int w = 0; w < wave; ++w) before += s_wave[key][w];
      const int slot = s_base[key] + before + my_rank;
      a.slot_of_leaf[i] = slot;
      a.leaf_of_slot[slot] = i;
    }
    __syncthreads();
    if (tid < a.R) {
      int tot = 0;
      for (int w = 0; w < kSortThreads / 64; ++w) tot += s_wave[tid][w];
      s_base[tid] += tot;
    }
    __syncthreads();
  }
}

__global__ void k_remap(int n, int nfaces, const int32_t* leaf_of_slot, const int32_t* slot_of_leaf,
                        const int32_t* fk_leaf, const int32_t* fn_leaf, const int32_t* lev_leaf,
                        const int32_t* mem_leaf, int32_t* fk, int32_t* fn, int32_t* lev, int32_t* mem) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * nfaces) return;
  const int slot = (int)(t / nfaces), f = (int)(t % nfaces);
  const int leaf = leaf_of_slot[slot];
  fk[t] = fk_leaf[(int64_t)leaf * nfaces + f];
  for (int q = 0; q < 4; ++q) {
    const int nb = fn_leaf[((int64_t)leaf * nfaces + f) * 4 + q];
    fn[t * 4 + q] = nb >= 0 ? slot_of_leaf[nb] : -1;
  }
  if (f == 0) {
    lev[slot] = lev_leaf[leaf];
    mem[slot] = mem_leaf[leaf];
  }
}

__global__ void k_permute(int64_t total, int n, int ld, int nd, const int32_t* leaf_of_slot,
                          const int32_t* old_slot_of_leaf, const double* src, double* dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int node = (int)(t % nd);
  const int64_t r = t / nd;
  const int slot = (int)(r % n);
  const int v = (int)(r / n);
  const int old = old_slot_of_leaf[leaf_of_slot[slot]];
  dst[((int64_t)v * ld + slot) * nd + node] = src[((int64_t)v * ld + old) * nd + node];
}

__global__ void k_leaf_to_slot(int64_t total, int n, int ld, int nv, int nd, const int32_t* leaf_of_slot,
                               const double* src, double* dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int node = (int)(t % nd);
  const int64_t r = t / nd;
  const int slot = (int)(r % n);
  const int v = (int)(r / n);
  dst[((int64_t)v * ld + slot) * nd + node] = src[((int64_t)leaf_of_slot[slot] * nv + v) * nd + node];
}

__global__ void k_slot_to_leaf(int64_t total, int ld, int nv, int nd, const int32_t* slot_of_leaf,
                               const double* src, double* dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int node = (int)(t % nd);
  const int64_t r = t / nd;
  const int v = (int)(r % nv);
  const int leaf = (int)(r / nv);
  dst[t] = src[((int64_t)v * ld + slot_of_leaf[leaf]) * nd + node];
}

// eta = h max |grad rho| / max rho over the nodes of one leaf; one lane per leaf.
template <int DIM, int N>
__global__ void k_indicator(int n, int ld, const int32_t* slot_of_leaf, const int32_t* lev_leaf, const double* U,
                            Ops op, Mesh m, double* eta) {
  constexpr int ND = G<DIM, N>::ND;
  const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
  if (leaf >= n) return;
  const int slot = slot_of_leaf[leaf];
  const int lev = lev_leaf[leaf];
  const double* rho = U + (int64_t)slot * ND;     // variable 0
  double rmax = 0.0, gmax = 0.0;
  for (int nd = 0; nd < ND; ++nd) {
    rmax = fmax(rmax, rho[nd]);
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int ia = node_index_dir<DIM, N>(nd, d);
      const int st = stride_dir<DIM, N>(d);
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < N; ++q) acc += op.D[ia * N + q] * rho[nd + (q - ia) * st];
      const double gd = m.jac[lev][d] * acc;
      g2 += gd * gd;
    }
    gmax = fmax(gmax, sqrt(g2));
  }
  const double h = 2.0 / m.jac[lev][0];
  eta[leaf] = h * gmax / rmax;
}

// Loehner's indicator on a primitive variable (0 rho, 1..DIM velocity, DIM+1 pressure): the
// largest |q_{i+1} - 2 q_i + q_{i-1}| / (|q_{i+1} - q_i| + |q_i - q_{i-1}| + f_wave (|q_{i+1}| +
// 2 |q_i| + |q_{i-1}|)) over the interior nodes of every coordinate line of the leaf's LGL nodes
// (0 where the denominator vanishes); one lane per leaf.
template <int DIM, int N>
__global__ void k_indicator_lohner(int n, int ld, const int32_t* slot_of_leaf, const double* U, int var,
                                   double f_wave, double gamma, double* eta) {
  constexpr int ND = G<DIM, N>::ND, NV = DIM + 2;
  const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
  if (leaf >= n) return;
  const int slot = slot_of_leaf[leaf];
  double q[ND];
#pragma unroll
  for (int nd = 0; nd < ND; ++nd) {
    const double rho = U[(int64_t)slot * ND + nd];
    double val = rho;
    if (var >= 1 && var <= DIM) {
      val = U[((int64_t)var * ld + slot) * ND + nd] / rho;
    } else if (var == DIM + 1) {
      double ke = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double m = U[((int64_t)(1 + d) * ld + slot) * ND + nd];
        ke += m * m;
      }
      val = (gamma - 1.0) * (U[((int64_t)(NV - 1) * ld + slot) * ND + nd] - 0.5 * ke / rho);
    }
    q[nd] = val;
  }
  double best = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int st = stride_dir<DIM, N>(d);
#pragma unroll
    for (int nd = 0; nd < ND; ++nd) {
      const int ia = node_index_dir<DIM, N>(nd, d);
      if (ia == 0 || ia == N - 1) continue;
      const double um = q[nd - st], u0 = q[nd], up = q[nd + st];
      const double num = fabs(up - 2.0 * u0 + um);
      const double den = fabs(up - u0) + fabs(u0 - um) + f_wave * (fabs(up) + 2.0 * fabs(u0) + fabs(um));
      const double e = den > 0.0 ? num / den : 0.0;
      best = e > best ? e : best;
    }
  }
  eta[leaf] = best;
}

// Shock-capturing indicator of Hennemann et al. used as a refinement indicator (the paper's
// Kelvin-Helmholtz run, Sec. 7.2.1): the density's coefficients in the orthonormal Legendre
// basis (Vinv, the seventh operator table, applied along each direction in turn), the energy
// share of the top modes E = max((all - clip_1)/all, (clip_1 - clip_2)/clip_1) (clip_k: modes of
// degree <= p - k in each direction) and the blending sigmoid 1/(1 + exp(-slope (E - T)))
// without cut-off or cap; one lane per leaf.
template <int N>
__global__ void k_indicator_hg(int n, const int32_t* slot_of_leaf, const double* U, const double* dD, double T,
                               double slope, double* eta) {
  constexpr int ND = N * N;
  const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
  if (leaf >= n) return;
  const int slot = slot_of_leaf[leaf];
  const double* Vi = dD + 6 * N * N;
  double q[ND], r[ND];
#pragma unroll
  for (int nd = 0; nd < ND; ++nd) q[nd] = U[(int64_t)slot * ND + nd];   // variable 0: the density
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) acc += Vi[a * N + i] * q[i + N * b];
      r[a + N * b] = acc;
    }
  double tot = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double m = 0.0;
#pragma unroll
      for (int j = 0; j < N; ++j) m += Vi[b * N + j] * r[a + N * j];
      const int deg = a > b ? a : b;
      const double m2 = m * m;
      tot += m2;
      if (deg <= N - 2) c1 += m2;
      if (deg <= N - 3) c2 += m2;
    }
  const double e1 = tot > 0.0 ? (tot - c1) / tot : 0.0;
  const double e2 = c1 > 0.0 ? (c1 - c2) / c1 : 0.0;
  const double E = e1 < e2 ? e2 : e1;
  eta[leaf] = 1.0 / (1.0 + exp(-slope * (E - T)));
}

// Largest convective wave speed per slot, scaled to the step-size bound of eq. (CFL_DG):
// w_e = max over nodes and directions of (k+1)(|v_d| + c) / h_d, one lane per slot.
template <int DIM, int N>
__global__ void k_wave_speed(int n, int ld, const double* U, Physics ph, Mesh m, double* w) {
  constexpr int ND = G<DIM, N>::ND, NV = DIM + 2;
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= n) return;
  const int lev = m.lev[slot];
  double wmax = 0.0;
  for (int nd = 0; nd < ND; ++nd) {
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[((int64_t)v * ld + slot) * ND + nd];
    const double ir = 1.0 / u[0];
    double ke = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) ke += u[1 + d] * u[1 + d];
    const double p = (ph.gamma - 1.0) * (u[NV - 1] - 0.5 * ke * ir);
    const double c = sqrt(ph.gamma * p * ir);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double s = (fabs(u[1 + d] * ir) + c) * (0.5 * N * m.jac[lev][d]);
      wmax = (s > wmax || s != s) ? s : wmax;      // NaN wins, so a broken state is reported
    }
  }
  w[slot] = wmax;
}

// Maximum per level over the slots; one block.  Non-negative doubles order like their bit
// patterns, and NaN's pattern is above +inf, so an integer maximum keeps NaN.
__global__ void k_level_max(int n, const int32_t* lev, const double* w, double* out) {
  __shared__ unsigned long long sm[kMaxLevels];
  if (threadIdx.x < kMaxLevels) sm[threadIdx.x] = 0ull;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double x = w[i];
    const unsigned long long b = x != x ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(x);
    atomicMax(&sm[lev[i]], b);
  }
  __syncthreads();
  if (threadIdx.x < kMaxLevels) out[threadIdx.x] = __longlong_as_double((long long)sm[threadIdx.x]);
}

// one lane per (new leaf, variable, node)
template <int DIM, int N>
__global__ void k_project(int64_t total, int ld, const int32_t* plan, const int32_t* old_slot_of_leaf,
                          const double* U, Ops op, double* dst) {
  constexpr int ND = G<DIM, N>::ND, NV = DIM + 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int node = (int)(t % ND);
  const int64_t r = t / ND;
  const int v = (int)(r % NV);
  const int leaf = (int)(r / NV);
  const int32_t* pl = plan + (int64_t)leaf * 10;
  const int kind = pl[0];
  int j[3] = {node % N, (node / N) % N, DIM == 3 ? node / (N * N) : 0};
  double val = 0.0;
  if (kind == 0) {
    const int slot = old_slot_of_leaf[pl[2]];
    val = U[((int64_t)v * ld + slot) * ND + node];
  } else if (kind == 1) {
    // child of a refined leaf: tensor-product interpolation of the parent polynomial
    const int pos = pl[1];
    const int slot = old_slot_of_leaf[pl[2]];
    const double* src = U + ((int64_t)v * ld + slot) * ND;
    for (int q = 0; q < ND; ++q) {
      const int k[3] = {q % N, (q / N) % N, DIM == 3 ? q / (N * N) : 0};
      double w = 1.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) w *= op.P[(pos >> d) & 1][j[d] * N + k[d]];
      val += w * src[q];
    }
  } else {
    // parent of a coarsened family: LGL-quadrature L2 projection of the children
    for (int c = 0; c < (1 << DIM); ++c) {
      const int slot = old_slot_of_leaf[pl[2 + c]];
      const double* src = U + ((int64_t)v * ld + slot) * ND;
      for (int q = 0; q < ND; ++q) {
        const int k[3] = {q % N, (q / N) % N, DIM == 3 ? q / (N * N) : 0};
        double w = 1.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) w *= op.R[(c >> d) & 1][j[d] * N + k[d]];
        val += w * src[q];
      }
    }
  }
  dst[t] = val;
}

// The kernels' own arithmetic routines on n arguments: OP 0 logarithm, 1 square root, 2 reciprocal.
template <int OP>
__global__ void k_device_math(int64_t n, const double* x, double* y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double v = x[t];
  y[t] = OP == 0 ? log_pos(v) : (OP == 1 ? sqrt_pos(v) : rcp(v));
}

// dt = cfl / max_l w_l and beta_l = 1 / w_l (0 for levels without elements) on the device; dt is
// NaN when a level's speed is not finite or every level's speed is zero.
__global__ void k_dt_from_levels(const double* w_level, double cfl, double* dt, double* beta) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double wmax = 0.0;
  bool finite = true;
  for (int l = 0; l < kMaxLevels; ++l) {
    const double w = w_level[l];
    finite = finite && (w - w == 0.0);
    wmax = w > wmax ? w : wmax;
    if (beta) beta[l] = w > 0.0 ? 1.0 / w : 0.0;
  }
  *dt = (finite && wmax > 0.0) ? cfl / wmax : __builtin_nan("");
}

__global__ void k_copy(double* dst, const double* src, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

__global__ __launch_bounds__(1024) void k_fold_evals(int n, Mesh m, int32_t* evals, unsigned long long* totals) {
  __shared__ unsigned long long s_tot[kMaxMembers];
  if (threadIdx.x < kMaxMembers) s_tot[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long mine[kMaxMembers] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    mine[member_of_slot(m, i)] += (unsigned long long)evals[i];
    evals[i] = 0;
  }
  for (int r = 0; r < m.R; ++r)
    if (mine[r]) atomicAdd(&s_tot[r], mine[r]);
  __syncthreads();
  if (threadIdx.x < m.R) totals[threadIdx.x] += s_tot[threadIdx.x];
}

}  // namespace

hipError_t launch_partition_sort(const PartitionArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_partition_sort, dim3(1), dim3(kSortThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_remap_connectivity(int n, int nfaces, const int32_t* leaf_of_slot, const int32_t* slot_of_leaf,
                                     const int32_t* fk_leaf, const int32_t* fn_leaf, const int32_t* lev_leaf,
                                     const int32_t* mem_leaf, int32_t* fk, int32_t* fn, int32_t* lev, int32_t* mem,
                                     hipStream_t s) {
  const int64_t total = (int64_t)n * nfaces;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_remap, dim3(grid_for(total, 256)), dim3(256), 0, s, n, nfaces, leaf_of_slot, slot_of_leaf,
                     fk_leaf, fn_leaf, lev_leaf, mem_leaf, fk, fn, lev, mem);
  return hipGetLastError();
}

hipError_t launch_permute_state(int n, int ld, int nv, int nd, const int32_t* leaf_of_slot,
                                const int32_t* old_slot_of_leaf, const double* src, double* dst, hipStream_t s) {
  const int64_t total = (int64_t)n * nv * nd;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute, dim3(grid_for(total, 256)), dim3(256), 0, s, total, n, ld, nd, leaf_of_slot,
                     old_slot_of_leaf, src, dst);
  return hipGetLastError();
}

hipError_t launch_leaf_to_slot(int n, int ld, int nv, int nd, const int32_t* leaf_of_slot, const double* src,
                               double* dst, hipStream_t s) {
  const int64_t total = (int64_t)n * nv * nd;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_leaf_to_slot, dim3(grid_for(total, 256)), dim3(256), 0, s, total, n, ld, nv, nd,
                     leaf_of_slot, src, dst);
  return hipGetLastError();
}

hipError_t launch_slot_to_leaf(int n, int ld, int nv, int nd, const int32_t* slot_of_leaf, const double* src,
                               double* dst, hipStream_t s) {
  const int64_t total = (int64_t)n * nv * nd;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_to_leaf, dim3(grid_for(total, 256)), dim3(256), 0, s, total, ld, nv, nd, slot_of_leaf,
                     src, dst);
  return hipGetLastError();
}

hipError_t launch_indicator_lohner(int dim, int N, int n, int ld, const int32_t* slot_of_leaf, const double* U,
                                   int var, double f_wave, double gamma, double* eta, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 g(grid_for(n, 128)), b(128);
  if (dim == 2 && N == 4)
    hipLaunchKernelGGL((k_indicator_lohner<2, 4>), g, b, 0, s, n, ld, slot_of_leaf, U, var, f_wave, gamma, eta);
  else if (dim == 2 && N == 3)
    hipLaunchKernelGGL((k_indicator_lohner<2, 3>), g, b, 0, s, n, ld, slot_of_leaf, U, var, f_wave, gamma, eta);
  else if (dim == 3 && N == 4)
    hipLaunchKernelGGL((k_indicator_lohner<3, 4>), g, b, 0, s, n, ld, slot_of_leaf, U, var, f_wave, gamma, eta);
  else if (dim == 3 && N == 3)
    hipLaunchKernelGGL((k_indicator_lohner<3, 3>), g, b, 0, s, n, ld, slot_of_leaf, U, var, f_wave, gamma, eta);
  else
    return hipErrorNotSupported;
  return hipGetLastError();
}

hipError_t launch_indicator_hg(int dim, int N, int n, int ld, const int32_t* slot_of_leaf, const double* U,
                               const double* dD, double T, double slope, double* eta, hipStream_t s) {
  (void)ld;   // the density is variable 0: slot-major within its slice
  if (n == 0) return hipSuccess;
  const dim3 g(grid_for(n, 128)), b(128);
  if (dim == 2 && N == 4)
    hipLaunchKernelGGL((k_indicator_hg<4>), g, b, 0, s, n, slot_of_leaf, U, dD, T, slope, eta);
  else if (dim == 2 && N == 3)
    hipLaunchKernelGGL((k_indicator_hg<3>), g, b, 0, s, n, slot_of_leaf, U, dD, T, slope, eta);
  else
    return hipErrorNotSupported;
  return hipGetLastError();
}

hipError_t launch_indicator(int dim, int N, int n, int ld, const int32_t* slot_of_leaf, const int32_t* lev_leaf,
                            const double* U, const Ops& op, const Mesh& m, double* eta, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 g(grid_for(n, 128)), b(128);
  if (dim == 2 && N == 4) hipLaunchKernelGGL((k_indicator<2, 4>), g, b, 0, s, n, ld, slot_of_leaf, lev_leaf, U, op, m, eta);
  else if (dim == 2 && N == 3) hipLaunchKernelGGL((k_indicator<2, 3>), g, b, 0, s, n, ld, slot_of_leaf, lev_leaf, U, op, m, eta);
  else if (dim == 3 && N == 4) hipLaunchKernelGGL((k_indicator<3, 4>), g, b, 0, s, n, ld, slot_of_leaf, lev_leaf, U, op, m, eta);
  else if (dim == 3 && N == 3) hipLaunchKernelGGL((k_indicator<3, 3>), g, b, 0, s, n, ld, slot_of_leaf, lev_leaf, U, op, m, eta);
  else return hipErrorNotSupported;
  return hipGetLastError();
}

hipError_t launch_project(int dim, int N, int n_new, int ld, const int32_t* plan, const int32_t* old_slot_of_leaf,
                          const double* U_old, const Ops& op, double* dst, hipStream_t s) {
  const int nd = dim == 2 ? N * N : N * N * N;
  const int64_t total = (int64_t)n_new * (dim + 2) * nd;
  if (total == 0) return hipSuccess;
  const dim3 g(grid_for(total, 256)), b(256);
  if (dim == 2 && N == 4) hipLaunchKernelGGL((k_project<2, 4>), g, b, 0, s, total, ld, plan, old_slot_of_leaf, U_old, op, dst);
  else if (dim == 2 && N == 3) hipLaunchKernelGGL((k_project<2, 3>), g, b, 0, s, total, ld, plan, old_slot_of_leaf, U_old, op, dst);
  else if (dim == 3 && N == 4) hipLaunchKernelGGL((k_project<3, 4>), g, b, 0, s, total, ld, plan, old_slot_of_leaf, U_old, op, dst);
  else if (dim == 3 && N == 3) hipLaunchKernelGGL((k_project<3, 3>), g, b, 0, s, total, ld, plan, old_slot_of_leaf, U_old, op, dst);
  else return hipErrorNotSupported;
  return hipGetLastError();
}

hipError_t launch_wave_speed(int dim, int N, int n, const double* U, const Physics& ph, const Mesh& m, double* w_slot,
                             double* w_level, hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  const dim3 g(grid_for(n, 128)), b(128);
  if (dim == 2 && N == 4) hipLaunchKernelGGL((k_wave_speed<2, 4>), g, b, 0, s, n, m.ld, U, ph, m, w_slot);
  else if (dim == 2 && N == 3) hipLaunchKernelGGL((k_wave_speed<2, 3>), g, b, 0, s, n, m.ld, U, ph, m, w_slot);
  else if (dim == 3 && N == 4) hipLaunchKernelGGL((k_wave_speed<3, 4>), g, b, 0, s, n, m.ld, U, ph, m, w_slot);
  else if (dim == 3 && N == 3) hipLaunchKernelGGL((k_wave_speed<3, 3>), g, b, 0, s, n, m.ld, U, ph, m, w_slot);
  else return hipErrorNotSupported;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_level_max, dim3(1), dim3(1024), 0, s, n, m.lev, w_slot, w_level);
  return hipGetLastError();
}

hipError_t launch_fold_evals(int n, const Mesh& m, int32_t* evals, unsigned long long* totals, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_evals, dim3(1), dim3(1024), 0, s, n, m, evals, totals);
  return hipGetLastError();
}

hipError_t noalloc_scratch(double** out) {
  static std::mutex mu;
  static double* ptrs[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    // once per device, with that device current: the device address of this device's copy
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptrs[dev] = static_cast<double*>(p);
  }
  *out = ptrs[dev];
  return hipSuccess;
}

hipError_t launch_max_dt_noalloc(int dim, int N, int n, const double* U, const Physics& ph, const Mesh& m,
                                 double cfl, double* dt, double* beta, hipStream_t s) {
  if (n <= 0 || n > kNoAllocMaxElements) return hipErrorInvalidValue;
  double* base = nullptr;
  hipError_t e = noalloc_scratch(&base);
  if (e != hipSuccess) return e;
  // every scratch value read below is written first by the same call: w_slot[0, n) by the wave
  // speed kernel, all kMaxLevels maxima by the level kernel
  e = launch_wave_speed(dim, N, n, U, ph, m, base, base + kNoAllocMaxElements, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dt_from_levels, dim3(1), dim3(64), 0, s, base + kNoAllocMaxElements, cfl, dt, beta);
  return hipGetLastError();
}

hipError_t launch_device_math(int64_t n, const double* x, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 g(grid_for(n, 256)), b(256);
  hipLaunchKernelGGL(k_device_math<0>, g, b, 0, s, n, x, out);
  hipLaunchKernelGGL(k_device_math<1>, g, b, 0, s, n, x, out + n);
  hipLaunchKernelGGL(k_device_math<2>, g, b, 0, s, n, x, out + 2 * n);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

}  // namespace perk
