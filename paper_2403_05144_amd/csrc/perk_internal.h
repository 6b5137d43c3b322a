// Internal declarations shared by the host side (perk_api.cpp) and the HIP kernels
// (perk_stage.hip, perk_mesh.hip) of libperk.  Not part of the public ABI (see include/perk.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace perk {

constexpr int kMaxMembers = 8;    // R
constexpr int kMaxStages = 32;    // S
constexpr int kMaxLevels = 16;    // refinement levels of the forest
constexpr int kMaxDevices = 64;   // devices whose static scratch address is kept
// elements the allocation-free step-size bound accepts (its static per-device scratch holds one
// double per element plus the per-level maxima: 8 MiB + 128 B)
constexpr int kNoAllocMaxElements = 1 << 20;
constexpr int kMaxN = 4;          // nodes per direction (degree 3)

// Face kinds of an element face (Sec. 6.2: interfaces between equal cells, mortars at 2:1
// hanging faces).  Packed with the sub-face position of a fine element on its coarse face.
enum FaceKind : int32_t { kConforming = 0, kFineSide = 1, kCoarseSide = 2 };
__host__ __device__ inline int32_t pack_face(int kind, int s0, int s1) { return kind | (s0 << 2) | (s1 << 3); }
__host__ __device__ inline int face_kind(int32_t f) { return f & 3; }
__host__ __device__ inline int face_sub0(int32_t f) { return (f >> 2) & 1; }
__host__ __device__ inline int face_sub1(int32_t f) { return (f >> 3) & 1; }

// One-dimensional LGL operators for N nodes (N <= kMaxN), passed to kernels by value.
struct Ops {
  double D[kMaxN * kMaxN];          // D[i*N + j] = l_j'(x_i)
  double w[kMaxN];                  // quadrature weights
  double iw[kMaxN];                 // 1 / w (host division, the same correctly rounded value)
  double P[2][kMaxN * kMaxN];       // mortar interpolation to the lower/upper half
  double R[2][kMaxN * kMaxN];       // mortar projection: exact L2 projection of the half faces (R_0 P_0 + R_1 P_1 = I)
  double x[kMaxN];                  // nodes on [-1, 1]
  double Vinv[kMaxN * kMaxN];       // [k N + i]: coefficient of sqrt(k + 1/2) P_k in the interpolant of nodal values
  // device copy (caller's workspace, written at bind): [0, N^2) 2 D with a zero diagonal,
  // [N^2, 2 N^2) D, then P[0], P[1], R[0], R[1], Vinv (N^2 each).  Lane-indexed reads of the tables
  // above come from kernel-argument memory, which is far slower than this L2-resident copy.
  const double* dD;
};

struct Physics {
  double gamma;
  double mu;
  double kappa;    // gamma mu / ((gamma - 1) Pr), gas constant 1
};

// Connectivity of the slots (sorted element order).
struct Mesh {
  const int32_t* fk;      // [slot][2 dim] packed face kind
  const int32_t* fn;      // [slot][2 dim][4] neighbour slots
  const int32_t* lev;     // [slot] refinement level
  const int32_t* mem;     // [slot] P-ERK member
  int ld;                 // leading dimension of the slot layout (reserved capacity)
  int R;                  // members
  int bnd[kMaxMembers];   // slot ranges per member in slot order: [bnd[k-1], bnd[k]) holds member R-1-k
  double jac[kMaxLevels][3];   // 2 / h per level and direction
};

// Member of a slot from the partition boundaries (slots are sorted by member, so the boundaries
// are non-decreasing and the slot lies past a prefix of them).  Counted without an early exit:
// the boundaries are then read together instead of one dependent read per member.
__host__ __device__ inline int member_of_slot(const Mesh& m, int s) {
  int k = 0;
#pragma unroll
  for (int j = 0; j < kMaxMembers - 1; ++j) k += (j < m.R - 1 && s >= m.bnd[j]) ? 1 : 0;
  return m.R - 1 - k;
}

// Everything one stage launch needs.  Stage indices are 0-based here.
struct StageArgs {
  const double* U;        // U_n (slot layout)
  double* K1;             // K_1 (written at stage 0)
  const double* Yin;      // Y_i of elements whose member was active at stages i-1 and i
  double* Yout;           // host side: the classic pattern's next-stage buffer (kernels use Yw)
  double* ACC;            // running sum of b_j K_j over the stages with b_j != 0 before the last
  double* Uout;           // U_{n+1} at the last stage (may alias U)
  double* Kout;           // if non-null: K_i is written here and nothing else (right-hand side)
  double* Fv;             // BR1 viscous flux [dim][n_v][slot][node] (Navier-Stokes; written by the
                          // gradient kernel, read by the stage kernel)
  int32_t* evals;         // [slot] right-hand-side evaluations of the slot's element, or null
  int n_act;              // active elements of the launch: n_act
  int n_rng;              // they are the slots of n_rng ranges in order (0 or 1: [0, n_act)):
  int rng_start[kMaxMembers];   // range k begins at slot rng_start[k] and holds the active
  int rng_cum[kMaxMembers];     // indices [rng_cum[k], rng_cum[k + 1]) (rng_cum[0] = 0)
  int n_halo;             // Navier-Stokes gradient kernel only: extra slots listed in halo
  const int32_t* halo;
  double dt;
  double ci;              // c_i
  double bi;              // b_i (accumulated when acc_mode != 0)
  double bS;              // b_S (last stage)
  int first;              // stage 0
  int last;               // stage S-1
  int acc_mode;           // 0: nothing, 1: ACC = b_i K, 2: ACC += b_i K
  int use_acc_last;       // last stage adds ACC
  int src[kMaxMembers];   // where Y_i of a member comes from: 0 U_n, 1 Yin, 2 U_n + dt c_i K_1
  int src_bits;           // the same codes, two bits per member (member r at bits 2r, 2r+1)
  int read_acc;           // the epilogue reads ACC (acc_mode 2, or the last stage with use_acc_last)
  int wr[kMaxMembers];    // member writes its next stage value Y_k (k = i+1 for the classic
                          // pattern) into Yw[member]
  double a1[kMaxMembers]; // a_{k,1}
  double a2[kMaxMembers]; // a_{k,i}
  double* Yw[kMaxMembers];
  // subcell shock capturing (2D Euler; Hennemann et al.): on, cap and cut-off of the blending
  // factor, threshold T and slope s / T of its sigmoid
  int sc;
  double sc_amax, sc_amin, sc_T, sc_slope;
};

// Slot of the v-th active element of a launch (v < n_act): ranges are few (one per member at
// most) and the same for every lane of a block, so this is scalar work.
__host__ __device__ inline int active_slot(const StageArgs& a, int v) {
  int k = 0;
#pragma unroll
  for (int j = 1; j < kMaxMembers; ++j) k += (j < a.n_rng && v >= a.rng_cum[j]) ? 1 : 0;
  return a.rng_start[k] + (v - a.rng_cum[k]);
}

__host__ __device__ inline int src_of(const StageArgs& a, int member) { return (a.src_bits >> (2 * member)) & 3; }

// Arguments of the adjoint right-hand-side kernel: the stage state of every slot (as in the
// stage kernel: src 0 U_n, 1 Yin, 2 U_n + dt c_i K_1), the cotangent W of the slots [0, n_w)
// (zero elsewhere), the launched slots ([0, n_act) and halo[0..n_halo)), and what to do with
// G = F'(Y)^T W of a launched slot: store it (Gout), add it (Ubar += G, K1bar += dt A1 G) and
// form the previous stage's cotangent (Kprev = dt (bprev lam + A2 G)); null pointers skip.
struct VjpArgs {
  const double* U;
  const double* K1;
  const double* Yin;
  double dt;
  double ci;
  int src[kMaxMembers];
  const double* W;
  int n_w;
  int n_act;
  int n_halo;
  const int32_t* halo;
  double* Gout;
  double* Ubar;
  double* K1bar;
  double* Kprev;
  const double* lam;
  double bprev;
  double A1[kMaxMembers];
  double A2[kMaxMembers];
};

// One run of a batched launch: its mesh tables, operators, physics, polynomial degree (N nodes
// per direction), stage count and the index of its first stage descriptor (S consecutive).
struct BatchRun {
  Mesh m;
  Ops op;
  Physics ph;
  int N;
  int S;
  int sarg0;
};

// Kernel launch wrappers (perk_stage.hip: stage and gradient kernels; perk_mesh.hip: the rest).  All return hipError_t.
// ev0/ev1 (optional): events recorded by the dispatch itself at kernel start and end
hipError_t launch_stage(int dim, int N, bool viscous, const StageArgs& a, const Mesh& m, const Ops& op,
                        const Physics& ph, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Which kernel body launch_stage picks for a stage with n_act active elements (0: the default
// body; 1: the two-wave 2D p=3 body of small launches).
int stage_body_id(int dim, int N, int n_act, bool sc);
// BR1 gradient pass over slots [0, n_act) and the n_halo slots of `halo`: lifted gradients of
// w = (v, T) with central face values, then the viscous flux F_v at every node into a.Fv.
hipError_t launch_gradients(int dim, int N, const StageArgs& a, const Mesh& m, const Ops& op,
                            const Physics& ph, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

struct PartitionArgs {
  const int32_t* lev_leaf;       // [n] level per leaf
  int32_t* mem_leaf;             // [n] member per leaf (out)
  int32_t* slot_of_leaf;         // [n] (out)
  int32_t* leaf_of_slot;         // [n] (out)
  int32_t* counts;               // [R] (out)
  int n;
  int R;
  int member_of_level[kMaxLevels];
};
hipError_t launch_partition_sort(const PartitionArgs& a, hipStream_t s);

// Rebuild slot-order connectivity from leaf-order connectivity.
hipError_t launch_remap_connectivity(int n, int nfaces, const int32_t* leaf_of_slot, const int32_t* slot_of_leaf,
                                     const int32_t* fk_leaf, const int32_t* fn_leaf, const int32_t* lev_leaf,
                                     const int32_t* mem_leaf, int32_t* fk, int32_t* fn, int32_t* lev, int32_t* mem,
                                     hipStream_t s);
// dst[v][slot][node] = src[v][old_slot_of_leaf[leaf_of_slot[slot]]][node]; both with stride ld
hipError_t launch_permute_state(int n, int ld, int nv, int nd, const int32_t* leaf_of_slot,
                                const int32_t* old_slot_of_leaf, const double* src, double* dst, hipStream_t s);
// leaf layout [leaf][v][node] <-> slot layout [v][slot (stride ld)][node]
hipError_t launch_leaf_to_slot(int n, int ld, int nv, int nd, const int32_t* leaf_of_slot, const double* src,
                               double* dst, hipStream_t s);
hipError_t launch_slot_to_leaf(int n, int ld, int nv, int nd, const int32_t* slot_of_leaf, const double* src,
                               double* dst, hipStream_t s);

// AMR indicator per leaf: eta = h max_nodes |grad rho| / max_nodes rho (h = element size in x).
// Loehner's indicator per leaf on primitive variable var (0 rho, 1..dim velocity, dim+1 pressure)
// Hennemann-Gassner shock-capturing indicator as a refinement indicator (2D), per leaf.
hipError_t launch_indicator_hg(int dim, int N, int n, int ld, const int32_t* slot_of_leaf, const double* U,
                               const double* dD, double T, double slope, double* eta, hipStream_t s);
hipError_t launch_indicator_lohner(int dim, int N, int n, int ld, const int32_t* slot_of_leaf, const double* U,
                                   int var, double f_wave, double gamma, double* eta, hipStream_t s);
hipError_t launch_indicator(int dim, int N, int n, int ld, const int32_t* slot_of_leaf, const int32_t* lev_leaf,
                            const double* U, const Ops& op, const Mesh& m, double* eta_leaf, hipStream_t s);

// Projection of the state onto an adapted forest.  plan[new][10]: kind (0 copy, 1 child of a
// refined leaf, 2 parent of coarsened leaves), child position bits (kind 1), then the old leaf
// (kind 0/1) or the 2^dim old children ordered by child position (kind 2).  Reads the old state
// in slot layout through old_slot_of_leaf, writes the new state in leaf layout.
hipError_t launch_project(int dim, int N, int n_new, int ld, const int32_t* plan, const int32_t* old_slot_of_leaf,
                          const double* U_old, const Ops& op, double* dst_leaf, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
// Step-size bound with the per-slot and per-level scratch in the library's static per-device
// array (no allocation): dt[0] = cfl / max_l w_l (NaN if a speed is not finite or all are 0),
// beta[l] = 1 / w_l or 0 (beta may be null).  n in [1, kNoAllocMaxElements].
hipError_t launch_max_dt_noalloc(int dim, int N, int n, const double* U, const Physics& ph, const Mesh& m,
                                 double cfl, double* dt, double* beta, hipStream_t s);
// Tangent of the Euler right-hand side (perk_jvp.hip): T = F'(U) V, F = F(U) if F is not null,
// for the n element slots.
hipError_t launch_rhs_jvp(int dim, int N, int n, const double* U, const double* V, double* T, double* F,
                          const Mesh& m, const Ops& op, const Physics& ph, hipStream_t s);
// Spectrum estimation (perk_spectrum.hip): out[j] = V_j . w for the k columns of V (stride ldv),
// through a scratch of multi_dot_scratch_doubles(k) doubles; w -= sum_j h_j V_j (h on the
// device); y = x + s v; y = (a - b) s.
int64_t multi_dot_scratch_doubles(int k);
hipError_t launch_multi_dot(int k, const double* V, int64_t ldv, const double* w, int64_t n, double* scratch,
                            double* out, hipStream_t s);
hipError_t launch_multi_axpy(int k, const double* V, int64_t ldv, const double* h, double* w, int64_t n,
                             hipStream_t s);
hipError_t launch_axpy_to(double* y, const double* x, double sc, const double* v, int64_t n, hipStream_t s);
hipError_t launch_diff_scale(double* y, const double* a, const double* b, double sc, int64_t n, hipStream_t s);
// out[0, n) = ln x, out[n, 2n) = sqrt x, out[2n, 3n) = 1/x with the kernels' own routines
hipError_t launch_device_math(int64_t n, const double* x, double* out, hipStream_t s);
// Add the per-slot evaluation counts into per-member totals (member from the partition
// boundaries) and zero them.
// Per slot: max over nodes and directions of (N)(|v_d| + c) * (2/h_d) / 2; per level the maximum
// over its slots into beta[kMaxLevels] (0 for empty levels, NaN propagates).
hipError_t launch_wave_speed(int dim, int N, int n, const double* U, const Physics& ph, const Mesh& m, double* w_slot,
                             double* w_level, hipStream_t s);
// One batched stage tick over the runs k0 <= k < k1, all of N nodes per direction (2D Euler,
// N = 3 or 4): M in {1, 2, 4} elements of N = 4 per tile (2M of N = 3), grid blocks;
// tile_off [n_runs + 1] are the tick's tile offsets.  persistent: the grid loops over the
// tiles; otherwise grid must equal the tile count (one block per tile).
hipError_t launch_stage_batch(int N, int M, int grid, bool persistent, const BatchRun* runs, const StageArgs* sargs,
                              const int32_t* tile_off, int k0, int k1, int64_t tick, hipStream_t s);
// G = F'(Y)^T W for the Euler right-hand side (perk_adjoint.hip), one element per block
hipError_t launch_rhs_vjp(int dim, int N, const VjpArgs& a, const Mesh& m, const Ops& op, const Physics& ph,
                          hipStream_t s);
// y = alpha x
hipError_t launch_scale(double* y, const double* x, double alpha, int64_t n, hipStream_t s);
hipError_t launch_fold_evals(int n, const Mesh& m, int32_t* evals, unsigned long long* totals, hipStream_t s);

}  // namespace perk
