// Host side of libperk: the C ABI of include/perk.h.
//
// Responsibilities: forest connectivity from a leaf list (periodic neighbour search,
// conforming faces, 2:1 mortars; Sec. 6.2), LGL operators, validation of the P-ERK family
// (Sec. 2.1-2.4, 3.1, 3.3), per-stage tables (which members evaluate stage i, where their
// stage values come from, the Butcher coefficients of the next stage value), the workspace
// carve-up of caller-owned device memory, and the orchestration of the device re-partition
// and of the stage launches.  No floating-point work of the time step runs on the host.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <chrono>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/perk.h"
#include "perk_internal.h"

using namespace perk;

struct pe_ctx {
  // physics
  int dim = 2, degree = 3, N = 4, equations = 0;
  Physics ph{};
  Ops ops{};
  // mesh (leaf order)
  bool have_mesh = false;
  int n_root[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  std::vector<int32_t> leaves;          // [n][4]
  std::vector<int32_t> fk_leaf, fn_leaf, lev_leaf;
  std::vector<int32_t> own_cells;       // connectivity scratch: owner leaf of every finest-level cell
  int n_e = 0, max_level = 0;
  int64_t capacity = 0;                 // reserved elements (leading dimension of the slot layout)
  // coefficients
  bool have_coeffs = false;
  int order = 2, R = 1, S = 1;
  std::vector<int32_t> E;
  std::vector<double> c, b, a_sub;      // a_sub [R][S]: a_{i,j} of row i's coupling column j
  // stage-evaluation pattern (Sec. 3.2.4).  Classic families (no coupling table given) couple
  // row i to column i-1 and keep two alternating stage buffers; a general pattern gives per
  // member and row the coupling column cpl[r][i] (-1: none), uses[r][j] is the row coupling
  // K_j (-1: none), and the stage values go to the buffers ybuf_of_stage assigns
  bool general = false;
  std::vector<int> cpl, uses;           // [R][S]
  std::vector<int> ybuf_of_stage;       // [S] (general pattern)
  int n_ybuf = 2;                       // stage buffers the coefficients need
  int n_ybuf_bound = 0;                 // stage buffers carved at the last bind
  std::vector<double*> ybuf;            // Ya, Yb, then the extra ones
  // level -> member rule applied when pe_partition / pe_amr_cycle get no explicit map
  bool have_rule = true;
  int rule = PE_LEVEL_RULE_PAPER;
  std::vector<double> rule_dt_opt;      // [R] optimal steps at a common element size (required-step rule)
  double rule_margin = 1.0;
  // refinement indicator of pe_amr_indicator / pe_amr_cycle
  int ind_kind = PE_INDICATOR_DENSITY_GRADIENT, ind_var = 1;
  // subcell shock capturing (2D Euler)
  bool sc_on = false;
  double sc_amax = 0.5, sc_amin = 0.001;
  double ind_fwave = 0.2;
  // binding
  bool bound = false;
  double* U = nullptr;
  char* ws = nullptr;
  double *K1 = nullptr, *Ya = nullptr, *Yb = nullptr, *ACC = nullptr, *Tmp = nullptr, *Fv = nullptr;
  int32_t *d_fk_leaf = nullptr, *d_fn_leaf = nullptr, *d_lev_leaf = nullptr;
  int32_t *d_fk = nullptr, *d_fn = nullptr, *d_lev = nullptr, *d_mem = nullptr, *d_mem_leaf = nullptr;
  int32_t *d_slot_of_leaf = nullptr, *d_leaf_of_slot = nullptr, *d_old_slot_of_leaf = nullptr, *d_counts = nullptr;
  int32_t* d_halo = nullptr;
  int32_t* d_plan = nullptr;            // AMR projection plan [capacity][10]
  double* d_eta = nullptr;              // AMR indicator per leaf; wave-speed bound per slot
  double* d_beta = nullptr;             // [kMaxLevels] largest (p+1)(|v_d|+c)/h_d per level
  double* d_dmat = nullptr;             // [7][N^2] operator tables (Ops::dD)
  unsigned long long* d_counter = nullptr;   // [R] folded totals
  int32_t* d_evals = nullptr;               // [capacity] per-slot evaluations since the last fold
  // partition
  bool partitioned = false;
  bool state_valid = false;
  bool pending_leaf_state = false;      // adapted state waiting in Tmp (leaf layout)
  std::vector<int32_t> counts;          // [R] elements per member
  std::vector<int32_t> leaf_of_slot, slot_of_leaf, mem_of_slot;
  std::vector<int> n_act;               // [S]
  std::vector<std::vector<std::pair<int, int>>> act_rng;   // [S] active slots as (first, count) ranges
  std::vector<int> halo_off, halo_cnt;  // [S] inactive face neighbours of the active prefix per stage
  bool halo_valid = false;              // built for Navier-Stokes at partition, on demand for the adjoint
  // adjoint workspace (caller-owned device memory): stage values Y_1..Y_{S-1}, stage cotangents
  char* adj_ws = nullptr;
  int adj_S = 0;
  int64_t adj_cap = 0;
  // replay of one captured step (HIP graph), valid until the partition, binding or dt changes
  bool graphs_enabled = true;
  bool graph_valid = false;
  double graph_dt = 0.0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int> graph_bodies;        // kernel body of every stage launch in gexec (stage_body_id)
  bool maps_on_host = false;            // leaf_of_slot / slot_of_leaf / mem_of_slot copied back
  // optional per-launch timing of the stage and gradient kernels with HIP events on the launch
  // stream; ev_kind[k] names the kernel of event pair k (0 stage, 1 gradient)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
  // kernel 2: re-partitions inside pe_amr_cycle (host call and its kernels, serialised)
  int64_t prof_launches[3] = {0, 0, 0}, prof_elems[3] = {0, 0, 0};
  double prof_ms[3] = {0.0, 0.0, 0.0};
  // pinned host staging of the adaptation's uploads and the indicator's download (grown on
  // demand); `stage_ev` marks the end of the last transfer out of it still in flight
  void* h_stage = nullptr;
  size_t h_stage_cap = 0;
  hipEvent_t stage_ev = nullptr;
  bool stage_pending = false;
  std::string err;
  ~pe_ctx() {
    if (stage_ev) (void)hipEventSynchronize(stage_ev);
    if (h_stage) (void)hipHostFree(h_stage);
    if (stage_ev) (void)hipEventDestroy(stage_ev);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace {

pe_status fail(pe_ctx* c, pe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

pe_status hip_check(pe_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(c, PE_EHIP, "%s: %s", what, hipGetErrorString(e));
  return PE_OK;
}

#define HIPCHK(call)                                   \
  do {                                                 \
    pe_status _st = hip_check(ctx, (call), #call);     \
    if (_st != PE_OK) return _st;                      \
  } while (0)

// ---------------------------------------------------------------- LGL operators (host)
void legendre(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

void make_ops(int N, Ops& op) {
  std::memset(&op, 0, sizeof op);
  const int p = N - 1;
  std::vector<double> x(N), w(N);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int j = 1; j < p; ++j) {
    double xi = -std::cos(M_PI * j / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, xi, P, dP);
      const double d2P = (2.0 * xi * dP - p * (p + 1.0) * P) / (1.0 - xi * xi);
      const double step = dP / d2P;
      xi -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[j] = xi;
  }
  // symmetric nodes exactly
  for (int j = 0; j < N / 2; ++j) {
    const double s = 0.5 * (x[N - 1 - j] - x[j]);
    x[j] = -s;
    x[N - 1 - j] = s;
  }
  if (N % 2) x[N / 2] = 0.0;
  for (int j = 0; j < N; ++j) {
    double P, dP;
    if (j == 0 || j == p) P = (j == 0 && (p % 2)) ? -1.0 : 1.0;
    else legendre(p, x[j], P, dP);
    w[j] = 2.0 / (p * (p + 1.0) * P * P);
  }
  // barycentric weights and differentiation matrix
  std::vector<double> lam(N, 1.0);
  for (int j = 0; j < N; ++j)
    for (int k = 0; k < N; ++k)
      if (k != j) lam[j] /= (x[j] - x[k]);
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int j = 0; j < N; ++j)
      if (j != i) {
        const double v = (lam[j] / lam[i]) / (x[i] - x[j]);
        op.D[i * N + j] = v;
        s += v;
      }
    op.D[i * N + i] = -s;
  }
  for (int j = 0; j < N; ++j) {
    op.w[j] = w[j];
    op.iw[j] = 1.0 / w[j];
    op.x[j] = x[j];
  }
  // modal transform for the shock-capturing indicator: Vinv = V^-1, V[i][k] = sqrt(k + 1/2)
  // P_k(x_i) (L2-orthonormal Legendre polynomials at the nodes), by Gauss-Jordan elimination
  {
    double V[kMaxN][2 * kMaxN];
    for (int i = 0; i < N; ++i)
      for (int c = 0; c < 2 * N; ++c) {
        if (c < N) {
          double P, dP;
          legendre(c, x[i], P, dP);
          V[i][c] = std::sqrt(c + 0.5) * P;
        } else {
          V[i][c] = c - N == i ? 1.0 : 0.0;
        }
      }
    for (int c = 0; c < N; ++c) {
      int piv = c;
      for (int r = c + 1; r < N; ++r)
        if (std::fabs(V[r][c]) > std::fabs(V[piv][c])) piv = r;
      for (int k = 0; k < 2 * N; ++k) std::swap(V[c][k], V[piv][k]);
      const double dg = V[c][c];
      for (int k = 0; k < 2 * N; ++k) V[c][k] /= dg;
      for (int r = 0; r < N; ++r)
        if (r != c) {
          const double f = V[r][c];
          for (int k = 0; k < 2 * N; ++k) V[r][k] -= f * V[c][k];
        }
    }
    for (int k = 0; k < N; ++k)
      for (int i = 0; i < N; ++i) op.Vinv[k * N + i] = V[k][N + i];
  }
  // mortar interpolation: P_m[j][k] = l_k((x_j -/+ 1)/2)
  for (int m = 0; m < 2; ++m) {
    for (int j = 0; j < N; ++j) {
      const double xi = m == 0 ? 0.5 * (x[j] - 1.0) : 0.5 * (x[j] + 1.0);
      for (int k = 0; k < N; ++k) {
        double l = 1.0;
        for (int q = 0; q < N; ++q)
          if (q != k) l *= (xi - x[q]) / (x[k] - x[q]);
        op.P[m][j * N + k] = l;
      }
    }
  }
  // mortar projection (Kopriva's conservative mortars): the L2 projection of the data on the
  // two half faces onto the coarse face's polynomials, with exact integrals, so that
  // R_0 P_0 + R_1 P_1 = I and a coarse polynomial survives the round trip.  The Lagrange basis is
  // expanded in monomials, products are integrated exactly (int_{-1}^{1} s^k ds), and
  // M R_m = 1/2 B_m is solved with M_ij = int l_i l_j, (B_m)_ij = int l_i((s -/+ 1)/2) l_j(s) ds.
  double mono[kMaxN][kMaxN];            // l_i(s) = sum_k mono[i][k] s^k
  {
    double V[kMaxN][2 * kMaxN];
    for (int r = 0; r < N; ++r)
      for (int c = 0; c < 2 * N; ++c) V[r][c] = c < N ? std::pow(x[r], c) : (c - N == r ? 1.0 : 0.0);
    for (int c = 0; c < N; ++c) {     // Gauss-Jordan: [V | I] -> [I | V^-1]
      int piv = c;
      for (int r = c + 1; r < N; ++r)
        if (std::fabs(V[r][c]) > std::fabs(V[piv][c])) piv = r;
      for (int k = 0; k < 2 * N; ++k) std::swap(V[c][k], V[piv][k]);
      const double d = V[c][c];
      for (int k = 0; k < 2 * N; ++k) V[c][k] /= d;
      for (int r = 0; r < N; ++r)
        if (r != c) {
          const double f = V[r][c];
          for (int k = 0; k < 2 * N; ++k) V[r][k] -= f * V[c][k];
        }
    }
    // monomial coefficients of l_i are column i of V^-1 (V_rk = x_r^k)
    for (int i = 0; i < N; ++i)
      for (int k = 0; k < N; ++k) mono[i][k] = V[k][N + i];
  }
  auto integral = [&](const double* a, const double* b) {   // int_{-1}^{1} (sum a_k s^k)(sum b_k s^k)
    double r = 0.0;
    for (int k = 0; k < N; ++k)
      for (int l = 0; l < N; ++l)
        if ((k + l) % 2 == 0) r += a[k] * b[l] * 2.0 / (k + l + 1);
    return r;
  };
  double Mx[kMaxN][kMaxN];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) Mx[i][j] = integral(mono[i], mono[j]);
  for (int m = 0; m < 2; ++m) {
    // l_i((s + sg)/2) in monomials of s, sg = -1 (m = 0) or +1 (m = 1)
    const double sg = m == 0 ? -1.0 : 1.0;
    double half[kMaxN][kMaxN];
    for (int i = 0; i < N; ++i) {
      for (int k = 0; k < N; ++k) half[i][k] = 0.0;
      for (int k = 0; k < N; ++k) {
        // ((s + sg)/2)^k = 2^-k sum_q C(k, q) s^q sg^(k-q)
        double binom = 1.0;
        for (int q = 0; q <= k; ++q) {
          half[i][q] += mono[i][k] * std::ldexp(binom, -k) * ((k - q) % 2 ? sg : 1.0);
          binom = binom * (k - q) / (q + 1);
        }
      }
    }
    double A[kMaxN][2 * kMaxN];
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        A[i][j] = Mx[i][j];
        A[i][N + j] = 0.5 * integral(half[i], mono[j]);
      }
    for (int c = 0; c < N; ++c) {     // Gauss-Jordan on [M | B/2] -> [I | R_m]
      int piv = c;
      for (int r = c + 1; r < N; ++r)
        if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
      for (int k = 0; k < 2 * N; ++k) std::swap(A[c][k], A[piv][k]);
      const double d = A[c][c];
      for (int k = 0; k < 2 * N; ++k) A[c][k] /= d;
      for (int r = 0; r < N; ++r)
        if (r != c) {
          const double f = A[r][c];
          for (int k = 0; k < 2 * N; ++k) A[r][k] -= f * A[c][k];
        }
    }
    for (int j = 0; j < N; ++j)
      for (int k = 0; k < N; ++k) op.R[m][j * N + k] = A[j][N + k];
  }
}

// ---------------------------------------------------------------- forest connectivity
// Pinned staging of at least `bytes`, free for the host to write: waits for the transfer still
// reading from it, grows it (by half again) when too small.
pe_status stage_reserve(pe_ctx* ctx, size_t bytes) {
  if (ctx->stage_pending) {
    HIPCHK(hipEventSynchronize(ctx->stage_ev));
    ctx->stage_pending = false;
  }
  if (!ctx->stage_ev) HIPCHK(hipEventCreateWithFlags(&ctx->stage_ev, hipEventDisableTiming));
  if (bytes <= ctx->h_stage_cap) return PE_OK;
  if (ctx->h_stage) HIPCHK(hipHostFree(ctx->h_stage));
  ctx->h_stage = nullptr;
  ctx->h_stage_cap = 0;
  const size_t cap = std::max(bytes + bytes / 2, (size_t)1 << 20);
  HIPCHK(hipHostMalloc(&ctx->h_stage, cap, hipHostMallocDefault));
  ctx->h_stage_cap = cap;
  return PE_OK;
}

// Marks the transfers just enqueued on `s` out of the staging buffer.
pe_status stage_mark(pe_ctx* ctx, hipStream_t s) {
  HIPCHK(hipEventRecord(ctx->stage_ev, s));
  ctx->stage_pending = true;
  return PE_OK;
}


struct KeyHash {
  size_t operator()(uint64_t k) const { return std::hash<uint64_t>()(k * 0x9E3779B97F4A7C15ull); }
};
inline uint64_t cell_key(int lev, int i, int j, int k) {
  return ((uint64_t)lev << 60) | ((uint64_t)(uint32_t)i << 40) | ((uint64_t)(uint32_t)j << 20) | (uint64_t)(uint32_t)k;
}

pe_status build_connectivity(pe_ctx* ctx) {
  const int n = ctx->n_e, dim = ctx->dim, nf = 2 * dim;
  ctx->max_level = 0;
  for (int e = 0; e < n; ++e) {
    const int32_t* L = &ctx->leaves[4 * e];
    const int lev = L[0];
    if (lev < 0 || lev >= kMaxLevels) return fail(ctx, PE_EINVAL, "leaf %d: level %d out of range [0,%d)", e, lev, kMaxLevels);
    for (int d = 0; d < dim; ++d) {
      const int nc = ctx->n_root[d] << lev;
      if (L[1 + d] < 0 || L[1 + d] >= nc) return fail(ctx, PE_EINVAL, "leaf %d: index out of range", e);
      if (nc >= (1 << 20)) return fail(ctx, PE_EINVAL, "leaf %d: grid too fine", e);
    }
    ctx->max_level = std::max(ctx->max_level, lev);
  }
  const int Lm = ctx->max_level;
  int64_t nfine[3] = {1, 1, 1}, total = 1;
  for (int d = 0; d < dim; ++d) {
    nfine[d] = (int64_t)ctx->n_root[d] << Lm;
    total *= nfine[d];
  }
  // Leaf lookup.  Dense: the owner of every cell of the finest level (one array read per
  // lookup; overlap and coverage checked while filling).  Hash map for very fine grids.
  const bool dense = total <= ((int64_t)1 << 24);
  std::vector<int32_t>& own = ctx->own_cells;   // kept between calls (no allocation per adaptation)
  std::unordered_map<uint64_t, int, KeyHash> idx;
  if (dense) {
    own.assign((size_t)total, -1);
    for (int e = 0; e < n; ++e) {
      const int32_t* L = &ctx->leaves[4 * e];
      const int sh = Lm - L[0], span = 1 << sh;
      const int64_t i0 = (int64_t)L[1] << sh, j0 = (int64_t)L[2] << sh, k0 = dim == 3 ? ((int64_t)L[3] << sh) : 0;
      const int sk = dim == 3 ? span : 1;
      for (int c = 0; c < sk; ++c)
        for (int b = 0; b < span; ++b) {
          int32_t* row = &own[(size_t)(((k0 + c) * nfine[1] + (j0 + b)) * nfine[0] + i0)];
          for (int a = 0; a < span; ++a) {
            if (row[a] >= 0) return fail(ctx, PE_EINVAL, "leaf %d overlaps leaf %d", e, row[a]);
            row[a] = e;
          }
        }
    }
    for (int64_t q = 0; q < total; ++q)
      if (own[(size_t)q] < 0) return fail(ctx, PE_EINVAL, "leaves do not cover the domain");
  } else {
    idx.reserve(n * 2);
    for (int e = 0; e < n; ++e) {
      const int32_t* L = &ctx->leaves[4 * e];
      if (!idx.emplace(cell_key(L[0], L[1], L[2], dim == 3 ? L[3] : 0), e).second)
        return fail(ctx, PE_EINVAL, "duplicate leaf %d", e);
    }
    // coverage: every leaf's ancestors must not be leaves; total volume must match
    double vol = 0.0;
    for (int e = 0; e < n; ++e) {
      const int lev = ctx->leaves[4 * e];
      vol += std::ldexp(1.0, -dim * lev);
      for (int up = 1; up <= lev; ++up) {
        const int32_t* L = &ctx->leaves[4 * e];
        if (idx.count(cell_key(lev - up, L[1] >> up, L[2] >> up, dim == 3 ? (L[3] >> up) : 0)))
          return fail(ctx, PE_EINVAL, "leaf %d overlaps an ancestor leaf", e);
      }
    }
    double roots = 1.0;
    for (int d = 0; d < dim; ++d) roots *= ctx->n_root[d];
    if (std::fabs(vol - roots) > 1e-9 * roots) return fail(ctx, PE_EINVAL, "leaves do not cover the domain");
  }
  ctx->fk_leaf.resize((size_t)n * nf);        // every entry is written below
  ctx->fn_leaf.resize((size_t)n * nf * 4);
  ctx->lev_leaf.resize(n);
  auto find = [&](int lev, int i, int j, int k) -> int {
    if (lev < 0 || lev > Lm) return -1;
    if (dense) {
      const int sh = Lm - lev;
      const int o = own[(size_t)((((int64_t)k << sh) * nfine[1] + ((int64_t)j << sh)) * nfine[0] + ((int64_t)i << sh))];
      return ctx->leaves[4 * o] == lev ? o : -1;
    }
    auto it = idx.find(cell_key(lev, i, j, k));
    return it == idx.end() ? -1 : it->second;
  };
  for (int e = 0; e < n; ++e) {
    const int32_t* L = &ctx->leaves[4 * e];
    const int lev = L[0];
    ctx->lev_leaf[e] = lev;
    for (int d = 0; d < dim; ++d)
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * d + s;
        int cc[3] = {L[1], L[2], dim == 3 ? L[3] : 0};
        const int nc = ctx->n_root[d] << lev;
        const int c = cc[d] + (s ? 1 : -1);   // periodic neighbour cell
        cc[d] = c < 0 ? c + nc : (c >= nc ? c - nc : c);
        int32_t* nb = &ctx->fn_leaf[((size_t)e * nf + f) * 4];
        nb[0] = nb[1] = nb[2] = nb[3] = -1;
        const int same = find(lev, cc[0], cc[1], cc[2]);
        if (same >= 0) {
          ctx->fk_leaf[(size_t)e * nf + f] = pack_face(kConforming, 0, 0);
          nb[0] = same;
          continue;
        }
        const int par = find(lev - 1, cc[0] >> 1, cc[1] >> 1, cc[2] >> 1);
        if (par >= 0) {
          int sub[2] = {0, 0}, t = 0;
          for (int q = 0; q < dim; ++q)
            if (q != d) sub[t++] = (q == 0 ? L[1] : (q == 1 ? L[2] : L[3])) & 1;
          ctx->fk_leaf[(size_t)e * nf + f] = pack_face(kFineSide, sub[0], sub[1]);
          nb[0] = par;
          continue;
        }
        int tang[2] = {0, 0}, t = 0;
        for (int q = 0; q < dim; ++q)
          if (q != d) tang[t++] = q;
        const int nsub = 1 << (dim - 1);
        for (int m = 0; m < nsub; ++m) {
          int ch[3] = {2 * cc[0], 2 * cc[1], 2 * cc[2]};
          ch[d] += s ? 0 : 1;
          ch[tang[0]] += m & 1;
          if (dim == 3) ch[tang[1]] += (m >> 1) & 1;
          const int c = find(lev + 1, ch[0], ch[1], dim == 3 ? ch[2] : 0);
          if (c < 0) return fail(ctx, PE_EINVAL, "leaf %d face %d: no 2:1-balanced neighbour", e, f);
          nb[m] = c;
        }
        ctx->fk_leaf[(size_t)e * nf + f] = pack_face(kCoarseSide, 0, 0);
      }
  }
  if (own.capacity() > ((size_t)1 << 20)) std::vector<int32_t>().swap(own);   // keep at most 4 MB
  return PE_OK;
}

int nodes_per_elem(const pe_ctx* c) { return c->dim == 2 ? c->N * c->N : c->N * c->N * c->N; }
int nvars(const pe_ctx* c) { return c->dim + 2; }
int64_t cap_of(const pe_ctx* c) { return c->capacity > c->n_e ? c->capacity : c->n_e; }
int64_t state_doubles(const pe_ctx* c) { return cap_of(c) * nvars(c) * nodes_per_elem(c); }

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace layout: five state-sized fp64 arrays (K1, two stage buffers, the weighted stage
// sum, a permutation temporary), the extra stage buffers of a general stage pattern, BR1
// gradients for Navier-Stokes, then int32 tables.
size_t carve(pe_ctx* c, char* base);

size_t workspace_bytes(const pe_ctx* c) {
  pe_ctx tmp;
  tmp.dim = c->dim;
  tmp.N = c->N;
  tmp.equations = c->equations;
  tmp.n_e = c->n_e;
  tmp.capacity = c->capacity;
  tmp.n_ybuf = c->n_ybuf;
  return carve(&tmp, nullptr);
}

size_t carve(pe_ctx* c, char* base) {
  size_t off = 0;
  const size_t sd = (size_t)state_doubles(c) * sizeof(double);
  const int n = (int)cap_of(c), nf = 2 * c->dim;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  c->K1 = (double*)take(sd);
  c->Ya = (double*)take(sd);
  c->Yb = (double*)take(sd);
  c->ACC = (double*)take(sd);
  c->Tmp = (double*)take(sd);
  c->ybuf.assign({c->Ya, c->Yb});
  for (int k = 2; k < c->n_ybuf; ++k) c->ybuf.push_back((double*)take(sd));
  c->Fv = c->equations == 1 ? (double*)take((size_t)c->dim * nvars(c) * n * nodes_per_elem(c) * sizeof(double))
                            : nullptr;
  c->d_fk_leaf = (int32_t*)take((size_t)n * nf * 4);
  c->d_fn_leaf = (int32_t*)take((size_t)n * nf * 4 * 4);
  c->d_lev_leaf = (int32_t*)take((size_t)n * 4);
  c->d_fk = (int32_t*)take((size_t)n * nf * 4);
  c->d_fn = (int32_t*)take((size_t)n * nf * 4 * 4);
  c->d_lev = (int32_t*)take((size_t)n * 4);
  c->d_mem = (int32_t*)take((size_t)n * 4);
  c->d_mem_leaf = (int32_t*)take((size_t)n * 4);
  c->d_slot_of_leaf = (int32_t*)take((size_t)n * 4);
  c->d_leaf_of_slot = (int32_t*)take((size_t)n * 4);
  c->d_old_slot_of_leaf = (int32_t*)take((size_t)n * 4);
  c->d_counts = (int32_t*)take(kMaxMembers * 4);
  c->d_halo = (int32_t*)take((size_t)n * 4 * (kMaxMembers + 1));
  c->d_counter = (unsigned long long*)take(kMaxMembers * 8);
  c->d_evals = (int32_t*)take((size_t)n * 4);
  c->d_plan = (int32_t*)take((size_t)n * 10 * 4);
  c->d_eta = (double*)take((size_t)n * 8);
  c->d_beta = (double*)take(kMaxLevels * 8);
  c->d_dmat = (double*)take(7 * kMaxN * kMaxN * 8);
  return off;
}

Mesh device_mesh(const pe_ctx* c) {
  Mesh m{};
  m.fk = c->d_fk;
  m.fn = c->d_fn;
  m.lev = c->d_lev;
  m.mem = c->d_mem;
  m.ld = (int)cap_of(c);
  m.R = c->R;
  {
    // slots are sorted by member, most stage evaluations first
    int acc = 0;
    for (int k = 0; k < kMaxMembers; ++k) {
      const int r = c->R - 1 - k;
      if (r >= 0 && (int)c->counts.size() == c->R) acc += c->counts[r];
      m.bnd[k] = acc;
    }
  }
  for (int l = 0; l < kMaxLevels; ++l)
    for (int d = 0; d < 3; ++d) {
      const double h = d < c->dim ? (c->hi[d] - c->lo[d]) / std::ldexp((double)c->n_root[d], l) : 1.0;
      m.jac[l][d] = 2.0 / h;
    }
  return m;
}

// member r evaluates 0-based stage i: classic pattern iff i == 0 or i >= S - E_r + 1; a general
// pattern iff i == 0, b_i != 0 or some row couples K_i
inline bool active(const pe_ctx* c, int r, int i) {
  if (!c->general) return i == 0 || i >= c->S - c->E[r] + 1;
  return i == 0 || c->b[i] != 0.0 || c->uses[(size_t)r * c->S + i] >= 0;
}

// where member r's stage value Y_i comes from at stage i: 0 U_n, 1 the stage buffer (computed at
// an earlier stage), 2 U_n + dt c_i K_1 formed on the fly
inline int src_code(const pe_ctx* c, int r, int i) {
  if (i == 0) return 0;
  if (!c->general) return (active(c, r, i) && active(c, r, i - 1)) ? 1 : 2;
  return c->cpl[(size_t)r * c->S + i] >= 0 ? 1 : 2;
}

// blending-factor parameters of subcell shock capturing (Hennemann et al.): threshold
// T = 0.5 10^(-1.8 (p+1)^(1/4)) and the sigmoid's slope s / T, s = ln((1 - 1e-4) / 1e-4)
void set_shock_capturing_args(const pe_ctx* c, StageArgs& a) {
  a.sc = c->sc_on ? 1 : 0;
  a.sc_amax = c->sc_amax;
  a.sc_amin = c->sc_amin;
  a.sc_T = 0.5 * std::pow(10.0, -1.8 * std::pow((double)c->N, 0.25));
  a.sc_slope = std::log((1.0 - 1e-4) / 1e-4) / a.sc_T;
}

void fill_stage(const pe_ctx* c, int i, double dt, StageArgs& a) {
  std::memset(&a, 0, sizeof a);
  set_shock_capturing_args(c, a);
  a.dt = dt;
  a.ci = c->c[i];
  a.first = i == 0;
  a.last = i == c->S - 1;
  a.n_act = c->n_act[i];
  // weighted sum of stages with b != 0 before the last
  int seen = 0;
  for (int j = 0; j < i; ++j)
    if (c->b[j] != 0.0) ++seen;
  if (!a.last && c->b[i] != 0.0) {
    a.acc_mode = seen == 0 ? 1 : 2;
    a.bi = c->b[i];
  }
  a.bS = c->b[c->S - 1];
  a.use_acc_last = 0;
  for (int j = 0; j < c->S - 1; ++j)
    if (c->b[j] != 0.0) a.use_acc_last = 1;
  a.read_acc = (a.acc_mode == 2 || (a.last && a.use_acc_last)) ? 1 : 0;
  for (int r = 0; r < c->R; ++r) {
    a.src[r] = src_code(c, r, i);
    a.src_bits |= a.src[r] << (2 * r);
    if (!c->general) {
      if (i + 1 < c->S) {
        a.wr[r] = active(c, r, i + 1) ? 1 : 0;
        a.a2[r] = c->a_sub[(size_t)r * c->S + i + 1];
        a.a1[r] = c->c[i + 1] - a.a2[r];
      }
    } else {
      // the one row k that couples K_i of this member gets Y_k = U_n + dt (a_{k,1} K_1 + a_{k,i} K_i)
      const int k = c->uses[(size_t)r * c->S + i];
      if (k >= 0) {
        a.wr[r] = 1;
        a.a2[r] = c->a_sub[(size_t)r * c->S + k];
        a.a1[r] = c->c[k] - a.a2[r];
      }
    }
  }
  // the active elements as slot ranges
  const auto& rg = c->act_rng[i];
  a.n_rng = (int)rg.size();
  for (int k = 0, cum = 0; k < (int)rg.size(); ++k) {
    a.rng_start[k] = rg[k].first;
    a.rng_cum[k] = cum;
    cum += rg[k].second;
  }
}

// Stage buffers of launch i: Yin holds Y_i (for members with src 1), Yw[r] receives the stage
// value member r forms at this stage.  Classic: Y_i alternates between Ya and Yb.
void set_stage_buffers(const pe_ctx* c, int i, StageArgs& a) {
  if (!c->general) {
    a.Yin = (i % 2 == 0) ? c->Ya : c->Yb;
    a.Yout = (i % 2 == 0) ? c->Yb : c->Ya;
    for (int r = 0; r < c->R; ++r) a.Yw[r] = a.wr[r] ? a.Yout : nullptr;
    return;
  }
  a.Yin = c->ybuf_of_stage[i] >= 0 ? c->ybuf[c->ybuf_of_stage[i]] : c->Ya;
  a.Yout = nullptr;
  for (int r = 0; r < c->R; ++r) {
    const int k = c->uses[(size_t)r * c->S + i];
    a.Yw[r] = (a.wr[r] && k >= 0) ? c->ybuf[c->ybuf_of_stage[k]] : nullptr;
  }
}

// Classic outputs into caller-chosen buffers: every member writing at this stage writes to a.Yout.
void classic_outputs(StageArgs& a) {
  for (int r = 0; r < kMaxMembers; ++r) a.Yw[r] = a.wr[r] ? a.Yout : nullptr;
}

// Active slot ranges per stage from the member counts: slots hold member R-1 first, then R-2, ...
// Adjacent active members merge into one range (the classic pattern: one range [0, n_act)).
void build_activity(pe_ctx* c) {
  c->n_act.assign(c->S, 0);
  c->act_rng.assign(c->S, {});
  for (int i = 0; i < c->S; ++i) {
    int start = 0;
    for (int r = c->R - 1; r >= 0; --r) {
      const int cnt = (int)c->counts.size() == c->R ? c->counts[r] : 0;
      if (active(c, r, i) && cnt > 0) {
        auto& rg = c->act_rng[i];
        if (!rg.empty() && rg.back().first + rg.back().second == start) rg.back().second += cnt;
        else rg.emplace_back(start, cnt);
        c->n_act[i] += cnt;
      }
      start += cnt;
    }
  }
}

// Stage buffers of a general pattern: Y_k (rows with a coupling in some member) is written at the
// stages of those couplings and read at stage k; two stage values share a buffer only if their
// [first write, read] intervals are disjoint (greedy colouring by first write, reads inclusive:
// a launch never reads and writes one buffer).
void assign_stage_buffers(pe_ctx* c) {
  const int S = c->S, R = c->R;
  c->ybuf_of_stage.assign(S, -1);
  if (!c->general) {
    c->n_ybuf = 2;
    return;
  }
  std::vector<int> first(S, S);
  for (int r = 0; r < R; ++r)
    for (int k = 0; k < S; ++k) {
      const int j = c->cpl[(size_t)r * S + k];
      if (j >= 0) first[k] = std::min(first[k], j);
    }
  std::vector<int> free_after;          // per buffer: the last stage that reads it
  for (int w = 0; w < S; ++w)
    for (int k = 0; k < S; ++k) {
      if (first[k] != w) continue;
      int buf = -1;
      for (int q = 0; q < (int)free_after.size(); ++q)
        if (free_after[q] < w) { buf = q; break; }
      if (buf < 0) {
        buf = (int)free_after.size();
        free_after.push_back(-1);
      }
      free_after[buf] = k;
      c->ybuf_of_stage[k] = buf;
    }
  c->n_ybuf = std::max(2, (int)free_after.size());
}

// Member of every level 0..n_levels-1 from the context's rule, the finest level being `finest`
// (levels finer than it take the member with the most stage evaluations).
//   paper rule (Sec. 6.4.1): the finest level takes member R-1, the next coarser R-2, and so on;
//     every level beyond the R finest takes member 0;
//   required-step rule: the spectrum of a convection-dominated problem scales with 1/h (Sec. 3.1),
//     so member r admits dt_opt[r] 2^(finest - l) on level l; level l takes the cheapest member
//     that admits the common step dt_opt[R-1] of the finest level times the margin (the finest
//     level itself without margin), or member R-1 if none does.
void level_map(const pe_ctx* c, int finest, int n_levels, int32_t* out) {
  const int R = c->R;
  for (int l = 0; l < n_levels; ++l) {
    if (l >= finest) {
      out[l] = R - 1;
      continue;
    }
    if (c->rule == PE_LEVEL_RULE_PAPER) {
      out[l] = std::max(0, (R - 1) - (finest - l));
      continue;
    }
    const double need = c->rule_dt_opt[R - 1] * c->rule_margin * (1.0 - 1e-12);
    const double scale = std::ldexp(1.0, finest - l);
    int r = R - 1;
    for (int k = 0; k < R; ++k)
      if (c->rule_dt_opt[k] * scale >= need) {
        r = k;
        break;
      }
    out[l] = r;
  }
}

bool last_stage_in_place_safe(const pe_ctx* c) {
  // At the last stage a neighbour reads U_n only if its stage value there is formed on the fly.
  for (int r = 0; r < c->R; ++r)
    if (c->S > 1 && src_code(c, r, c->S - 1) != 1) return false;
  return true;
}

}  // namespace

extern "C" {

pe_status pe_create(pe_ctx** out, const pe_physics* phys) {
  if (!out || !phys) return PE_EINVAL;
  *out = nullptr;
  pe_ctx* c = new (std::nothrow) pe_ctx();
  if (!c) return PE_ENOMEM;
  if (phys->dim != 2 && phys->dim != 3) {
    delete c;
    return PE_EINVAL;
  }
  if (phys->degree < 1 || phys->degree + 1 > kMaxN || phys->gamma <= 1.0 || phys->equations < 0 ||
      phys->equations > 1 || (phys->equations == 1 && (phys->mu < 0.0 || phys->prandtl <= 0.0))) {
    delete c;
    return PE_EINVAL;
  }
  c->dim = phys->dim;
  c->degree = phys->degree;
  c->N = phys->degree + 1;
  c->equations = phys->equations;
  c->ph.gamma = phys->gamma;
  c->ph.mu = phys->equations == 1 ? phys->mu : 0.0;
  c->ph.kappa = phys->equations == 1 ? phys->gamma * phys->mu / ((phys->gamma - 1.0) * phys->prandtl) : 0.0;
  make_ops(c->N, c->ops);
  *out = c;
  return PE_OK;
}

void pe_destroy(pe_ctx* ctx) { delete ctx; }

const char* pe_last_error(const pe_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

pe_status pe_mesh_build(pe_ctx* ctx, const pe_mesh_desc* mesh) {
  if (!ctx) return PE_EINVAL;
  if (!mesh || mesh->dim != ctx->dim || mesh->n_leaves <= 0 || !mesh->leaves)
    return fail(ctx, PE_EINVAL, "mesh: bad descriptor (dimension must match the physics)");
  for (int d = 0; d < ctx->dim; ++d)
    if (mesh->n_root[d] <= 0 || !(mesh->hi[d] > mesh->lo[d])) return fail(ctx, PE_EINVAL, "mesh: bad box");
  ctx->have_mesh = false;
  ctx->bound = false;
  ctx->partitioned = false;
  ctx->graph_valid = false;
  ctx->state_valid = false;
  for (int d = 0; d < 3; ++d) {
    ctx->n_root[d] = d < ctx->dim ? mesh->n_root[d] : 1;
    ctx->lo[d] = d < ctx->dim ? mesh->lo[d] : 0.0;
    ctx->hi[d] = d < ctx->dim ? mesh->hi[d] : 1.0;
  }
  ctx->n_e = mesh->n_leaves;
  ctx->leaves.assign(mesh->leaves, mesh->leaves + 4 * (size_t)mesh->n_leaves);
  if (ctx->dim == 2)
    for (int e = 0; e < ctx->n_e; ++e) ctx->leaves[4 * e + 3] = 0;
  pe_status st = build_connectivity(ctx);
  if (st != PE_OK) return st;
  ctx->have_mesh = true;
  return PE_OK;
}

pe_status pe_set_perk_coefficients(pe_ctx* ctx, const pe_perk_coeffs* co) {
  if (!ctx) return PE_EINVAL;
  if (!co || !co->E || !co->c || !co->a_sub || !co->b) return fail(ctx, PE_EINVAL, "coefficients: null pointer");
  const int R = co->n_members, S = co->n_stages;
  if (R < 1 || R > kMaxMembers || S < 1 || S > kMaxStages || (co->order != 2 && co->order != 3))
    return fail(ctx, PE_EINVAL, "coefficients: R=%d S=%d order=%d out of range", R, S, co->order);
  for (int r = 0; r < R; ++r) {
    if (co->E[r] < 1 || co->E[r] > S || (r > 0 && co->E[r] <= co->E[r - 1]))
      return fail(ctx, PE_EINVAL, "coefficients: E must be strictly ascending in [1, S]");
  }
  if (co->E[R - 1] != S) return fail(ctx, PE_EINVAL, "coefficients: largest member must use all S stages");
  // stage pattern: the classic chain, or one coupling column per row from the table
  const bool general = co->coupling != nullptr;
  std::vector<int> cpl((size_t)R * S, -1), uses((size_t)R * S, -1);
  if (general) {
    if (ctx->equations != 0)
      return fail(ctx, PE_EUNSUPPORTED, "coefficients: alternative stage patterns are supported for Euler only");
    if (ctx->sc_on)
      return fail(ctx, PE_EUNSUPPORTED, "coefficients: alternative stage patterns are not supported with shock capturing");
    for (int r = 0; r < R; ++r)
      for (int i = 0; i < S; ++i) {
        const int j = co->coupling[(size_t)r * S + i];
        const double av = co->a_sub[(size_t)r * S + i];
        if (j == -1) {
          if (av != 0.0) return fail(ctx, PE_EINVAL, "member %d row %d: coefficient without a coupling", r, i + 1);
          continue;
        }
        if (j < 1 || j >= i)
          return fail(ctx, PE_EINVAL, "member %d row %d: coupling column %d outside [2, %d]", r, i + 1, j + 1, i);
        if (uses[(size_t)r * S + j] >= 0)
          return fail(ctx, PE_EINVAL, "member %d: K_%d feeds two stage values", r, j + 1);
        cpl[(size_t)r * S + i] = j;
        uses[(size_t)r * S + j] = i;
      }
    for (int r = 0; r < R; ++r) {
      int ev = 0;
      for (int i = 0; i < S; ++i)
        if (i == 0 || co->b[i] != 0.0 || uses[(size_t)r * S + i] >= 0) ++ev;
      if (ev != co->E[r])
        return fail(ctx, PE_EINVAL, "member %d evaluates %d stages under its coupling table, E says %d", r, ev,
                    co->E[r]);
    }
  } else {
    for (int r = 0; r < R; ++r)
      for (int i = S - co->E[r] + 2; i < S; ++i)
        if (i >= 2) {
          cpl[(size_t)r * S + i] = i - 1;
          uses[(size_t)r * S + i - 1] = i;
        }
  }
  const double tol = 1e-12;
  double sb = 0.0, sbc = 0.0, sbc2 = 0.0;
  for (int i = 0; i < S; ++i) {
    sb += co->b[i];
    sbc += co->b[i] * co->c[i];
    sbc2 += co->b[i] * co->c[i] * co->c[i];
  }
  if (std::fabs(co->c[0]) > tol) return fail(ctx, PE_EINVAL, "coefficients: c_1 must be 0");
  if (std::fabs(sb - 1.0) > tol) return fail(ctx, PE_EINVAL, "order condition b^T 1 = 1 violated (%g)", sb);
  if (co->order >= 2 && std::fabs(sbc - 0.5) > tol)
    return fail(ctx, PE_EINVAL, "order condition b^T c = 1/2 violated (%g)", sbc);
  if (co->order >= 3 && std::fabs(sbc2 - 1.0 / 3.0) > tol)
    return fail(ctx, PE_EINVAL, "order condition b^T c^2 = 1/3 violated (%g)", sbc2);
  for (int r = 0; r < R; ++r) {
    const double* a = co->a_sub + (size_t)r * S;
    if ((S > 0 && a[0] != 0.0) || (S > 1 && a[1] != 0.0))
      return fail(ctx, PE_EINVAL, "member %d: a_sub rows 0 and 1 must be zero", r);
    if (!general)
      for (int i = 2; i < S; ++i)
        if (i <= S - co->E[r] + 1 && a[i] != 0.0)
          return fail(ctx, PE_EINVAL, "member %d (E=%d): a_{%d,%d} must be zero for a stage it skips", r, co->E[r],
                      i + 1, i);
    if (co->order >= 3) {
      // b^T A c = sum_i b_i (a_{i,1} c_1 + a_{i,j} c_j) with c_1 = 0, j the coupling column of row i
      double s = 0.0;
      for (int i = 2; i < S; ++i) {
        const int j = cpl[(size_t)r * S + i];
        if (j >= 0) s += co->b[i] * a[i] * co->c[j];
      }
      if (S > 1) s += co->b[1] * co->c[1] * co->c[0];
      if (std::fabs(s - 1.0 / 6.0) > tol)
        return fail(ctx, PE_EINVAL, "member %d: order condition b^T A c = 1/6 violated (%g)", r, s);
    }
  }
  // every stage with b != 0 evaluated by every member (checked before anything is stored, so a
  // rejected family leaves the context as it was); a general pattern evaluates such stages by
  // definition
  if (!general)
    for (int i = 0; i < S; ++i)
      if (co->b[i] != 0.0)
        for (int r = 0; r < R; ++r)
          if (!(i == 0 || i >= S - co->E[r] + 1))
            return fail(ctx, PE_EINVAL, "stage %d has b != 0 but member %d does not evaluate it", i + 1, r);
  // the largest member evaluates every stage
  if (general)
    for (int i = 1; i < S; ++i)
      if (co->b[i] == 0.0 && uses[(size_t)(R - 1) * S + i] < 0)
        return fail(ctx, PE_EINVAL, "coefficients: the largest member must evaluate every stage (stage %d)", i + 1);
  // stage buffers the pattern needs; a bound workspace must already hold them
  pe_ctx probe;
  probe.general = general;
  probe.R = R;
  probe.S = S;
  probe.cpl = cpl;
  assign_stage_buffers(&probe);
  if (ctx->bound && probe.n_ybuf > ctx->n_ybuf_bound)
    return fail(ctx, PE_EINVAL, "coefficients: the pattern needs %d stage buffers, the bound workspace has %d "
                "(query sizes and bind again)", probe.n_ybuf, ctx->n_ybuf_bound);
  if (ctx->have_rule && ctx->rule == PE_LEVEL_RULE_REQUIRED_STEP && (int)ctx->rule_dt_opt.size() != R)
    ctx->have_rule = false;   // the step sizes belonged to another family
  ctx->order = co->order;
  ctx->R = R;
  ctx->S = S;
  ctx->E.assign(co->E, co->E + R);
  ctx->c.assign(co->c, co->c + S);
  ctx->b.assign(co->b, co->b + S);
  ctx->a_sub.assign(co->a_sub, co->a_sub + (size_t)R * S);
  ctx->general = general;
  ctx->cpl = cpl;
  ctx->uses = uses;
  ctx->ybuf_of_stage = probe.ybuf_of_stage;
  ctx->n_ybuf = probe.n_ybuf;
  ctx->have_coeffs = true;
  ctx->partitioned = false;
  ctx->graph_valid = false;
  return PE_OK;
}

pe_status pe_set_level_rule(pe_ctx* ctx, int rule, const double* dt_opt, double margin) {
  if (!ctx) return PE_EINVAL;
  if (rule == PE_LEVEL_RULE_PAPER) {
    ctx->rule = rule;
    ctx->rule_dt_opt.clear();
    ctx->rule_margin = 1.0;
    ctx->have_rule = true;
    return PE_OK;
  }
  if (rule != PE_LEVEL_RULE_REQUIRED_STEP) return fail(ctx, PE_EINVAL, "level rule %d unknown", rule);
  if (!ctx->have_coeffs) return fail(ctx, PE_ESTATE, "required-step rule needs the coefficients first");
  if (!dt_opt) return fail(ctx, PE_EINVAL, "required-step rule: null dt_opt");
  if (!(margin >= 1.0) || !std::isfinite(margin)) return fail(ctx, PE_EINVAL, "required-step rule: margin must be >= 1");
  for (int r = 0; r < ctx->R; ++r)
    if (!(dt_opt[r] > 0.0) || !std::isfinite(dt_opt[r]))
      return fail(ctx, PE_EINVAL, "required-step rule: dt_opt[%d] must be positive and finite", r);
  ctx->rule = rule;
  ctx->rule_dt_opt.assign(dt_opt, dt_opt + ctx->R);
  ctx->rule_margin = margin;
  ctx->have_rule = true;
  return PE_OK;
}

pe_status pe_level_map(const pe_ctx* cctx, int finest_level, int n_levels, int32_t* member_of_level) {
  if (!cctx) return PE_EINVAL;
  pe_ctx* ctx = const_cast<pe_ctx*>(cctx);
  if (!ctx->have_coeffs) return fail(ctx, PE_ESTATE, "level_map before set_perk_coefficients");
  if (!ctx->have_rule) return fail(ctx, PE_ESTATE, "level_map: no level rule set");
  if (finest_level < 0) {
    if (!ctx->have_mesh) return fail(ctx, PE_ESTATE, "level_map: finest level of the mesh asked before mesh_build");
    finest_level = ctx->max_level;
  }
  if (!member_of_level || n_levels < 1 || n_levels > kMaxLevels || finest_level >= kMaxLevels)
    return fail(ctx, PE_EINVAL, "level_map: need 1 <= n_levels <= %d and finest_level < %d", kMaxLevels, kMaxLevels);
  level_map(ctx, finest_level, n_levels, member_of_level);
  return PE_OK;
}

pe_status pe_query_sizes(const pe_ctx* ctx, int64_t* n_state, int64_t* n_ws, int64_t* n_elem) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->have_mesh) return fail(const_cast<pe_ctx*>(ctx), PE_ESTATE, "query_sizes before mesh_build");
  if (n_state) *n_state = state_doubles(ctx);
  if (n_ws) *n_ws = (int64_t)workspace_bytes(ctx);
  if (n_elem) *n_elem = ctx->n_e;
  return PE_OK;
}

pe_status pe_bind(pe_ctx* ctx, double* u_dev, void* ws, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->have_mesh) return fail(ctx, PE_ESTATE, "bind before mesh_build");
  if (!u_dev || !ws) return fail(ctx, PE_EINVAL, "bind: null buffer");
  if (((uintptr_t)ws & 255) != 0) return fail(ctx, PE_EINVAL, "bind: workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  ctx->U = u_dev;
  ctx->ws = (char*)ws;
  carve(ctx, ctx->ws);
  ctx->n_ybuf_bound = ctx->n_ybuf;
  const int n = ctx->n_e, nf = 2 * ctx->dim;
  HIPCHK(hipMemcpyAsync(ctx->d_fk_leaf, ctx->fk_leaf.data(), (size_t)n * nf * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->d_fn_leaf, ctx->fn_leaf.data(), (size_t)n * nf * 16, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->d_lev_leaf, ctx->lev_leaf.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(ctx->d_counter, 0, kMaxMembers * 8, s));
  HIPCHK(hipMemsetAsync(ctx->d_evals, 0, (size_t)cap_of(ctx) * 4, s));
  const int N = ctx->N;
  double dm[7 * kMaxN * kMaxN];
  for (int i = 0; i < N * N; ++i) {
    dm[i] = i / N == i % N ? 0.0 : 2.0 * ctx->ops.D[i];
    dm[N * N + i] = ctx->ops.D[i];
    for (int mm = 0; mm < 2; ++mm) {
      dm[(2 + mm) * N * N + i] = ctx->ops.P[mm][i];
      dm[(4 + mm) * N * N + i] = ctx->ops.R[mm][i];
    }
    dm[6 * N * N + i] = ctx->ops.Vinv[i];
  }
  HIPCHK(hipMemcpyAsync(ctx->d_dmat, dm, 7 * (size_t)N * N * 8, hipMemcpyHostToDevice, s));
  ctx->ops.dD = ctx->d_dmat;
  ctx->pending_leaf_state = false;
  HIPCHK(hipStreamSynchronize(s));
  ctx->bound = true;
  ctx->graph_valid = false;
  ctx->partitioned = false;
  ctx->graph_valid = false;
  ctx->state_valid = false;
  return PE_OK;
}

namespace {
// slot maps and members back to the host (for element_info and the halo lists)
pe_status copy_maps(pe_ctx* ctx, hipStream_t s) {
  const int n = ctx->n_e;
  ctx->leaf_of_slot.resize(n);
  ctx->slot_of_leaf.resize(n);
  ctx->mem_of_slot.resize(n);
  HIPCHK(hipMemcpyAsync(ctx->leaf_of_slot.data(), ctx->d_leaf_of_slot, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(ctx->slot_of_leaf.data(), ctx->d_slot_of_leaf, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(ctx->mem_of_slot.data(), ctx->d_mem, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  ctx->maps_on_host = true;
  return PE_OK;
}
// Per stage, the inactive face neighbours of the active prefix (sorted slots, shared between
// stages with the same active count).  Needs the slot maps on the host.
pe_status build_halo(pe_ctx* ctx, hipStream_t s) {
  const int n = ctx->n_e, nf = 2 * ctx->dim;
  if (!ctx->maps_on_host) {
    pe_status st = copy_maps(ctx, s);
    if (st != PE_OK) return st;
    HIPCHK(hipStreamSynchronize(s));
  }
  ctx->halo_off.assign(ctx->S, 0);
  ctx->halo_cnt.assign(ctx->S, 0);
  std::vector<int32_t> all;
  std::vector<int> seen_na;
  std::vector<char> mark(n, 0);
  for (int i = 0; i < ctx->S; ++i) {
    const int na = ctx->n_act[i];
    auto it = std::find(seen_na.begin(), seen_na.end(), na);
    if (it != seen_na.end()) {
      int j = 0;
      for (; j < i; ++j)
        if (ctx->n_act[j] == na) break;
      ctx->halo_off[i] = ctx->halo_off[j];
      ctx->halo_cnt[i] = ctx->halo_cnt[j];
      continue;
    }
    seen_na.push_back(na);
    std::vector<int32_t> h;
    if (na < n) {
      std::fill(mark.begin(), mark.end(), 0);
      for (int sl = 0; sl < na; ++sl) {
        const int leaf = ctx->leaf_of_slot[sl];
        for (int f = 0; f < nf; ++f) {
          const int kind = face_kind(ctx->fk_leaf[(size_t)leaf * nf + f]);
          const int cnt = kind == kCoarseSide ? (1 << (ctx->dim - 1)) : 1;
          for (int q = 0; q < cnt; ++q) {
            const int t = ctx->slot_of_leaf[ctx->fn_leaf[((size_t)leaf * nf + f) * 4 + q]];
            if (t >= na && !mark[t]) {
              mark[t] = 1;
              h.push_back(t);
            }
          }
        }
      }
      std::sort(h.begin(), h.end());
    }
    ctx->halo_off[i] = (int)all.size();
    ctx->halo_cnt[i] = (int)h.size();
    all.insert(all.end(), h.begin(), h.end());
  }
  if (!all.empty()) {
    HIPCHK(hipMemcpyAsync(ctx->d_halo, all.data(), all.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  ctx->halo_valid = true;
  return PE_OK;
}

}  // namespace

pe_status pe_partition(pe_ctx* ctx, const int32_t* member_of_level, int n_levels, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->bound || !ctx->have_coeffs) return fail(ctx, PE_ESTATE, "partition needs a bound mesh and coefficients");
  int32_t rule_map[kMaxLevels];
  if (!member_of_level) {
    // the context's level rule at the finest level of the current mesh
    if (!ctx->have_rule) return fail(ctx, PE_ESTATE, "partition: no member_of_level and no level rule set");
    n_levels = ctx->max_level + 1;
    level_map(ctx, ctx->max_level, n_levels, rule_map);
    member_of_level = rule_map;
  }
  if (n_levels <= ctx->max_level || n_levels > kMaxLevels)
    return fail(ctx, PE_EINVAL, "member_of_level must cover levels 0..%d", ctx->max_level);
  PartitionArgs pa{};
  for (int l = 0; l < kMaxLevels; ++l) pa.member_of_level[l] = l < n_levels ? member_of_level[l] : 0;
  for (int l = 0; l < n_levels; ++l)
    if (member_of_level[l] < 0 || member_of_level[l] >= ctx->R)
      return fail(ctx, PE_EINVAL, "member_of_level[%d] = %d outside [0, %d)", l, member_of_level[l], ctx->R);
  hipStream_t s = (hipStream_t)stream;
  const int n = ctx->n_e, nf = 2 * ctx->dim;
  const bool permute = ctx->state_valid && ctx->partitioned && !ctx->pending_leaf_state;
  if (ctx->partitioned) HIPCHK(launch_fold_evals(n, device_mesh(ctx), ctx->d_evals, ctx->d_counter, s));
  if (permute)
    HIPCHK(hipMemcpyAsync(ctx->d_old_slot_of_leaf, ctx->d_slot_of_leaf, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  pa.lev_leaf = ctx->d_lev_leaf;
  pa.mem_leaf = ctx->d_mem_leaf;
  pa.slot_of_leaf = ctx->d_slot_of_leaf;
  pa.leaf_of_slot = ctx->d_leaf_of_slot;
  pa.counts = ctx->d_counts;
  pa.n = n;
  pa.R = ctx->R;
  HIPCHK(launch_partition_sort(pa, s));
  HIPCHK(launch_remap_connectivity(n, nf, ctx->d_leaf_of_slot, ctx->d_slot_of_leaf, ctx->d_fk_leaf, ctx->d_fn_leaf,
                                   ctx->d_lev_leaf, ctx->d_mem_leaf, ctx->d_fk, ctx->d_fn, ctx->d_lev, ctx->d_mem, s));
  if (permute) {
    HIPCHK(launch_permute_state(n, (int)cap_of(ctx), nvars(ctx), nodes_per_elem(ctx), ctx->d_leaf_of_slot,
                                ctx->d_old_slot_of_leaf, ctx->U, ctx->Tmp, s));
    HIPCHK(launch_copy(ctx->U, ctx->Tmp, state_doubles(ctx), s));
  }
  if (ctx->pending_leaf_state) {
    HIPCHK(launch_leaf_to_slot(n, (int)cap_of(ctx), nvars(ctx), nodes_per_elem(ctx), ctx->d_leaf_of_slot, ctx->Tmp,
                               ctx->U, s));
    ctx->pending_leaf_state = false;
    ctx->state_valid = true;
  }
  // elements per member from the host's leaf levels (the same counts the sort kernel forms)
  ctx->counts.assign(ctx->R, 0);
  for (int e = 0; e < n; ++e) ctx->counts[member_of_level[ctx->lev_leaf[e]]] += 1;
  ctx->maps_on_host = false;
  build_activity(ctx);
  ctx->halo_valid = false;
  if (ctx->equations == 1) {
    pe_status st = build_halo(ctx, s);
    if (st != PE_OK) return st;
  }
  ctx->partitioned = true;
  ctx->graph_valid = false;
  return PE_OK;
}

pe_status pe_set_state(pe_ctx* ctx, const double* u_leaf, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned) return fail(ctx, PE_ESTATE, "set_state before partition");
  if (!u_leaf) return fail(ctx, PE_EINVAL, "set_state: null");
  HIPCHK(launch_leaf_to_slot(ctx->n_e, (int)cap_of(ctx), nvars(ctx), nodes_per_elem(ctx), ctx->d_leaf_of_slot, u_leaf,
                             ctx->U, (hipStream_t)stream));
  ctx->state_valid = true;
  ctx->pending_leaf_state = false;
  return PE_OK;
}

pe_status pe_get_state(pe_ctx* ctx, double* u_leaf, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned || !ctx->state_valid) return fail(ctx, PE_ESTATE, "get_state without a state");
  if (!u_leaf) return fail(ctx, PE_EINVAL, "get_state: null");
  HIPCHK(launch_slot_to_leaf(ctx->n_e, (int)cap_of(ctx), nvars(ctx), nodes_per_elem(ctx), ctx->d_slot_of_leaf, ctx->U,
                             u_leaf, (hipStream_t)stream));
  return PE_OK;
}

pe_status pe_element_info(const pe_ctx* cctx, int32_t* leaf_of_slot, int32_t* member_of_slot) {
  pe_ctx* ctx = const_cast<pe_ctx*>(cctx);
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned) return fail(ctx, PE_ESTATE, "element_info before partition");
  if (!ctx->maps_on_host) {
    pe_status st = copy_maps(ctx, nullptr);
    if (st != PE_OK) return st;
  }
  if (leaf_of_slot) std::memcpy(leaf_of_slot, ctx->leaf_of_slot.data(), (size_t)ctx->n_e * 4);
  if (member_of_slot) std::memcpy(member_of_slot, ctx->mem_of_slot.data(), (size_t)ctx->n_e * 4);
  return PE_OK;
}

pe_status pe_node_coords(pe_ctx* ctx, double* x_leaf, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->have_mesh) return fail(ctx, PE_ESTATE, "node_coords before mesh_build");
  if (!x_leaf) return fail(ctx, PE_EINVAL, "node_coords: null");
  const int nd = nodes_per_elem(ctx), N = ctx->N, dim = ctx->dim;
  std::vector<double> x((size_t)ctx->n_e * dim * nd);
  for (int e = 0; e < ctx->n_e; ++e) {
    const int32_t* L = &ctx->leaves[4 * e];
    for (int node = 0; node < nd; ++node) {
      const int ijk[3] = {node % N, (node / N) % N, node / (N * N)};
      for (int d = 0; d < dim; ++d) {
        const double h = (ctx->hi[d] - ctx->lo[d]) / std::ldexp((double)ctx->n_root[d], L[0]);
        x[((size_t)e * dim + d) * nd + node] = ctx->lo[d] + h * L[1 + d] + 0.5 * h * (1.0 + ctx->ops.x[ijk[d]]);
      }
    }
  }
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(x_leaf, x.data(), x.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return PE_OK;
}

pe_status pe_rhs(pe_ctx* ctx, const double* u, double* du, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned) return fail(ctx, PE_ESTATE, "rhs before partition");
  if (!u || !du) return fail(ctx, PE_EINVAL, "rhs: null");
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.U = u;
  a.Kout = du;
  a.first = 1;          // F(U): stage values are U itself (src 0 for every member)
  a.n_act = ctx->n_e;
  set_shock_capturing_args(ctx, a);
  a.Fv = ctx->Fv;
  Mesh m = device_mesh(ctx);
  if (ctx->equations == 1)
    HIPCHK(launch_gradients(ctx->dim, ctx->N, a, m, ctx->ops, ctx->ph, (hipStream_t)stream));
  HIPCHK(launch_stage(ctx->dim, ctx->N, ctx->equations == 1, a, m, ctx->ops, ctx->ph, (hipStream_t)stream));
  return PE_OK;
}

pe_status pe_rhs_vjp(pe_ctx* ctx, const double* u, const double* w, double* out, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned) return fail(ctx, PE_ESTATE, "rhs_vjp before partition");
  if (ctx->equations != 0) return fail(ctx, PE_EUNSUPPORTED, "rhs_vjp: Euler only");
  if (ctx->sc_on) return fail(ctx, PE_EUNSUPPORTED, "rhs_vjp: not with shock capturing");
  if (!u || !w || !out) return fail(ctx, PE_EINVAL, "rhs_vjp: null");
  VjpArgs a;
  std::memset(&a, 0, sizeof a);
  a.U = u;                 // src 0 for every member: the state itself
  a.W = w;
  a.n_w = ctx->n_e;
  a.n_act = ctx->n_e;
  a.Gout = out;
  HIPCHK(launch_rhs_vjp(ctx->dim, ctx->N, a, device_mesh(ctx), ctx->ops, ctx->ph, (hipStream_t)stream));
  return PE_OK;
}

pe_status pe_adjoint_query(const pe_ctx* ctx, int64_t* bytes) {
  if (!ctx || !bytes) return PE_EINVAL;
  if (!ctx->have_coeffs || !ctx->bound) return PE_ESTATE;
  *bytes = (int64_t)(ctx->S + 2) * state_doubles(ctx) * (int64_t)sizeof(double);
  return PE_OK;
}

pe_status pe_adjoint_bind(pe_ctx* ctx, void* workspace) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->have_coeffs || !ctx->bound) return fail(ctx, PE_ESTATE, "adjoint_bind needs coefficients and a binding");
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(ctx, PE_EINVAL, "adjoint_bind: null or not 256-byte aligned");
  ctx->adj_ws = (char*)workspace;
  ctx->adj_S = ctx->S;
  ctx->adj_cap = cap_of(ctx);
  return PE_OK;
}

namespace {
// Checks shared by the adjoint step entry points.
pe_status adjoint_ready(pe_ctx* ctx, double dt, const char* who) {
  if (!ctx->partitioned) return fail(ctx, PE_ESTATE, "%s before partition", who);
  if (ctx->equations != 0) return fail(ctx, PE_EUNSUPPORTED, "%s: Euler only", who);
  if (ctx->general) return fail(ctx, PE_EUNSUPPORTED, "%s: classic stage pattern only", who);
  if (ctx->sc_on) return fail(ctx, PE_EUNSUPPORTED, "%s: not with shock capturing", who);
  if (!(dt > 0.0)) return fail(ctx, PE_EINVAL, "%s: dt must be > 0", who);
  if (!ctx->adj_ws || ctx->adj_S != ctx->S || ctx->adj_cap != cap_of(ctx))
    return fail(ctx, PE_ESTATE, "%s: adjoint workspace not bound for these coefficients and capacity", who);
  return PE_OK;
}

// Stage-value slot i (1 <= i < S, holding Y_{i+1}) of a record: state array i + off from ybase.
struct StageSlots {
  double* ybase;
  int off;
  int64_t sd;
  double* operator()(int i) const { return ybase + (int64_t)(i + off) * sd; }
};

// One step from u_n keeping what the reverse sweep reads: K_1 in K1 and the stage values
// Y_2..Y_S in the slots Y(1..S-1); U_{n+1} goes to u_next.
pe_status record_step(pe_ctx* ctx, double dt, const double* u_n, double* K1, StageSlots Y, double* u_next,
                      hipStream_t s) {
  const int S = ctx->S;
  Mesh m = device_mesh(ctx);
  for (int i = 0; i < S; ++i) {
    StageArgs a;
    fill_stage(ctx, i, dt, a);
    a.U = u_n;
    a.K1 = K1;
    a.Yin = i >= 1 ? Y(i) : ctx->Ya;
    a.Yout = i + 1 < S ? Y(i + 1) : ctx->Yb;
    classic_outputs(a);
    a.ACC = ctx->ACC;
    a.Uout = u_next;
    a.evals = nullptr;
    HIPCHK(launch_stage(ctx->dim, ctx->N, false, a, m, ctx->ops, ctx->ph, s));
  }
  return PE_OK;
}

// The reverse sweep of one step (lam_prev = Phi'(u_n)^T lam_next) from the recorded K_1 and
// stage values; the stage cotangents live in the adjoint workspace.
pe_status reverse_sweep(pe_ctx* ctx, double dt, const double* u_n, const double* K1, StageSlots Y,
                        const double* lam_next, double* lam_prev, hipStream_t s) {
  if (!ctx->halo_valid) {
    pe_status st = build_halo(ctx, s);
    if (st != PE_OK) return st;
  }
  const int64_t sd = state_doubles(ctx);
  const int S = ctx->S, R = ctx->R;
  double* base = (double*)ctx->adj_ws;
  double* Kcur = base + (int64_t)(S - 1) * sd;
  double* Kprev = Kcur + sd;
  double* K1bar = Kprev + sd;
  Mesh m = device_mesh(ctx);
  HIPCHK(launch_copy(lam_prev, lam_next, sd, s));
  HIPCHK(launch_scale(K1bar, lam_next, dt * ctx->b[0], sd, s));
  if (S > 1) HIPCHK(launch_scale(Kcur, lam_next, dt * ctx->b[S - 1], sd, s));
  for (int i = S - 1; i >= 1; --i) {
    StageArgs sa;
    fill_stage(ctx, i, dt, sa);
    VjpArgs a;
    std::memset(&a, 0, sizeof a);
    a.U = u_n;
    a.K1 = K1;
    a.Yin = Y(i);
    a.dt = dt;
    a.ci = ctx->c[i];
    for (int r = 0; r < kMaxMembers; ++r) a.src[r] = sa.src[r];
    a.W = Kcur;
    a.n_w = ctx->n_act[i];
    a.n_act = ctx->n_act[i];
    a.n_halo = ctx->halo_cnt[i];
    a.halo = ctx->d_halo + ctx->halo_off[i];
    a.Ubar = lam_prev;
    a.K1bar = K1bar;
    a.Kprev = i - 1 >= 1 ? Kprev : nullptr;
    a.lam = lam_next;
    a.bprev = ctx->b[i - 1];
    for (int r = 0; r < R; ++r) {
      const double a2 = ctx->a_sub[(size_t)r * S + i];     // a_{i+1,i} in 1-based numbering
      a.A1[r] = ctx->c[i] - a2;
      a.A2[r] = a2;
    }
    HIPCHK(launch_rhs_vjp(ctx->dim, ctx->N, a, m, ctx->ops, ctx->ph, s));
    std::swap(Kcur, Kprev);
  }
  {
    VjpArgs a;
    std::memset(&a, 0, sizeof a);
    a.U = u_n;
    a.W = K1bar;
    a.n_w = ctx->n_e;
    a.n_act = ctx->n_e;
    a.Ubar = lam_prev;
    HIPCHK(launch_rhs_vjp(ctx->dim, ctx->N, a, m, ctx->ops, ctx->ph, s));
  }
  return PE_OK;
}
}  // namespace

pe_status pe_step_adjoint(pe_ctx* ctx, double dt, const double* u_n, const double* lam_next, double* lam_prev,
                          void* stream) {
  if (!ctx) return PE_EINVAL;
  pe_status st = adjoint_ready(ctx, dt, "step_adjoint");
  if (st != PE_OK) return st;
  if (!u_n || !lam_next || !lam_prev) return fail(ctx, PE_EINVAL, "step_adjoint: null");
  if (lam_prev == lam_next || lam_prev == u_n) return fail(ctx, PE_EINVAL, "step_adjoint: lam_prev must not alias");
  hipStream_t s = (hipStream_t)stream;
  const int64_t sd = state_doubles(ctx);
  double* base = (double*)ctx->adj_ws;
  const StageSlots Y{base, -1, sd};   // Y_2 .. Y_S in workspace arrays 0 .. S-2
  // forward recomputation of the step from u_n, keeping every stage value
  st = record_step(ctx, dt, u_n, ctx->K1, Y, ctx->Tmp, s);
  if (st != PE_OK) return st;
  return reverse_sweep(ctx, dt, u_n, ctx->K1, Y, lam_next, lam_prev, s);
}

pe_status pe_adjoint_record_size(const pe_ctx* ctx, int64_t* doubles) {
  if (!ctx || !doubles) return PE_EINVAL;
  if (!ctx->have_coeffs || !ctx->bound) return PE_ESTATE;
  *doubles = (int64_t)ctx->S * state_doubles(ctx);
  return PE_OK;
}

pe_status pe_step_record(pe_ctx* ctx, double dt, const double* u_n, double* u_next, double* record, void* stream) {
  if (!ctx) return PE_EINVAL;
  pe_status st = adjoint_ready(ctx, dt, "step_record");
  if (st != PE_OK) return st;
  if (!u_n || !u_next || !record) return fail(ctx, PE_EINVAL, "step_record: null");
  const int64_t sd = state_doubles(ctx);
  const double* r0 = record;
  const double* r1 = record + (int64_t)ctx->S * sd;
  auto overlaps = [&](const double* p) { return p && p + sd > r0 && p < r1; };
  if (u_next == u_n || overlaps(u_n) || overlaps(u_next))
    return fail(ctx, PE_EINVAL, "step_record: u_n, u_next and record must not overlap");
  const StageSlots Y{record, 0, sd};   // K_1 in array 0, Y_2 .. Y_S in arrays 1 .. S-1
  return record_step(ctx, dt, u_n, record, Y, u_next, (hipStream_t)stream);
}

pe_status pe_step_adjoint_recorded(pe_ctx* ctx, double dt, const double* u_n, const double* record,
                                   const double* lam_next, double* lam_prev, void* stream) {
  if (!ctx) return PE_EINVAL;
  pe_status st = adjoint_ready(ctx, dt, "step_adjoint_recorded");
  if (st != PE_OK) return st;
  if (!u_n || !record || !lam_next || !lam_prev) return fail(ctx, PE_EINVAL, "step_adjoint_recorded: null");
  const int64_t sd = state_doubles(ctx);
  const double* r1 = record + (int64_t)ctx->S * sd;
  if (lam_prev == lam_next || lam_prev == u_n || (lam_prev + sd > record && lam_prev < r1))
    return fail(ctx, PE_EINVAL, "step_adjoint_recorded: lam_prev must not alias");
  const StageSlots Y{const_cast<double*>(record), 0, sd};   // read only here
  return reverse_sweep(ctx, dt, u_n, record, Y, lam_next, lam_prev, (hipStream_t)stream);
}

namespace {
pe_status prof_event(pe_ctx* ctx, hipStream_t s) {
  if (ctx->ev_used == ctx->ev_pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    ctx->ev_pool.push_back(e);
  }
  HIPCHK(hipEventRecord(ctx->ev_pool[ctx->ev_used++], s));
  return PE_OK;
}

// Next pair of pool events (start, end) for a dispatch-recorded timing of kernel `kind`.
pe_status prof_pair(pe_ctx* ctx, int kind, hipEvent_t* e0, hipEvent_t* e1) {
  while (ctx->ev_pool.size() < ctx->ev_used + 2) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    ctx->ev_pool.push_back(e);
  }
  if (ctx->ev_kind.size() < ctx->ev_pool.size() / 2) ctx->ev_kind.resize(ctx->ev_pool.size() / 2);
  ctx->ev_kind[ctx->ev_used / 2] = kind;
  *e0 = ctx->ev_pool[ctx->ev_used++];
  *e1 = ctx->ev_pool[ctx->ev_used++];
  return PE_OK;
}

// Sum the event pairs recorded so far per kernel (waits for them).
pe_status prof_collect(pe_ctx* ctx) {
  for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
    HIPCHK(hipEventSynchronize(ctx->ev_pool[i + 1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_pool[i], ctx->ev_pool[i + 1]));
    ctx->prof_ms[ctx->ev_kind[i / 2]] += ms;
  }
  ctx->ev_used = 0;
  return PE_OK;
}
}  // namespace

namespace {
// Enqueue the launches of one P-ERK step on stream s (optionally timing every stage launch).
pe_status enqueue_step(pe_ctx* ctx, double dt, hipStream_t s, bool timed) {
  Mesh m = device_mesh(ctx);
  const bool in_place = last_stage_in_place_safe(ctx);
  for (int i = 0; i < ctx->S; ++i) {
    StageArgs a;
    fill_stage(ctx, i, dt, a);
    a.U = ctx->U;
    a.K1 = ctx->K1;
    set_stage_buffers(ctx, i, a);
    a.ACC = ctx->ACC;
    a.Uout = in_place ? ctx->U : ctx->Tmp;
    a.evals = ctx->d_evals;
    a.Fv = ctx->Fv;
    if (!a.U || !a.K1 || !a.Yin || !a.ACC || !a.Uout || (ctx->equations == 1 && !a.Fv))
      return fail(ctx, PE_ESTATE, "step: stage buffers not bound");
    if (ctx->equations == 1) {
      a.n_halo = ctx->halo_cnt[i];
      a.halo = ctx->d_halo + ctx->halo_off[i];
      if (timed && a.n_act + a.n_halo > 0) {
        hipEvent_t e0, e1;
        pe_status st = prof_pair(ctx, 1, &e0, &e1);
        if (st != PE_OK) return st;
        HIPCHK(launch_gradients(ctx->dim, ctx->N, a, m, ctx->ops, ctx->ph, s, e0, e1));
        ctx->prof_launches[1] += 1;
        ctx->prof_elems[1] += a.n_act + a.n_halo;
      } else {
        HIPCHK(launch_gradients(ctx->dim, ctx->N, a, m, ctx->ops, ctx->ph, s));
      }
    }
    if (timed && a.n_act > 0) {
      // events recorded by the dispatch itself around the stage kernel
      hipEvent_t e0, e1;
      pe_status st = prof_pair(ctx, 0, &e0, &e1);
      if (st != PE_OK) return st;
      HIPCHK(launch_stage(ctx->dim, ctx->N, ctx->equations == 1, a, m, ctx->ops, ctx->ph, s, e0, e1));
      ctx->prof_launches[0] += 1;
      ctx->prof_elems[0] += a.n_act;
      if (ctx->ev_used >= 4096) {
        st = prof_collect(ctx);
        if (st != PE_OK) return st;
      }
    } else {
      HIPCHK(launch_stage(ctx->dim, ctx->N, ctx->equations == 1, a, m, ctx->ops, ctx->ph, s));
    }
  }
  if (!in_place) HIPCHK(launch_copy(ctx->U, ctx->Tmp, state_doubles(ctx), s));
  return PE_OK;
}

// Capture one step into an executable graph (on a private stream of default priority).
pe_status capture_step(pe_ctx* ctx, double dt) {
  if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  pe_status st = enqueue_step(ctx, dt, ctx->cap_stream, false);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
  if (st != PE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  HIPCHK(e);
  // the kernel body of every stage launch: a partition that moves a stage's active count across
  // the point where the 2D p=3 launches change body changes that node's kernel and block size,
  // which an in-place update is not relied on to carry over: then the graph is instantiated anew
  std::vector<int> bodies(ctx->S);
  for (int i = 0; i < ctx->S; ++i) bodies[i] = stage_body_id(ctx->dim, ctx->N, ctx->n_act[i], ctx->sc_on);
  const bool same_bodies = bodies == ctx->graph_bodies;
  ctx->graph_bodies = bodies;
  if (ctx->gexec && same_bodies) {
    // same launches with new sizes (after a re-partition): update the executable graph in
    // place, which costs less than instantiating a new one; otherwise replace it
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    if (hipGraphExecUpdate(ctx->gexec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
      (void)hipGraphDestroy(g);
      ctx->graph_valid = true;
      ctx->graph_dt = dt;
      return PE_OK;
    }
    (void)hipGetLastError();
  }
  if (ctx->gexec) {
    HIPCHK(hipGraphExecDestroy(ctx->gexec));
    ctx->gexec = nullptr;
  }
  e = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e);
  ctx->graph_valid = true;
  ctx->graph_dt = dt;
  return PE_OK;
}
}  // namespace

pe_status pe_step(pe_ctx* ctx, double dt, int n_steps, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned || !ctx->state_valid) return fail(ctx, PE_ESTATE, "step needs a partition and a state");
  if (!(dt > 0.0) || n_steps < 0) return fail(ctx, PE_EINVAL, "step: dt must be > 0 and n_steps >= 0");
  hipStream_t s = (hipStream_t)stream;
  if (ctx->profiling || !ctx->graphs_enabled) {
    for (int step = 0; step < n_steps; ++step) {
      pe_status st = enqueue_step(ctx, dt, s, ctx->profiling);
      if (st != PE_OK) return st;
    }
    return PE_OK;
  }
  if (n_steps == 0) return PE_OK;
  int replays = n_steps;
  if (!ctx->graph_valid || ctx->graph_dt != dt) {
    // the first step after a re-partition or a new step size goes out as plain launches, so
    // that the device starts at once; the capture and graph update below (host work of the
    // order of 100 us) then run while those kernels execute
    pe_status st = enqueue_step(ctx, dt, s, false);
    if (st != PE_OK) return st;
    --replays;
    if (capture_step(ctx, dt) != PE_OK) {
      // graph replay is an optimisation: without a graph the context goes on with plain
      // launches (the step above has already advanced the state)
      (void)hipGetLastError();
      ctx->graphs_enabled = false;
      for (int step = 0; step < replays; ++step) {
        st = enqueue_step(ctx, dt, s, false);
        if (st != PE_OK) return st;
      }
      return PE_OK;
    }
  }
  for (int step = 0; step < replays; ++step) HIPCHK(hipGraphLaunch(ctx->gexec, s));
  return PE_OK;
}

pe_status pe_set_graph_replay(pe_ctx* ctx, int on) {
  if (!ctx) return PE_EINVAL;
  ctx->graphs_enabled = on != 0;
  ctx->graph_valid = false;
  return PE_OK;
}

pe_status pe_reserve(pe_ctx* ctx, int64_t max_elements) {
  if (!ctx) return PE_EINVAL;
  if (max_elements < 0 || max_elements > (int64_t)1 << 28) return fail(ctx, PE_EINVAL, "reserve: bad capacity");
  ctx->capacity = max_elements;
  ctx->bound = false;
  ctx->partitioned = false;
  ctx->graph_valid = false;
  ctx->state_valid = false;
  ctx->pending_leaf_state = false;
  return PE_OK;
}

pe_status pe_get_leaves(const pe_ctx* ctx, int32_t* leaves, int64_t* n) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->have_mesh) return fail(const_cast<pe_ctx*>(ctx), PE_ESTATE, "get_leaves before mesh_build");
  if (n) *n = ctx->n_e;
  if (leaves) std::memcpy(leaves, ctx->leaves.data(), ctx->leaves.size() * 4);
  return PE_OK;
}

pe_status pe_set_shock_capturing(pe_ctx* ctx, int on, double alpha_max, double alpha_min) {
  if (!ctx) return PE_EINVAL;
  if (on && (ctx->dim != 2 || ctx->equations != 0))
    return fail(ctx, PE_EUNSUPPORTED, "shock capturing: 2D Euler only");
  if (on && ctx->general) return fail(ctx, PE_EUNSUPPORTED, "shock capturing: classic stage pattern only");
  if (on && !(alpha_min >= 0.0 && alpha_min <= alpha_max && alpha_max <= 1.0))
    return fail(ctx, PE_EINVAL, "shock capturing: need 0 <= alpha_min <= alpha_max <= 1");
  ctx->sc_on = on != 0;
  if (on) {
    ctx->sc_amax = alpha_max;
    ctx->sc_amin = alpha_min;
  }
  ctx->graph_valid = false;
  return PE_OK;
}

pe_status pe_set_amr_indicator(pe_ctx* ctx, int kind, int variable, double f_wave) {
  if (!ctx) return PE_EINVAL;
  if (kind == PE_INDICATOR_DENSITY_GRADIENT) {
    ctx->ind_kind = kind;
    return PE_OK;
  }
  if (kind == PE_INDICATOR_HENNEMANN_GASSNER) {
    if (variable != 0) return fail(ctx, PE_EINVAL, "indicator: Hennemann-Gassner on the density (variable 0) only");
    if (ctx->dim != 2) return fail(ctx, PE_EUNSUPPORTED, "indicator: Hennemann-Gassner in 2D only");
    ctx->ind_kind = kind;
    ctx->ind_var = 0;
    return PE_OK;
  }
  if (kind != PE_INDICATOR_LOHNER) return fail(ctx, PE_EINVAL, "indicator %d unknown", kind);
  if (variable < 0 || variable > ctx->dim + 1)
    return fail(ctx, PE_EINVAL, "indicator: variable %d outside [0, %d]", variable, ctx->dim + 1);
  if (!(f_wave >= 0.0) || !std::isfinite(f_wave)) return fail(ctx, PE_EINVAL, "indicator: f_wave must be >= 0");
  ctx->ind_kind = kind;
  ctx->ind_var = variable;
  ctx->ind_fwave = f_wave;
  return PE_OK;
}

pe_status pe_amr_indicator(pe_ctx* ctx, double* eta_leaf, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned || !ctx->state_valid) return fail(ctx, PE_ESTATE, "indicator needs a partition and a state");
  if (!eta_leaf) return fail(ctx, PE_EINVAL, "indicator: null");
  hipStream_t s = (hipStream_t)stream;
  Mesh m = device_mesh(ctx);
  if (ctx->ind_kind == PE_INDICATOR_LOHNER)
    HIPCHK(launch_indicator_lohner(ctx->dim, ctx->N, ctx->n_e, (int)cap_of(ctx), ctx->d_slot_of_leaf, ctx->U,
                                   ctx->ind_var, ctx->ind_fwave, ctx->ph.gamma, ctx->d_eta, s));
  else if (ctx->ind_kind == PE_INDICATOR_HENNEMANN_GASSNER) {
    StageArgs a;
    set_shock_capturing_args(ctx, a);
    HIPCHK(launch_indicator_hg(ctx->dim, ctx->N, ctx->n_e, (int)cap_of(ctx), ctx->d_slot_of_leaf, ctx->U,
                               ctx->ops.dD, a.sc_T, a.sc_slope, ctx->d_eta, s));
  }
  else
    HIPCHK(launch_indicator(ctx->dim, ctx->N, ctx->n_e, (int)cap_of(ctx), ctx->d_slot_of_leaf, ctx->d_lev_leaf,
                            ctx->U, ctx->ops, m, ctx->d_eta, s));
  const size_t bytes = (size_t)ctx->n_e * 8;
  pe_status st = stage_reserve(ctx, bytes);
  if (st != PE_OK) return st;
  HIPCHK(hipMemcpyAsync(ctx->h_stage, ctx->d_eta, bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::memcpy(eta_leaf, ctx->h_stage, bytes);
  return PE_OK;
}

pe_status pe_max_dt(pe_ctx* ctx, double cfl, double* dt_out, double* beta_of_level, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned || !ctx->state_valid) return fail(ctx, PE_ESTATE, "max_dt needs a partition and a state");
  if (!dt_out) return fail(ctx, PE_EINVAL, "max_dt: null dt_out");
  if (!(cfl > 0.0)) return fail(ctx, PE_EINVAL, "max_dt: cfl must be positive");
  hipStream_t s = (hipStream_t)stream;
  Mesh m = device_mesh(ctx);
  HIPCHK(launch_wave_speed(ctx->dim, ctx->N, ctx->n_e, ctx->U, ctx->ph, m, ctx->d_eta, ctx->d_beta, s));
  double w[kMaxLevels];
  HIPCHK(hipMemcpyAsync(w, ctx->d_beta, sizeof(w), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double wmax = 0.0;
  for (int l = 0; l < kMaxLevels; ++l) {
    if (!std::isfinite(w[l])) return fail(ctx, PE_ENONFINITE, "max_dt: non-finite wave speed on level %d", l);
    if (beta_of_level) beta_of_level[l] = w[l] > 0.0 ? 1.0 / w[l] : 0.0;
    wmax = std::max(wmax, w[l]);
  }
  if (!(wmax > 0.0)) return fail(ctx, PE_ENONFINITE, "max_dt: zero wave speed");
  *dt_out = cfl / wmax;
  return PE_OK;
}

pe_status pe_max_dt_noalloc(pe_ctx* ctx, double cfl, double* dt_dev, double* beta_dev, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned || !ctx->state_valid)
    return fail(ctx, PE_ESTATE, "max_dt_noalloc needs a partition and a state");
  if (!dt_dev) return fail(ctx, PE_EINVAL, "max_dt_noalloc: null dt");
  if (!(cfl > 0.0)) return fail(ctx, PE_EINVAL, "max_dt_noalloc: cfl must be positive");
  if (ctx->n_e > kNoAllocMaxElements)
    return fail(ctx, PE_EINVAL, "max_dt_noalloc: %d elements exceed the static scratch of %d", ctx->n_e,
                kNoAllocMaxElements);
  HIPCHK(launch_max_dt_noalloc(ctx->dim, ctx->N, ctx->n_e, ctx->U, ctx->ph, device_mesh(ctx), cfl, dt_dev, beta_dev,
                               (hipStream_t)stream));
  return PE_OK;
}

namespace {
// spread the low 21 bits of x to every 2nd (dim 2) or 3rd (dim 3) bit
inline uint64_t spread2(uint64_t x) {
  x &= 0x1FFFFFull;
  x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
  x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}
inline uint64_t spread3(uint64_t x) {
  x &= 0x1FFFFFull;
  x = (x | (x << 32)) & 0x001F00000000FFFFull;
  x = (x | (x << 16)) & 0x001F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}
// Morton key of a leaf: coordinates at level kMaxLevels-1, bit b of axis d at position dim*b + d
uint64_t morton_key(const int32_t* L, int dim) {
  const int shift = kMaxLevels - 1 - L[0];
  const uint64_t x = (uint64_t)L[1] << shift, y = (uint64_t)L[2] << shift;
  if (dim == 2) return spread2(x) | (spread2(y) << 1);
  const uint64_t z = (uint64_t)L[3] << shift;
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
}  // namespace

pe_status pe_adapt(pe_ctx* ctx, const int8_t* flags, int level_min, int level_max, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned || !ctx->state_valid) return fail(ctx, PE_ESTATE, "adapt needs a partition and a state");
  if (!flags) return fail(ctx, PE_EINVAL, "adapt: null flags");
  if (level_min < 0 || level_max < level_min || level_max >= kMaxLevels)
    return fail(ctx, PE_EINVAL, "adapt: bad level range [%d, %d]", level_min, level_max);
  const int n = ctx->n_e, dim = ctx->dim, nf = 2 * dim, nch = 1 << dim;
  std::vector<int> lev(n), t(n);
  for (int e = 0; e < n; ++e) {
    lev[e] = ctx->leaves[4 * e];
    t[e] = lev[e] + ((flags[e] > 0 && lev[e] < level_max) ? 1 : 0);
  }
  auto for_nbrs = [&](int e, auto&& fn) {
    for (int f = 0; f < nf; ++f) {
      const int kind = face_kind(ctx->fk_leaf[(size_t)e * nf + f]);
      const int cnt = kind == kCoarseSide ? (1 << (dim - 1)) : 1;
      for (int q = 0; q < cnt; ++q) fn(ctx->fn_leaf[((size_t)e * nf + f) * 4 + q]);
    }
  };
  // 2:1 balance after refinement: face neighbours may differ by at most one target level
  for (bool changed = true; changed;) {
    changed = false;
    for (int e = 0; e < n; ++e)
      for_nbrs(e, [&](int g) {
        if (t[e] - t[g] >= 2) {
          t[g] = lev[g] + 1;
          changed = true;
        }
      });
  }
  // coarsening of complete sibling families
  std::unordered_map<uint64_t, std::vector<int>, KeyHash> fams;
  for (int e = 0; e < n; ++e) {
    if (lev[e] <= level_min || flags[e] >= 0 || t[e] != lev[e]) continue;
    const int32_t* L = &ctx->leaves[4 * e];
    fams[cell_key(lev[e] - 1, L[1] >> 1, L[2] >> 1, dim == 3 ? (L[3] >> 1) : 0)].push_back(e);
  }
  std::vector<int> parent_of(n, -1);   // index of the family's first member for coarsened leaves
  std::unordered_map<int, std::vector<int>> members;   // first member -> the family
  for (auto& kv : fams) {
    auto& mem = kv.second;
    if ((int)mem.size() != nch) continue;
    bool ok = true;
    for (int e : mem)
      for_nbrs(e, [&](int g) {
        if (std::find(mem.begin(), mem.end(), g) == mem.end() && t[g] > lev[e]) ok = false;
      });
    if (!ok) continue;
    const int first = *std::min_element(mem.begin(), mem.end());
    for (int e : mem) parent_of[e] = first;
    members[first] = mem;
  }
  // new leaves with their projection plans
  struct NewLeaf {
    std::array<int32_t, 4> L;
    std::array<int32_t, 10> plan;
    uint64_t key;
  };
  std::vector<NewLeaf> nl;
  nl.reserve(n * 2);
  for (int e = 0; e < n; ++e) {
    const int32_t* L = &ctx->leaves[4 * e];
    NewLeaf x{};
    if (parent_of[e] >= 0) {
      if (parent_of[e] != e) continue;
      x.L = {lev[e] - 1, L[1] >> 1, L[2] >> 1, dim == 3 ? (L[3] >> 1) : 0};
      x.plan[0] = 2;
      for (int g : members[e]) {
        const int32_t* G = &ctx->leaves[4 * g];
        const int pos = (G[1] & 1) | ((G[2] & 1) << 1) | (dim == 3 ? ((G[3] & 1) << 2) : 0);
        x.plan[2 + pos] = g;
      }
      nl.push_back(x);
    } else if (t[e] == lev[e] + 1) {
      for (int c = 0; c < nch; ++c) {
        NewLeaf y{};
        y.L = {lev[e] + 1, 2 * L[1] + (c & 1), 2 * L[2] + ((c >> 1) & 1), dim == 3 ? 2 * L[3] + ((c >> 2) & 1) : 0};
        y.plan[0] = 1;
        y.plan[1] = c;
        y.plan[2] = e;
        nl.push_back(y);
      }
    } else {
      x.L = {L[0], L[1], L[2], L[3]};
      x.plan[0] = 0;
      x.plan[2] = e;
      nl.push_back(x);
    }
  }
  if ((int64_t)nl.size() > cap_of(ctx))
    return fail(ctx, PE_ENOMEM, "adapt: %zu elements exceed the reserved capacity %lld", nl.size(),
                (long long)cap_of(ctx));
  std::vector<std::pair<uint64_t, int32_t>> order(nl.size());
  for (size_t i = 0; i < nl.size(); ++i) order[i] = {morton_key(nl[i].L.data(), dim), (int32_t)i};
  std::sort(order.begin(), order.end());
  // uploads through the pinned staging buffer: the plan now, the connectivity after it is built
  const size_t nn_new = nl.size();
  const size_t plan_bytes = align256(nn_new * 40), fk_bytes = align256(nn_new * nf * 4);
  const size_t fn_bytes = align256(nn_new * nf * 16), lev_bytes = align256(nn_new * 4);
  {
    pe_status st = stage_reserve(ctx, plan_bytes + fk_bytes + fn_bytes + lev_bytes);
    if (st != PE_OK) return st;
  }
  char* const stage = static_cast<char*>(ctx->h_stage);
  int32_t* plan = reinterpret_cast<int32_t*>(stage);
  std::vector<int32_t> leaves(nn_new * 4);
  for (size_t i = 0; i < nn_new; ++i) {
    const NewLeaf& x = nl[(size_t)order[i].second];
    std::memcpy(&plan[i * 10], x.plan.data(), 40);
    std::memcpy(&leaves[i * 4], x.L.data(), 16);
  }
  hipStream_t s = (hipStream_t)stream;
  // evaluation counts of the old partition into the per-member totals
  HIPCHK(launch_fold_evals(ctx->n_e, device_mesh(ctx), ctx->d_evals, ctx->d_counter, s));
  // project the old state (slot layout, old slot map) onto the new leaves (leaf layout, in Tmp)
  HIPCHK(hipMemcpyAsync(ctx->d_plan, plan, nn_new * 40, hipMemcpyHostToDevice, s));
  {
    pe_status st = stage_mark(ctx, s);
    if (st != PE_OK) return st;
  }
  HIPCHK(launch_project(dim, ctx->N, (int)nl.size(), (int)cap_of(ctx), ctx->d_plan, ctx->d_slot_of_leaf, ctx->U,
                        ctx->ops, ctx->Tmp, s));
  // new forest
  std::vector<int32_t> old_leaves;
  old_leaves.swap(ctx->leaves);
  const int old_n = ctx->n_e;
  ctx->leaves.swap(leaves);
  ctx->n_e = (int)nl.size();
  pe_status st = build_connectivity(ctx);
  if (st != PE_OK) {
    ctx->leaves.swap(old_leaves);
    ctx->n_e = old_n;
    build_connectivity(ctx);
    return st;
  }
  const int nn = ctx->n_e;
  // the staging region after the plan is not read by the plan copy still in flight
  char* const up = stage + plan_bytes;
  std::memcpy(up, ctx->fk_leaf.data(), (size_t)nn * nf * 4);
  std::memcpy(up + fk_bytes, ctx->fn_leaf.data(), (size_t)nn * nf * 16);
  std::memcpy(up + fk_bytes + fn_bytes, ctx->lev_leaf.data(), (size_t)nn * 4);
  HIPCHK(hipMemcpyAsync(ctx->d_fk_leaf, up, (size_t)nn * nf * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->d_fn_leaf, up + fk_bytes, (size_t)nn * nf * 16, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->d_lev_leaf, up + fk_bytes + fn_bytes, (size_t)nn * 4, hipMemcpyHostToDevice, s));
  {
    pe_status st2 = stage_mark(ctx, s);
    if (st2 != PE_OK) return st2;
  }
  // no wait here: what follows on the host reads only host data, the device work is in order
  ctx->partitioned = false;
  ctx->graph_valid = false;
  ctx->state_valid = false;
  ctx->pending_leaf_state = true;
  return PE_OK;
}

pe_status pe_amr_cycle(pe_ctx* ctx, double refine_above, double coarsen_below, int level_min, int level_max,
                       const int32_t* member_of_level, int n_levels, int8_t* flags_host, int64_t* n_leaves,
                       void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!member_of_level && !ctx->have_rule)
    return fail(ctx, PE_ESTATE, "amr_cycle: no member_of_level and no level rule set");
  const int n = ctx->n_e;
  std::vector<double> eta(n);
  pe_status st = pe_amr_indicator(ctx, eta.data(), stream);
  if (st != PE_OK) return st;
  std::vector<int8_t> flags(n);
  for (int e = 0; e < n; ++e) {
    int8_t f = 0;
    if (eta[e] > refine_above) f = 1;
    if (eta[e] < coarsen_below) f = -1;
    flags[e] = f;
  }
  if (flags_host) std::memcpy(flags_host, flags.data(), (size_t)n);
  st = pe_adapt(ctx, flags.data(), level_min, level_max, stream);
  if (st != PE_OK) return st;
  if (ctx->profiling) {
    // the re-partition on its own: from an idle stream to the end of its kernels
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    const auto t0 = std::chrono::steady_clock::now();
    st = pe_partition(ctx, member_of_level, n_levels, stream);
    if (st != PE_OK) return st;
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    ctx->prof_ms[2] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ctx->prof_launches[2] += 1;
    ctx->prof_elems[2] += ctx->n_e;
  } else {
    st = pe_partition(ctx, member_of_level, n_levels, stream);
    if (st != PE_OK) return st;
  }
  if (n_leaves) *n_leaves = ctx->n_e;
  return PE_OK;
}

pe_status pe_orthogonalize_scratch(int k, int64_t* doubles) {
  if (k < 0 || k > (1 << 20) || !doubles) return PE_EINVAL;
  *doubles = multi_dot_scratch_doubles(k > 0 ? k : 1) + (k > 0 ? k : 1);
  return PE_OK;
}

pe_status pe_orthogonalize(pe_ctx* ctx, const double* V, int k, int64_t ldv, double* w, int64_t n, double* scratch,
                           double* h_host, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (k < 0 || n <= 0 || !w || !scratch || !h_host || (k > 0 && (!V || ldv < n)))
    return fail(ctx, PE_EINVAL, "orthogonalize: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const int kk = k > 0 ? k : 1;
  double* hd = scratch + multi_dot_scratch_doubles(kk);    // [k] projections of one pass
  std::vector<double> h(k, 0.0), hp(kk);
  for (int pass = 0; pass < 2 && k > 0; ++pass) {
    HIPCHK(launch_multi_dot(k, V, ldv, w, n, scratch, hd, s));
    HIPCHK(launch_multi_axpy(k, V, ldv, hd, w, n, s));
    HIPCHK(hipMemcpyAsync(hp.data(), hd, (size_t)k * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j) h[j] += hp[j];
  }
  double nn = 0.0;
  HIPCHK(launch_multi_dot(1, w, n, w, n, scratch, hd, s));
  HIPCHK(hipMemcpyAsync(&nn, hd, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double norm = std::sqrt(nn);
  for (int j = 0; j < k; ++j) h_host[j] = h[j];
  h_host[k] = norm;
  if (norm > 0.0) HIPCHK(launch_scale(w, w, 1.0 / norm, n, s));
  return PE_OK;
}

pe_status pe_rhs_jvp_fd(pe_ctx* ctx, const double* u, const double* v, double eps, double* out, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned) return fail(ctx, PE_ESTATE, "rhs_jvp_fd before partition");
  if (!u || !v || !out) return fail(ctx, PE_EINVAL, "rhs_jvp_fd: null");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ctx, PE_EINVAL, "rhs_jvp_fd: eps must be positive");
  const int64_t sd = state_doubles(ctx);
  if (sd < multi_dot_scratch_doubles(1) + 2) return fail(ctx, PE_EINVAL, "rhs_jvp_fd: mesh too small");
  hipStream_t s = (hipStream_t)stream;
  // step h = eps |u|_2 / |v|_2 (relative perturbation eps), norms reduced on the device
  double nrm[2];
  HIPCHK(launch_multi_dot(1, u, sd, u, sd, ctx->Ya, ctx->Ya + sd - 2, s));
  HIPCHK(launch_multi_dot(1, v, sd, v, sd, ctx->Ya, ctx->Ya + sd - 1, s));
  HIPCHK(hipMemcpyAsync(nrm, ctx->Ya + sd - 2, 16, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!(nrm[1] > 0.0)) return fail(ctx, PE_EINVAL, "rhs_jvp_fd: zero direction");
  const double h = eps * std::sqrt(nrm[0] > 0.0 ? nrm[0] : 1.0) / std::sqrt(nrm[1]);
  HIPCHK(launch_axpy_to(ctx->Ya, u, h, v, sd, s));
  HIPCHK(launch_axpy_to(ctx->Tmp, u, -h, v, sd, s));
  // the right-hand side writes the element slots only: the padding slots of the reserved
  // capacity must read zero in the difference
  if (cap_of(ctx) > ctx->n_e) {
    HIPCHK(hipMemsetAsync(ctx->Yb, 0, (size_t)sd * 8, s));
    HIPCHK(hipMemsetAsync(ctx->ACC, 0, (size_t)sd * 8, s));
  }
  pe_status st = pe_rhs(ctx, ctx->Ya, ctx->Yb, stream);
  if (st != PE_OK) return st;
  st = pe_rhs(ctx, ctx->Tmp, ctx->ACC, stream);
  if (st != PE_OK) return st;
  HIPCHK(launch_diff_scale(out, ctx->Yb, ctx->ACC, 0.5 / h, sd, s));
  return PE_OK;
}

pe_status pe_rhs_jvp(pe_ctx* ctx, const double* u, const double* v, double* t, double* f, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->partitioned) return fail(ctx, PE_ESTATE, "rhs_jvp before partition");
  if (ctx->equations != 0) return fail(ctx, PE_EUNSUPPORTED, "rhs_jvp: Euler only");
  if (ctx->sc_on) return fail(ctx, PE_EUNSUPPORTED, "rhs_jvp: not with shock capturing");
  if (!u || !v || !t) return fail(ctx, PE_EINVAL, "rhs_jvp: null");
  HIPCHK(launch_rhs_jvp(ctx->dim, ctx->N, (int)ctx->n_e, u, v, t, f, device_mesh(ctx), ctx->ops, ctx->ph,
                        (hipStream_t)stream));
  return PE_OK;
}

pe_status pe_device_math(pe_ctx* ctx, const double* x, int64_t n, double* out, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (n < 0 || (n > 0 && (!x || !out))) return fail(ctx, PE_EINVAL, "device_math: bad arguments");
  HIPCHK(launch_device_math(n, x, out, (hipStream_t)stream));
  return PE_OK;
}

pe_status pe_quadrature(const pe_ctx* ctx, double* nodes, double* weights) {
  if (!ctx) return PE_EINVAL;
  for (int i = 0; i < ctx->N; ++i) {
    if (nodes) nodes[i] = ctx->ops.x[i];
    if (weights) weights[i] = ctx->ops.w[i];
  }
  return PE_OK;
}

pe_status pe_mortar_operators(const pe_ctx* ctx, double* P, double* R) {
  if (!ctx) return PE_EINVAL;
  const int N = ctx->N;
  for (int m = 0; m < 2; ++m)
    for (int i = 0; i < N * N; ++i) {
      if (P) P[m * N * N + i] = ctx->ops.P[m][i];
      if (R) R[m * N * N + i] = ctx->ops.R[m][i];
    }
  return PE_OK;
}

pe_status pe_set_profiling(pe_ctx* ctx, int on) {
  if (!ctx) return PE_EINVAL;
  ctx->profiling = on != 0;
  ctx->ev_used = 0;
  for (int k = 0; k < 3; ++k) {
    ctx->prof_ms[k] = 0.0;
    ctx->prof_launches[k] = 0;
    ctx->prof_elems[k] = 0;
  }
  return PE_OK;
}

pe_status pe_profile_stats(pe_ctx* ctx, double* kernel_ms, int64_t* launches, int64_t* element_stages) {
  return pe_profile_kernel_stats(ctx, 0, kernel_ms, launches, element_stages);
}

pe_status pe_profile_kernel_stats(pe_ctx* ctx, int kernel, double* kernel_ms, int64_t* launches, int64_t* elements) {
  if (!ctx) return PE_EINVAL;
  if (kernel < 0 || kernel > 2) return fail(ctx, PE_EINVAL, "profile_kernel_stats: kernel must be 0, 1 or 2");
  pe_status st = prof_collect(ctx);
  if (st != PE_OK) return st;
  if (kernel_ms) *kernel_ms = ctx->prof_ms[kernel];
  if (launches) *launches = ctx->prof_launches[kernel];
  if (elements) *elements = ctx->prof_elems[kernel];
  return PE_OK;
}

pe_status pe_counters(pe_ctx* ctx, int64_t* total, int64_t* per_member, int reset, void* stream) {
  if (!ctx) return PE_EINVAL;
  if (!ctx->bound) return fail(ctx, PE_ESTATE, "counters before bind");
  hipStream_t s = (hipStream_t)stream;
  if (ctx->partitioned) HIPCHK(launch_fold_evals(ctx->n_e, device_mesh(ctx), ctx->d_evals, ctx->d_counter, s));
  unsigned long long h[kMaxMembers];
  HIPCHK(hipMemcpyAsync(h, ctx->d_counter, sizeof h, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int64_t t = 0;
  for (int r = 0; r < ctx->R; ++r) {
    t += (int64_t)h[r];
    if (per_member) per_member[r] = (int64_t)h[r];
  }
  if (total) *total = t;
  if (reset) {
    HIPCHK(hipMemsetAsync(ctx->d_counter, 0, sizeof h, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return PE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batched runs
struct pe_batch {
  std::vector<pe_ctx*> runs;             // caller's order
  std::vector<int> order;                // internal position -> caller's index (degree 3 first)
  int split = 0;                         // internal positions [0, split) have N = 4, the rest N = 3
  int M = 1;                             // elements of p = 3 per tile (2M of p = 2)
  int grid = 0;                          // blocks per tick; 0: one block per tile
  bool have_steps = false;
  std::vector<int64_t> ticks;            // per run: n_steps * S
  int64_t n_ticks = 0;
  int64_t elem_stages = 0;
  std::vector<StageArgs> sargs;
  std::vector<BatchRun> brun;
  std::vector<int32_t> tiles;            // [n_ticks][n_runs + 1]
  BatchRun* d_runs = nullptr;
  StageArgs* d_sargs = nullptr;
  int32_t* d_tiles = nullptr;
  size_t cap_tiles = 0, cap_sargs = 0, cap_runs = 0;
  std::string err;
  ~pe_batch() {
    if (d_runs) (void)hipFree(d_runs);
    if (d_sargs) (void)hipFree(d_sargs);
    if (d_tiles) (void)hipFree(d_tiles);
  }
};

namespace {
thread_local std::string g_batch_err;

pe_status bfail(pe_batch* b, pe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  (b ? b->err : g_batch_err) = buf;
  return st;
}

#define BCHK(call)                                                                         \
  do {                                                                                     \
    hipError_t _e = (call);                                                                \
    if (_e != hipSuccess) return bfail(b, PE_EHIP, "%s: %s", #call, hipGetErrorString(_e)); \
  } while (0)

int elems_per_tile(const pe_batch* b, int N) { return N == 4 ? b->M : 2 * b->M; }

void build_tiles(pe_batch* b) {
  const int nr = (int)b->runs.size();
  b->tiles.assign((size_t)b->n_ticks * (nr + 1), 0);
  b->elem_stages = 0;
  for (int64_t t = 0; t < b->n_ticks; ++t) {
    int32_t* row = &b->tiles[(size_t)t * (nr + 1)];
    int acc = 0;
    for (int q = 0; q < nr; ++q) {
      row[q] = acc;
      const int k = b->order[q];
      const pe_ctx* c = b->runs[k];
      if (t < b->ticks[k]) {
        const int na = c->n_act[(size_t)(t % c->S)];
        const int ept = elems_per_tile(b, c->N);
        acc += (na + ept - 1) / ept;
        b->elem_stages += na;
      }
    }
    row[nr] = acc;
  }
}

template <class T>
pe_status upload(pe_batch* b, T*& dptr, size_t& cap, const std::vector<T>& h) {
  const size_t bytes = h.size() * sizeof(T);
  if (bytes > cap) {
    if (dptr) BCHK(hipFree(dptr));
    dptr = nullptr;
    cap = 0;
    BCHK(hipMalloc((void**)&dptr, bytes));
    cap = bytes;
  }
  if (bytes) BCHK(hipMemcpy(dptr, h.data(), bytes, hipMemcpyHostToDevice));
  return PE_OK;
}
}  // namespace

extern "C" {

pe_status pe_batch_create(pe_batch** out, pe_ctx* const* runs, int n_runs) {
  if (!out) return bfail(nullptr, PE_EINVAL, "batch: null output");
  *out = nullptr;
  if (!runs || n_runs < 1) return bfail(nullptr, PE_EINVAL, "batch: need at least one run");
  for (int k = 0; k < n_runs; ++k) {
    const pe_ctx* c = runs[k];
    if (!c) return bfail(nullptr, PE_EINVAL, "batch: run %d is null", k);
    if (c->dim != 2 || c->equations != 0 || (c->N != 3 && c->N != 4))
      return bfail(nullptr, PE_EUNSUPPORTED, "batch: run %d is not 2D Euler with degree 2 or 3", k);
    if (c->general) return bfail(nullptr, PE_EUNSUPPORTED, "batch: run %d has an alternative stage pattern", k);
    if (c->sc_on) return bfail(nullptr, PE_EUNSUPPORTED, "batch: run %d has shock capturing", k);
    if (!c->partitioned || !c->state_valid || !c->bound)
      return bfail(nullptr, PE_ESTATE, "batch: run %d needs a bound state and a partition", k);
    if (!last_stage_in_place_safe(c))
      return bfail(nullptr, PE_EUNSUPPORTED, "batch: run %d has a member with fewer than 3 evaluations", k);
    for (int j = 0; j < k; ++j)
      if (runs[j] == c) return bfail(nullptr, PE_EINVAL, "batch: run %d appears twice", k);
  }
  pe_batch* b = new (std::nothrow) pe_batch();
  if (!b) return bfail(nullptr, PE_ENOMEM, "batch: out of host memory");
  b->runs.assign(runs, runs + n_runs);
  for (int k = 0; k < n_runs; ++k)
    if (runs[k]->N == 4) b->order.push_back(k);
  b->split = (int)b->order.size();
  for (int k = 0; k < n_runs; ++k)
    if (runs[k]->N == 3) b->order.push_back(k);
  *out = b;
  return PE_OK;
}

void pe_batch_destroy(pe_batch* b) { delete b; }

const char* pe_batch_last_error(const pe_batch* b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

pe_status pe_batch_set_steps(pe_batch* b, const double* dt, const int64_t* n_steps) {
  if (!b) return bfail(nullptr, PE_EINVAL, "batch: null");
  if (!dt || !n_steps) return bfail(b, PE_EINVAL, "batch: null dt or n_steps");
  const int nr = (int)b->runs.size();
  b->sargs.clear();
  b->brun.assign(nr, BatchRun{});
  b->ticks.assign(nr, 0);
  b->n_ticks = 0;
  for (int k = 0; k < nr; ++k)
    if (!(dt[k] > 0.0) || n_steps[k] < 0) return bfail(b, PE_EINVAL, "batch: run %d: dt must be > 0, n_steps >= 0", k);
  for (int q = 0; q < nr; ++q) {
    const int k = b->order[q];
    pe_ctx* c = b->runs[k];
    if (!c->partitioned || !c->state_valid || (int)c->n_act.size() != c->S)
      return bfail(b, PE_ESTATE, "batch: run %d lost its partition or state", k);
    BatchRun& r = b->brun[q];
    r.m = device_mesh(c);
    r.op = c->ops;
    r.ph = c->ph;
    r.N = c->N;
    r.S = c->S;
    r.sarg0 = (int)b->sargs.size();
    for (int i = 0; i < c->S; ++i) {
      StageArgs a;
      fill_stage(c, i, dt[k], a);
      a.U = c->U;
      a.K1 = c->K1;
      set_stage_buffers(c, i, a);
      a.ACC = c->ACC;
      a.Uout = c->U;
      a.evals = c->d_evals;
      b->sargs.push_back(a);
    }
    b->ticks[k] = n_steps[k] * c->S;
    b->n_ticks = std::max(b->n_ticks, b->ticks[k]);
  }
  build_tiles(b);
  pe_status st = upload(b, b->d_runs, b->cap_runs, b->brun);
  if (st == PE_OK) st = upload(b, b->d_sargs, b->cap_sargs, b->sargs);
  if (st == PE_OK) st = upload(b, b->d_tiles, b->cap_tiles, b->tiles);
  if (st != PE_OK) return st;
  b->have_steps = true;
  return PE_OK;
}

pe_status pe_batch_set_tiling(pe_batch* b, int elems_per_tile_p3, int grid_blocks) {
  if (!b) return bfail(nullptr, PE_EINVAL, "batch: null");
  if ((elems_per_tile_p3 != 1 && elems_per_tile_p3 != 2 && elems_per_tile_p3 != 4) || grid_blocks < 0)
    return bfail(b, PE_EINVAL, "batch: tiles of 1, 2 or 4 elements of degree 3, grid >= 0");
  b->M = elems_per_tile_p3;
  b->grid = grid_blocks;
  if (b->have_steps) {
    build_tiles(b);
    return upload(b, b->d_tiles, b->cap_tiles, b->tiles);
  }
  return PE_OK;
}

pe_status pe_batch_info(const pe_batch* b, int64_t* n_ticks, int64_t* element_stages) {
  if (!b) return PE_EINVAL;
  if (n_ticks) *n_ticks = b->n_ticks;
  if (element_stages) *element_stages = b->elem_stages;
  return PE_OK;
}

pe_status pe_batch_run(pe_batch* b, int64_t tick_begin, int64_t tick_end, void* stream) {
  if (!b) return bfail(nullptr, PE_EINVAL, "batch: null");
  if (!b->have_steps) return bfail(b, PE_ESTATE, "batch: set_steps first");
  if (tick_begin < 0 || tick_end > b->n_ticks || tick_begin > tick_end)
    return bfail(b, PE_EINVAL, "batch: ticks [%lld, %lld) outside [0, %lld)", (long long)tick_begin,
                 (long long)tick_end, (long long)b->n_ticks);
  const int nr = (int)b->runs.size();
  hipStream_t s = (hipStream_t)stream;
  for (int64_t t = tick_begin; t < tick_end; ++t) {
    const int32_t* row = &b->tiles[(size_t)t * (nr + 1)];
    const int32_t* drow = b->d_tiles + (size_t)t * (nr + 1);
    // one launch per degree present at this tick: runs [0, split) of degree 3, then degree 2
    const int cls[2][3] = {{4, 0, b->split}, {3, b->split, nr}};
    for (const auto& cl : cls) {
      const int n_tiles = row[cl[2]] - row[cl[1]];
      if (n_tiles <= 0) continue;
      const bool persistent = b->grid > 0 && b->grid < n_tiles;
      const int g = persistent ? b->grid : n_tiles;
      BCHK(launch_stage_batch(cl[0], b->M, g, persistent, b->d_runs, b->d_sargs, drow, cl[1], cl[2], t, s));
    }
  }
  return PE_OK;
}

}  // extern "C"
