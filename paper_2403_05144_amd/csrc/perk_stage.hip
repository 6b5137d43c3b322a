// HIP kernels of libperk for gfx950 (CDNA4).  fp64 on the vector ALUs throughout: flux
// differencing is a pairwise nonlinear function of node states, not a dense contraction, so
// the matrix cores have nothing to do here.
//
// Stage kernel (one launch per P-ERK stage, Sec. 3.1 and eq. PartitionedRKSystem):
//   * one element per group of N^dim lanes (one lane per LGL node), EPB elements per block;
//     an element's conservative state and derived node quantities are staged in LDS;
//   * only the active prefix [0, n_act) of the partition-sorted slots is launched: elements of
//     inactive members cost neither blocks nor lanes (Sec. 6.1);
//   * every element computes the numerical fluxes of its own faces (conforming faces, the
//     fine side of a 2:1 mortar from the interpolated coarse trace, and the coarse side by
//     projecting the fluxes of all sub-faces), so no face buffers and no second launch;
//     both neighbours evaluate a shared face flux from identical inputs in the same order,
//     so the two sides see bitwise identical fluxes and conservation holds to round-off;
//   * traces of neighbours whose member is inactive at this stage are formed on the fly as
//     U_n + dt c_i K_1 (the stage value of a member with a_{i,i-1} = 0);
//   * the epilogue applies the per-member stage combination of the P-ERK tableau
//     (Y_{i+1} = U_n + dt (a_{i+1,1} K_1 + a_{i+1,i} K_i)), the running weighted sum of the
//     stages with b_j != 0, and the final update, so K_i is never stored (low storage, Sec. 3.1).
//
// Memory layout: slot layout [var][slot][node]; lanes of a block read consecutive nodes of
// consecutive elements, so every state access of the own element is one coalesced segment
// per variable.

#include <hip/hip_ext.h>

#include "perk_device.h"

#ifndef STAGE_SPLIT_MAX
#define STAGE_SPLIT_MAX 2048
#endif

namespace perk {
namespace {

// Logarithmic mean (a - b)/(ln a - ln b) from precomputed node logarithms.  With
// f = (a-b)/(a+b), u = f^2 it equals (a+b) / (2 F(u)), F(u) = sum_k u^k/(2k+1); for u < 1e-2
// the series through u^7/15 is used (truncation < 1e-17), so the difference of logarithms is
// only used where |ln a - ln b| > 0.2 and loses little to cancellation.
__device__ __forceinline__ double series_F(double u) {
  return 1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0 + u * (1.0 / 9.0 +
         u * (1.0 / 11.0 + u * (1.0 / 13.0 + u * (1.0 / 15.0)))))));
}

// 1/F(u) as its own power series (coefficients by series inversion of F, exact rationals):
// through u^7 the truncation is below 2e-18 relative for u < 1e-2, and no division is needed.
__device__ __forceinline__ double series_invF(double u) {
  return 1.0 - u * (1.0 / 3.0 + u * (4.0 / 45.0 + u * (44.0 / 945.0 + u * (428.0 / 14175.0 +
         u * (10196.0 / 467775.0 + u * (10719068.0 / 638512875.0 + u * (25865068.0 / 1915538625.0)))))));
}

__device__ __forceinline__ double log_mean(double a, double b, double la, double lb) {
  const double dd = a - b, ss = a + b;
  if (dd * dd < 1e-2 * ss * ss) {
    const double f = dd * rcp(ss);
    return 0.5 * ss * series_invF(f * f);
  }
  return dd * rcp(la - lb);
}

__device__ __forceinline__ double inv_log_mean(double a, double b, double la, double lb) {
  const double dd = a - b, ss = a + b;
  const double iss = rcp(ss);
  if (dd * dd < 1e-2 * ss * ss) {
    const double f = dd * iss;
    return 2.0 * series_F(f * f) * iss;
  }
  return (la - lb) * rcp(dd);
}

// The node pairs (x < y) of one coordinate line in pair order, one nibble per pair.
template <int N>
struct PairNodes {
  static constexpr unsigned pack(bool second) {
    unsigned r = 0;
    int c = 0;
    for (int x = 0; x < N; ++x)
      for (int y = x + 1; y < N; ++y) r |= (unsigned)(second ? y : x) << (4 * c++);
    return r;
  }
  static constexpr unsigned kFirst = pack(false), kSecond = pack(true);
  // pair index of nodes (i, j) of a line, one nibble per (i N + j); the diagonal reads pair 0
  static constexpr unsigned long long index_table() {
    unsigned long long r = 0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const int a = i < j ? i : j, b = i < j ? j : i;
        const unsigned long long pi = i == j ? 0 : (unsigned long long)(a * (2 * N - a - 1) / 2 + (b - a - 1));
        r |= pi << (4 * (i * N + j));
      }
    return r;
  }
  static constexpr unsigned long long kIndexOf = index_table();
};

template <int DIM>
struct NodeQ {
  double rho, v[DIM], p, lrho, beta, lbeta;
};

template <int DIM>
__device__ __forceinline__ void cons_to_prim(const double* u, double gamma, double& rho, double* v, double& p) {
  rho = u[0];
  const double ir = rcp(rho);
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    v[d] = u[1 + d] * ir;
    ke += u[1 + d] * v[d];
  }
  p = (gamma - 1.0) * (u[DIM + 1] - 0.5 * ke);
}

// Entropy-conserving, kinetic-energy-preserving two-point flux (Ranocha), direction d.
template <int DIM>
__device__ __forceinline__ void ec_flux(const NodeQ<DIM>& L, const NodeQ<DIM>& R, int d, double inv_gm1,
                                        double* f) {
  const double rho_ln = log_mean(L.rho, R.rho, L.lrho, R.lrho);
  const double ibeta_ln = inv_log_mean(L.beta, R.beta, L.lbeta, R.lbeta);
  // the direction differs from lane to lane: components along d by selects, not by indexing
  // (an indexed register array goes to scratch memory)
  double vdL = L.v[0], vdR = R.v[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) {
    vdL = k == d ? L.v[k] : vdL;
    vdR = k == d ? R.v[k] : vdR;
  }
  double vd = 0.5 * (vdL + vdR);
  double vv = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) vv += L.v[k] * R.v[k];
  const double fr = rho_ln * vd;
  const double pm = 0.5 * (L.p + R.p);
  f[0] = fr;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double fk = fr * 0.5 * (L.v[k] + R.v[k]);
    f[1 + k] = k == d ? fk + pm : fk;
  }
  f[DIM + 1] = fr * (0.5 * vv + ibeta_ln * inv_gm1) + 0.5 * (L.p * vdR + R.p * vdL);
}

// HLL flux with Davis wave speeds, normal +e_d from L to R; uL, uR conservative.
template <int DIM>
__device__ __forceinline__ void hll_flux(const double* uL, const double* uR, int d, double gamma, double* f) {
  double rl, vl[DIM], pl, rr, vr[DIM], pr;
  cons_to_prim<DIM>(uL, gamma, rl, vl, pl);
  cons_to_prim<DIM>(uR, gamma, rr, vr, pr);
  // normal components by selects (the direction differs from lane to lane)
  double vnl = vl[0], vnr = vr[0], mnl = uL[1], mnr = uR[1];
#pragma unroll
  for (int k = 1; k < DIM; ++k) {
    vnl = k == d ? vl[k] : vnl;
    vnr = k == d ? vr[k] : vnr;
    mnl = k == d ? uL[1 + k] : mnl;
    mnr = k == d ? uR[1 + k] : mnr;
  }
  const double cl = sqrt_pos(gamma * pl * rcp(rl)), cr = sqrt_pos(gamma * pr * rcp(rr));
  const double sl = fmin(vnl - cl, vnr - cr);
  const double sr = fmax(vnl + cl, vnr + cr);
  double fl[DIM + 2], fr[DIM + 2];
  fl[0] = mnl;
  fr[0] = mnr;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double al = uL[1 + k] * vnl, ar = uR[1 + k] * vnr;
    fl[1 + k] = k == d ? al + pl : al;
    fr[1 + k] = k == d ? ar + pr : ar;
  }
  fl[DIM + 1] = (uL[DIM + 1] + pl) * vnl;
  fr[DIM + 1] = (uR[DIM + 1] + pr) * vnr;
  if (sl >= 0.0) {
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) f[v] = fl[v];
  } else if (sr <= 0.0) {
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) f[v] = fr[v];
  } else {
    const double inv = rcp(sr - sl);
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) f[v] = (sr * fl[v] - sl * fr[v] + sl * sr * (uR[v] - uL[v])) * inv;
  }
}

// Stage value of variable v at (slot, node) as seen at this stage (see StageArgs::src).
// (one load from the source buffer the code selects, and K_1 only where it is needed: lanes of
// one wave whose neighbours have different sources share that load instead of one per source)
__device__ __forceinline__ double stage_value(const StageArgs& a, int src, int64_t idx) {
  const double b = (src == 1 ? a.Yin : a.U)[idx];
  return src == 2 ? b + a.dt * a.ci * a.K1[idx] : b;
}

// ------------------------------------------------------------------------------------------
// Stage kernel.  One element per T lanes (T = 64 for 2D p=3, one wave), EPB elements per
// block.  Phases, separated by block barriers:
//   A  connectivity of the element into LDS; own stage value and the epilogue operands
//      (U_n, K_1) loaded into registers, one (variable, node) item per lane;
//   B  neighbour face traces into LDS (conforming: the neighbour's face; fine side of a
//      mortar: the coarse neighbour's whole face; coarse side: every fine neighbour's face);
//   C  node quantities (primitives, logarithms) and, on fine sides, interpolation of the
//      coarse trace to the sub-face;
//   D  one two-point flux per lane: every unordered node pair along a coordinate line gets
//      one entropy-conserving flux (symmetric, used by both nodes), every face node (and
//      every sub-face node of a coarse side) one HLL flux;
//   E  per (variable, node): flux-differencing sum, lifting of the face fluxes (projected
//      with R_m on coarse sides), Jacobian, and the P-ERK stage combination.
// ------------------------------------------------------------------------------------------
template <int DIM, int N, bool SPLIT_ = false>
struct SK {
  using g = G<DIM, N>;
  static constexpr int ND = g::ND, NF = g::NF, NFC = g::NFC, NV = g::NV, NSUB = g::NSUB;
  static constexpr int NPL = N * (N - 1) / 2;                 // pairs per coordinate line
  static constexpr int NLINE = DIM == 2 ? N : N * N;          // lines per direction
  static constexpr int NP = DIM * NLINE * NPL;                // pairs per element
  static constexpr int WORK = NP + NFC * NF;                  // flux items without mortars
  // 2D p=3: two waves per element; the flux phase puts the pair fluxes on the first wave and
  // the face fluxes on the second, so their dependency chains run side by side instead of one
  // after the other in a divergent wave (the face flux chain is the longest of the kernel)
  static constexpr bool SPLIT = SPLIT_ && DIM == 2 && N == 4;
  // 3D p=3: 7 waves, the pair fluxes on the first five (288 of 320 lanes), the face fluxes on
  // the last two, so that no wave runs both flux paths (with 6 waves one wave did)
  static constexpr int T = DIM == 2 ? (N == 4 ? (SPLIT ? 128 : 64) : 32) : (N == 4 ? 448 : 192);
  // lanes of the pair fluxes in phase D when pairs and face nodes have waves of their own
  // (0: one mixed loop over both)
  static constexpr int PLN = SPLIT ? T / 2 : (DIM == 3 && N == 4 ? 320 : 0);
  static constexpr int EPB = T >= 64 ? 1 : 64 / T;
  // elements per block of the single-run kernel: the one-wave 2D p=3 body runs four (their
  // flux phase mapped across the block, see stage_block)
  static constexpr int epb() { return DIM == 2 && N == 4 && !SPLIT ? 4 : EPB; }
  static constexpr int NITEM = (NV * ND + T - 1) / T;         // (variable, node) items per lane
  // waves per SIMD the register allocation must allow.  A second 6-wave block fits on a CU
  // only when every SIMD can hold 4 waves (at most 128 VGPRs) and the LDS allows it (measured:
  // at 3 waves per SIMD a second 384-lane block never starts, whatever its LDS size).
  static constexpr int MINW = T >= 384 ? 4 : 1;
};

// The stage work of one block of EPB elements: block `blk` of the launch covers the slots
// [blk EPB, blk EPB + EPB).  Shared by the single-run kernel and the batched kernel, which
// therefore compute bitwise identical stages.
template <int DIM, int N, bool VISC, int EPB, bool SPLIT = false, bool SC = false>
__device__ __forceinline__ void stage_block(const StageArgs& a, const Mesh& m, const Ops& op, const Physics& ph,
                                            int blk) {
  using K = SK<DIM, N, SPLIT>;
  constexpr int ND = K::ND, NF = K::NF, NFC = K::NFC, NV = K::NV, NSUB = K::NSUB, T = K::T;
  constexpr int NP = K::NP, NPL = K::NPL, NITEM = K::NITEM;
  // 2D stages the own sub-face traces of coarse sides (phase C) and the own viscous flux in LDS.
  // 3D does not: a coarse-side flux lane interpolates its own trace itself, the own viscous flux
  // is read where it is used (an L2 hit), and the projected mortar fluxes overwrite the sub-face
  // fluxes in place.  That keeps a 384-lane 3D block under the LDS size (about 53 KB) at which
  // two blocks share a CU; with the 72 KB of the staged layout only one does.
  constexpr bool LDS_OWN = DIM == 2;
  constexpr int EO = LDS_OWN ? EPB : 1, NSO = LDS_OWN ? NSUB : 1;
  constexpr bool FVL = VISC && LDS_OWN;
  __shared__ double s_u[EPB][NV][ND];
  __shared__ NodeQ<DIM> s_q[EPB][ND];
  __shared__ double s_tr[EPB][NFC][NSUB][NV][NF];   // neighbour traces, later HLL fluxes in place
  __shared__ double s_tro[EO][LDS_OWN ? NFC : 1][NSO][LDS_OWN ? NV : 1][LDS_OWN ? NF : 1];  // coarse sides: own trace on every sub-face
  // 3D Navier-Stokes: the neighbours' viscous traces on sub-faces 1.. of coarse sides are dead
  // once phase C has formed the projected central face values, before phase D writes the pair
  // fluxes: the two share storage (1440 doubles each at p=3), which brings the block from 50 KB
  // of LDS to 38 KB, so that four blocks fit a CU instead of three
  constexpr bool ALIAS = VISC && !LDS_OWN;
  // 2D split Euler body with shock capturing: the face lanes compute their fluxes in phase C,
  // beside the node quantities and the blending factor, into s_tro, and project the coarse sides
  // in phase D, beside the pair fluxes, into s_tr (one barrier fewer; the face chain no longer
  // waits for the node quantities).  Measured per body: 7.4 -> 6.7 us per launch of the
  // Kelvin-Helmholtz run with shock capturing (~450 elements); without shock capturing the
  // same order was 1.5 % (KH, ~1400 elements) and 6 % (two-level vortex) slower, so the plain
  // bodies keep the original order.
  constexpr bool EARLYF = SPLIT && !VISC && SC;
  // four one-wave 2D p=3 elements per block (large launches and batch tiles, throughput-bound
  // on the VALU): the node quantities of all four on the first wave, and in the flux phase the
  // 4 x 48 pair fluxes on the first three waves and the 4 x 16 face fluxes on the fourth, so
  // that no wave issues both flux paths (one wave per element ran pairs and faces one after
  // the other, divergent, in every element).  With shock capturing the blending factors of
  // the four come from the second wave and their subcell fluxes (HLL, like the face fluxes)
  // from the fourth.
  constexpr bool XM = DIM == 2 && N == 4 && T == 64 && EPB == 4 && !SPLIT;
  constexpr int NPF = NP * NV, NTV1 = NFC * (NSUB - 1) * NV * NF;
  constexpr int NX = ALIAS && NTV1 > NPF ? NTV1 : NPF;
  __shared__ double s_pf[EPB][NX];   // pair flux w, variable v at [w NV + v]
  auto tv1 = [](int f, int sub, int v, int j) { return ((f * (NSUB - 1) + sub - 1) * NV + v) * NF + j; };
  __shared__ int s_fk[EPB][NFC];
  __shared__ int s_fn[EPB][NFC][4];
  // BR1: own viscous flux at every node (2D) and the neighbours' viscous face traces
  __shared__ double s_fv[FVL ? EPB : 1][FVL ? DIM : 1][FVL ? NV : 1][FVL ? ND : 1];
  __shared__ double s_trv[VISC ? EPB : 1][VISC ? NFC : 1][VISC && !ALIAS ? NSUB : 1][VISC ? NV : 1][VISC ? NF : 1];
  // the derivative matrix: the epilogue reads row `pos` of the lane's node, which from kernel
  // argument memory would be a gather with a memory round after the last barrier.  s_D2 holds
  // 2 D with a zero diagonal (the flux-differencing weights, no pair (i, i)), s_D plain D (BR1)
  __shared__ double s_D2[N * N];
  __shared__ double s_D[VISC ? N * N : 1];
  // 3D: the mortar operators P_0, P_1, R_0, R_1 too (coarse/fine faces are common in 3D
  // refinement zones, and their lane-indexed reads from kernel-argument memory are slow); all
  // six tables come in on the block's last wave in phase A.  2D reads P and R from the kernel
  // arguments (only mortar blocks do, and they are not the slowest blocks of a launch).
  // Epilogue operands U_n, K_1 and the weighted stage sum: loaded in phase A and held (the split
  // 2D block: its launches are latency-bound, no memory round after the last barrier), or read
  // where they are used (L2 hits that other resident blocks hide), which keeps them out of
  // registers across the flux phases.  Measured per body: the one-wave 2D body and the batched
  // kernels lose their spills at 96-99 VGPRs (batch ticks 6 % shorter); 3D Navier-Stokes loses a
  // 20-byte spill at equal time; 3D Euler holds them (a 20-byte spill, 2-4 % faster than without).
  constexpr bool HOLD_OPS = SPLIT || (DIM == 3 && !VISC);
  constexpr bool OPS_A = DIM == 3;
  __shared__ double s_PR[OPS_A ? 4 : 1][OPS_A ? N * N : 1];
  // subcell shock capturing (2D Euler): the modal transform, the element's blending factor and
  // the first-order fluxes between neighbouring nodes of every coordinate line (subcell faces)
  static_assert(!SC || (DIM == 2 && !VISC && K::T >= 32 && K::ND <= 16), "shock capturing: 2D Euler bodies");
  constexpr int NFVI = SC ? DIM * K::NLINE * (N - 1) : 1;
  __shared__ double s_fvs[SC ? EPB : 1][NFVI][NV];
  __shared__ double s_vinv[SC ? N * N : 1];
  __shared__ double s_alpha[SC ? EPB : 1];
  auto Pm = [&](int mm, int idx) -> double { return OPS_A ? s_PR[mm][idx] : op.P[mm][idx]; };
  auto Rm = [&](int mm, int idx) -> double { return OPS_A ? s_PR[2 + mm][idx] : op.R[mm][idx]; };

  // one element per block: the element index is the same on every lane (scalar registers)
  const int le = EPB == 1 ? 0 : (int)threadIdx.x / T;
  const int lane = threadIdx.x - le * T;
  const int v_act = blk * EPB + le;                 // index among the launch's active elements
  const bool act = v_act < a.n_act;
  const int e = act ? active_slot(a, v_act) : v_act;
  const int ld = m.ld;
  const double gamma = ph.gamma;
  const double inv_gm1 = 1.0 / (gamma - 1.0);
  // own viscous flux, direction d, variable v, node nd
  // (the device array is addressed through the block's own slot e: only the 3D bodies read
  // it, whose flux phase works on the lane's own element, q == le)
  auto fv_own_q = [&](int q, int d, int v, int nd) -> double {
    if (FVL) return s_fv[q][d][v][nd];
    return a.Fv[(((int64_t)d * NV + v) * ld + e) * ND + nd];
  };
  auto fv_own = [&](int d, int v, int nd) -> double { return fv_own_q(le, d, v, nd); };
  static_assert(!XM || !VISC || FVL, "cross-element flux mapping reads the viscous flux from LDS");

  // ---- A+B: connectivity, own values and epilogue operands, neighbour traces, all in flight
  //      together; one barrier before the node quantities
  constexpr int NTRI = NSUB * NFC * NV * NF;             // trace items of the element
  constexpr int NTR = (NTRI + T - 1) / T;                // per lane
  constexpr int TB = T * EPB, L0 = TB > 64 ? TB - 64 : 0;   // the block's last wave: [L0, TB)
  constexpr int NTAB = 6 * N * N, NTL = (NTAB + (TB - L0) - 1) / (TB - L0);
  double tab[OPS_A ? NTL : 1];
  if (OPS_A) {
#pragma unroll
    for (int k = 0; k < NTL; ++k) {
      const int t = (int)threadIdx.x - L0 + k * (TB - L0);
      tab[k] = op.dD[t >= 0 && t < NTAB ? t : 0];
    }
  }
  int my_mem = 0, my_src = 0;
  double J[DIM];
  double un[NITEM], k1[NITEM], acc[NITEM];
  if (act) {
    my_mem = member_of_slot(m, e);
    // one element per block: the member is the same on every lane, so the epilogue's per-member
    // argument reads (coefficients, output buffer) are scalar loads, not per-lane indexed ones
    if (EPB == 1) my_mem = __builtin_amdgcn_readfirstlane(my_mem);
    my_src = src_of(a, my_mem);   // (a shift of one argument word, not an indexed argument load)
    int tr_nb[NTR], tr_pk[NTR];
#pragma unroll
    for (int it = 0; it < NTR; ++it) {
      const int w = lane + it * T;
      tr_pk[it] = -1;
      if (w < NTRI) {
        const int f = (w / (NF * NV)) % NFC;
        const int sub = w / (NF * NV * NFC);
        tr_pk[it] = m.fk[(int64_t)e * NFC + f];
        tr_nb[it] = m.fn[((int64_t)e * NFC + f) * 4 + sub];
      }
    }
    const int lev = m.lev[e];
    if (lane < NFC) s_fk[le][lane] = m.fk[(int64_t)e * NFC + lane];
    if (lane < NFC * 4) s_fn[le][lane / 4][lane % 4] = m.fn[(int64_t)e * NFC * 4 + lane];
    double own[NITEM];
#pragma unroll
    for (int it = 0; it < NITEM; ++it) {
      const int w = lane + it * T;
      if (w < NV * ND) {
        const int v = w / ND, nd = w - v * ND;
        const int64_t idx = ((int64_t)v * ld + e) * ND + nd;
        un[it] = a.U[idx];
        // K_1 exists only after the first stage of a step; right-hand-side launches never read it
        if (HOLD_OPS) {
          k1[it] = (a.first || a.Kout) ? 0.0 : a.K1[idx];
          acc[it] = a.read_acc ? a.ACC[idx] : 0.0;
        } else {
          k1[it] = (my_src == 2 && !a.first && !a.Kout) ? a.K1[idx] : 0.0;
        }
        own[it] = my_src == 0 ? un[it] : (my_src == 1 ? a.Yin[idx] : un[it] + a.dt * a.ci * k1[it]);
      }
    }
#pragma unroll
    for (int it = 0; it < NTR; ++it) {
      const int w = lane + it * T;
      if (w >= NTRI) continue;
      const int j = w % NF;
      const int v = (w / NF) % NV;
      const int f = (w / (NF * NV)) % NFC;
      const int sub = w / (NF * NV * NFC);
      if (sub > 0 && face_kind(tr_pk[it]) != kCoarseSide) continue;
      const int nb = tr_nb[it];
      const int d = f >> 1, side = f & 1;
      const int src = src_of(a, member_of_slot(m, nb));
      const int nn = face_node<DIM, N>(d, 1 - side, j);
      s_tr[le][f][sub][v][j] = stage_value(a, src, ((int64_t)v * ld + nb) * ND + nn);
      if (VISC) {
        const double fvn = a.Fv[(((int64_t)d * NV + v) * ld + nb) * ND + nn];
        if (ALIAS && sub > 0) s_pf[le][tv1(f, sub, v, j)] = fvn;
        else s_trv[le][f][ALIAS ? 0 : sub][v][j] = fvn;
      }
    }
    if (FVL) {
      for (int w = lane; w < DIM * NV * ND; w += T) {
        const int nd = w % ND, v = (w / ND) % NV, d = w / (ND * NV);
        s_fv[le][d][v][nd] = a.Fv[(((int64_t)d * NV + v) * ld + e) * ND + nd];
      }
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) J[d] = m.jac[lev][d];
#pragma unroll
    for (int it = 0; it < NITEM; ++it) {
      const int w = lane + it * T;
      if (w < NV * ND) s_u[le][w / ND][w % ND] = own[it];
    }
    if (lane == 0 && a.evals) atomicAdd(&a.evals[e], 1);
  }
  if (OPS_A) {
#pragma unroll
    for (int k = 0; k < NTL; ++k) {
      const int t = (int)threadIdx.x - L0 + k * (TB - L0);
      if (t < 0 || t >= NTAB) continue;
      const int tb = t / (N * N), ti = t % (N * N);
      if (tb == 0) s_D2[ti] = tab[k];
      else if (tb == 1) { if (VISC) s_D[ti] = tab[k]; }
      else s_PR[tb - 2][ti] = tab[k];
    }
  }
  if (SC && threadIdx.x < N * N) s_vinv[threadIdx.x] = op.dD[6 * N * N + threadIdx.x];
  __syncthreads();

  // ---- C: node quantities; fine sides: coarse trace interpolated into sub-slot 1
  // The derivative tables for the epilogue come in on the block's last lanes: in split and 3D
  // blocks a wave with little to do here, so that the load stays off the node-quantity wave.
  if (!OPS_A) {
    const int t = (int)threadIdx.x - (T * EPB - 2 * N * N);
    if (t >= 0) {
      const double dv = op.dD[t];
      if (t < N * N) s_D2[t] = dv;
      else if (VISC) s_D[t - N * N] = dv;
    }
  }
  constexpr int NCV = ALIAS ? (NFC * NV * NF + T - 1) / T : 1;
  double cv_hold[NCV];
  if (act) {
    // Node quantities.  When the element's nodes fill whole waves and the block has waves to
    // spare (3D p=3: 64 nodes, 7 waves), the two logarithms of a node go to two waves: the first
    // forms the primitives and ln rho, the second beta = rho/p and ln beta, side by side.
    constexpr bool SPLITQ = ND % 64 == 0 && T >= 2 * ND;
    if (SPLITQ) {
      const int w = lane < ND ? lane : lane - ND;
      if (lane < 2 * ND) {
        double uu[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) uu[v] = s_u[le][v][w];
        double rho, vel[DIM], p;
        cons_to_prim<DIM>(uu, gamma, rho, vel, p);
        if (lane < ND) {
          s_q[le][w].rho = rho;
#pragma unroll
          for (int d = 0; d < DIM; ++d) s_q[le][w].v[d] = vel[d];
          s_q[le][w].p = p;
          s_q[le][w].lrho = log_pos(rho);
        } else {
          const double beta = rho * rcp(p);
          s_q[le][w].beta = beta;
          s_q[le][w].lbeta = log_pos(beta);
        }
      }
    } else {
      // XM: the block's first wave forms the nodes of all four elements, node w of element qe
      // on lane qe ND + w (it gets here whenever any element of the block is active: the
      // active elements of a block come first)
      const int qe = XM ? (int)threadIdx.x / ND : le;
      const int w0 = XM ? (int)threadIdx.x - qe * ND : lane;
      const bool qact = XM ? (qe < EPB && blk * EPB + qe < a.n_act) : true;
      for (int w = w0; qact && w < ND; w += XM ? ND : T) {
        double uu[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) uu[v] = s_u[qe][v][w];
        NodeQ<DIM> q;
        cons_to_prim<DIM>(uu, gamma, q.rho, q.v, q.p);
        q.lrho = log_pos(q.rho);
        q.beta = q.rho * rcp(q.p);
        q.lbeta = log_pos(q.beta);
        s_q[qe][w] = q;
      }
    }
    // (interpolations start on the wave after the node quantities)
    const int lane_c = (lane + (SPLITQ ? 2 * ND : 64)) % T;
    for (int w = lane_c; !EARLYF && w < NFC * NV * NF; w += T) {
      const int j = w % NF;
      const int v = (w / NF) % NV;
      const int f = w / (NF * NV);
      const int32_t pk = s_fk[le][f];
      if (face_kind(pk) != kFineSide) continue;
      const int s0 = face_sub0(pk), s1 = face_sub1(pk);
      double val = 0.0;
      if (DIM == 2) {
#pragma unroll
        for (int k = 0; k < N; ++k) val += Pm(s0, j * N + k) * s_tr[le][f][0][v][k];
      } else {
        const int ja = j % N, jb = j / N;
#pragma unroll
        for (int kb = 0; kb < N; ++kb) {
          double row = 0.0;
#pragma unroll
          for (int ka = 0; ka < N; ++ka) row += Pm(s0, ja * N + ka) * s_tr[le][f][0][v][ka + N * kb];
          val += Pm(s1, jb * N + kb) * row;
        }
      }
      s_tr[le][f][1][v][j] = val;
      if (VISC && !ALIAS) {
        double vv = 0.0;
        if (DIM == 2) {
#pragma unroll
          for (int k = 0; k < N; ++k) vv += Pm(s0, j * N + k) * s_trv[le][f][0][v][k];
        } else {
          const int ja = j % N, jb = j / N;
#pragma unroll
          for (int kb = 0; kb < N; ++kb) {
            double row = 0.0;
#pragma unroll
            for (int ka = 0; ka < N; ++ka) row += Pm(s0, ja * N + ka) * s_trv[le][f][0][v][ka + N * kb];
            vv += Pm(s1, jb * N + kb) * row;
          }
        }
        s_trv[le][f][1][v][j] = vv;
      }
    }
    // coarse sides: own trace interpolated to every sub-face (2D: one item per lane here
    // instead of a whole interpolation per flux lane in phase D) and, for BR1, the central
    // average of the interpolated own viscous flux with the fine neighbour's
    for (int w = lane_c; !EARLYF && (LDS_OWN || (VISC && !ALIAS)) && w < NFC * NSUB * NV * NF; w += T) {
      const int j = w % NF;
      const int v = (w / NF) % NV;
      const int sub = (w / (NF * NV)) % NSUB;
      const int f = w / (NF * NV * NSUB);
      if (face_kind(s_fk[le][f]) != kCoarseSide) continue;
      const int d = f >> 1, side = f & 1;
      const int m0 = sub & 1, m1 = (sub >> 1) & 1;
      double x = 0.0, xv = 0.0;
      if (DIM == 2) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double c = Pm(m0, j * N + k);
          const int on = face_node<DIM, N>(d, side, k);
          if (LDS_OWN) x += c * s_u[le][v][on];
          if (VISC) xv += c * fv_own(d, v, on);
        }
      } else {
        const int ja = j % N, jb = j / N;
#pragma unroll
        for (int kb = 0; kb < N; ++kb) {
          double row = 0.0, rowv = 0.0;
#pragma unroll
          for (int ka = 0; ka < N; ++ka) {
            const double c = Pm(m0, ja * N + ka);
            const int on = face_node<DIM, N>(d, side, ka + N * kb);
            if (LDS_OWN) row += c * s_u[le][v][on];
            if (VISC) rowv += c * fv_own(d, v, on);
          }
          const double cb = Pm(m1, jb * N + kb);
          x += cb * row;
          if (VISC) xv += cb * rowv;
        }
      }
      if (LDS_OWN) s_tro[le][f][sub][v][j] = x;
      if (VISC) s_trv[le][f][sub][v][j] = 0.5 * (xv + s_trv[le][f][sub][v][j]);
    }
    if constexpr (ALIAS) {
      // BR1 central viscous values on the element's own face nodes: conforming faces
      // (own + neighbour)/2, fine sides with the coarse trace interpolated, coarse sides
      // sum_m R_m (P_m own + nb_m)/2 = (own + sum_m R_m nb_m)/2 (sum_m R_m P_m = I)
#pragma unroll
      for (int q = 0; q < NCV; ++q) {
        const int w = lane_c + q * T;
        cv_hold[q] = 0.0;
        if (w >= NFC * NV * NF) continue;
        const int j = w % NF, v = (w / NF) % NV, f = w / (NF * NV);
        const int32_t pk = s_fk[le][f];
        const int kind = face_kind(pk);
        const int d = f >> 1, side = f & 1;
        const int ja = j % N, jb = j / N;
        double nbv = 0.0;
        if (kind == kConforming) {
          nbv = s_trv[le][f][0][v][j];
        } else if (kind == kFineSide) {
          const int s0 = face_sub0(pk), s1 = face_sub1(pk);
#pragma unroll
          for (int kb = 0; kb < N; ++kb) {
            double row = 0.0;
#pragma unroll
            for (int ka = 0; ka < N; ++ka) row += Pm(s0, ja * N + ka) * s_trv[le][f][0][v][ka + N * kb];
            nbv += Pm(s1, jb * N + kb) * row;
          }
        } else {
#pragma unroll 1
          for (int ms = 0; ms < NSUB; ++ms) {
            const int m0 = ms & 1, m1 = (ms >> 1) & 1;
#pragma unroll
            for (int kb = 0; kb < N; ++kb) {
              double row = 0.0;
#pragma unroll
              for (int ka = 0; ka < N; ++ka) {
                const int k = ka + N * kb;
                row += Rm(m0, ja * N + ka) * (ms == 0 ? s_trv[le][f][0][v][k] : s_pf[le][tv1(f, ms, v, k)]);
              }
              nbv += Rm(m1, jb * N + kb) * row;
            }
          }
        }
        cv_hold[q] = 0.5 * (fv_own(d, v, face_node<DIM, N>(d, side, j)) + nbv);
      }
    }
    if constexpr (EARLYF) {
      // face fluxes on the face lanes [PLN, PLN + NSUB NFC NF): the neighbour's trace from s_tr
      // (fine sides: the coarse trace interpolated here), the own one from s_u (coarse sides:
      // interpolated to the sub-face here); the flux goes to s_tro, so that no lane overwrites a
      // trace another lane still reads
      constexpr int NFI = NSUB * NFC * NF;
      const int r = lane - K::PLN;
      if (r >= 0 && r < NFI) {
        const int j = r % NF, f = (r / NF) % NFC, sub = r / (NF * NFC);
        const int32_t pk = s_fk[le][f];
        const int kind = face_kind(pk);
        if (sub == 0 || kind == kCoarseSide) {
          const int d = f >> 1, side = f & 1;
          double mine[NV], oth[NV], fl[NV];
          if (kind == kCoarseSide) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              double x = 0.0;
#pragma unroll
              for (int k = 0; k < N; ++k) x += Pm(sub, j * N + k) * s_u[le][v][face_node<DIM, N>(d, side, k)];
              mine[v] = x;
              oth[v] = s_tr[le][f][sub][v][j];
            }
          } else {
            const int on = face_node<DIM, N>(d, side, j);
            const int s0 = face_sub0(pk);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              mine[v] = s_u[le][v][on];
              double x = s_tr[le][f][0][v][j];
              if (kind == kFineSide) {
                x = 0.0;
#pragma unroll
                for (int k = 0; k < N; ++k) x += Pm(s0, j * N + k) * s_tr[le][f][0][v][k];
              }
              oth[v] = x;
            }
          }
          double uL[NV], uR[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            uL[v] = side == 1 ? mine[v] : oth[v];
            uR[v] = side == 1 ? oth[v] : mine[v];
          }
          hll_flux<DIM>(uL, uR, d, gamma, fl);
#pragma unroll
          for (int v = 0; v < NV; ++v) s_tro[le][f][sub][v][j] = fl[v];
        }
      }
    }
  }
  if constexpr (SC) {
    // blending factor of subcell shock capturing: the density's coefficients in the
    // orthonormal Legendre basis, one per lane of a 16-lane group (lanes [16, 32) of the
    // element's wave, idle in this phase; XM: the second wave, a group per element), the
    // energies of all modes, of those of degree <= p - 1 and <= p - 2 in each direction summed
    // over the group, E = max((all - clip_1)/all, (clip_1 - clip_2)/clip_1), and the sigmoid
    const int tq = XM ? (int)threadIdx.x - T : lane - 16;
    const int qa = XM ? (tq >= 0 ? tq / 16 : EPB) : le;
    const bool on = XM ? (tq >= 0 && qa < EPB && blk * EPB + qa < a.n_act) : (act && lane >= 16 && lane < 32);
    if (on) {
      const int t = XM ? tq - qa * 16 : tq;
      double tot = 0.0, c1 = 0.0, c2 = 0.0;
      if (t < ND) {
        const int ia = t % N, ib = t / N;
        double mo = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          double row = 0.0;
#pragma unroll
          for (int i = 0; i < N; ++i) row += s_vinv[ia * N + i] * s_u[qa][0][i + N * j];
          mo += s_vinv[ib * N + j] * row;
        }
        const int deg = ia > ib ? ia : ib;
        tot = mo * mo;
        c1 = deg <= N - 2 ? tot : 0.0;
        c2 = deg <= N - 3 ? tot : 0.0;
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o, 16);
        c1 += __shfl_xor(c1, o, 16);
        c2 += __shfl_xor(c2, o, 16);
      }
      if (t == 0) {
        const double e1 = tot > 0.0 ? (tot - c1) / tot : 0.0;
        const double e2 = c1 > 0.0 ? (c1 - c2) / c1 : 0.0;
        const double E = e1 < e2 ? e2 : e1;
        const double al = 1.0 / (1.0 + exp(-a.sc_slope * (E - a.sc_T)));
        s_alpha[qa] = al < a.sc_amin ? 0.0 : (al < a.sc_amax ? al : a.sc_amax);
      }
    }
  }
  __syncthreads();

  // ---- D: fluxes.  Pairs first, then face nodes sub-face-major (sub 0 of every face first).
  double alpha = 0.0;
  if (SC && act) alpha = s_alpha[le];
  // (XM: a lane's flux item may belong to another element of the block; activity per item)
  if (act || XM) {
    if constexpr (ALIAS) {
      // the central viscous face values of phase C (the sub-face traces they replace are dead:
      // their storage takes the pair fluxes now)
      const int lane_c = (lane + (ND % 64 == 0 && T >= 2 * ND ? 2 * ND : 64)) % T;
#pragma unroll
      for (int q = 0; q < NCV; ++q) {
        const int w = lane_c + q * T;
        if (w < NFC * NV * NF) s_trv[le][w / (NF * NV)][0][(w / NF) % NV][w % NF] = cv_hold[q];
      }
    }
    // pair fluxes (w in [0, NP)) and face fluxes (r in [0, NFI)); with the split on, each on
    // lanes of its own ([0, PLN) and [PLN, T)), else one loop over both
    constexpr int NFI = NSUB * NFC * NF;
    // pair flux w and face flux r of element q of the block
    auto pair_flux = [&](int q, int w) {
      const int pl = w % NPL;
      const int line = (w / NPL) % K::NLINE;
      const int d = w / (NPL * K::NLINE);
      const int pa = (PairNodes<N>::kFirst >> (4 * pl)) & 15, pb = (PairNodes<N>::kSecond >> (4 * pl)) & 15;
      double f[NV];
      ec_flux<DIM>(s_q[q][node_on_line<DIM, N>(d, line, pa)], s_q[q][node_on_line<DIM, N>(d, line, pb)], d,
                   inv_gm1, f);
#pragma unroll
      for (int v = 0; v < NV; ++v) s_pf[q][w * NV + v] = f[v];
    };
    auto face_flux = [&](int q, int r) {
      const int j = r % NF;
      const int f = (r / NF) % NFC;
      const int sub = r / (NF * NFC);
      const int32_t pk = s_fk[q][f];
      const int kind = face_kind(pk);
      if (sub > 0 && kind != kCoarseSide) return;
      const int d = f >> 1, side = f & 1;
      double mine[NV], oth[NV], fl[NV];
      if (kind == kCoarseSide && LDS_OWN) {
        // own trace interpolated to sub-face `sub` (phase C)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          mine[v] = s_tro[q][f][sub][v][j];
          oth[v] = s_tr[q][f][sub][v][j];
        }
      } else if (kind == kCoarseSide) {
        // own trace interpolated to sub-face `sub` here: P_{m1} (x) P_{m0} on the face, one
        // variable at a time (five accumulators at once would spill at 128 VGPRs)
        const int m0 = sub & 1, m1 = (sub >> 1) & 1;
        const int ja = j % N, jb = j / N;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          oth[v] = s_tr[q][f][sub][v][j];
          double x = 0.0;
#pragma unroll 1
          for (int kb = 0; kb < N; ++kb) {
            double row = 0.0;
#pragma unroll
            for (int ka = 0; ka < N; ++ka)
              row += Pm(m0, ja * N + ka) * s_u[q][v][face_node<DIM, N>(d, side, ka + N * kb)];
            x += Pm(m1, jb * N + kb) * row;
          }
          mine[v] = x;
        }
      } else {
        const int on = face_node<DIM, N>(d, side, j);
        const int ts = kind == kFineSide ? 1 : 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          mine[v] = s_u[q][v][on];
          oth[v] = s_tr[q][f][ts][v][j];
        }
      }
      // one flux call with the states ordered along +e_d (two calls, one per side, would run
      // both inlined copies in every wave whose lanes see both sides)
      double uL[NV], uR[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        uL[v] = side == 1 ? mine[v] : oth[v];
        uR[v] = side == 1 ? oth[v] : mine[v];
      }
      hll_flux<DIM>(uL, uR, d, gamma, fl);
#pragma unroll
      for (int v = 0; v < NV; ++v) s_tr[q][f][sub][v][j] = fl[v];
      if (VISC && !ALIAS && kind != kCoarseSide) {
        // BR1 central viscous flux on this face node: 1/2 (own + neighbour); coarse sides
        // were averaged in phase C
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double ownv = fv_own_q(q, d, v, face_node<DIM, N>(d, side, j));
          const int ts = kind == kFineSide ? 1 : 0;
          s_trv[q][f][sub][v][j] = 0.5 * (ownv + s_trv[q][f][ts][v][j]);
        }
      }
    };
    if (EARLYF) {
      if (lane < K::PLN) {
        for (int w = lane; w < NP; w += K::PLN) pair_flux(le, w);
      } else {
        // coarse sides: the sub-face fluxes projected back with R_m into s_tr (sub-face 0)
        for (int w = lane - K::PLN; w < NFC * NV * NF; w += T - K::PLN) {
          const int i = w % NF, v = (w / NF) % NV, f = w / (NF * NV);
          if (face_kind(s_fk[le][f]) != kCoarseSide) continue;
          double fs = 0.0;
#pragma unroll
          for (int ms = 0; ms < 2; ++ms)
#pragma unroll
            for (int kk = 0; kk < N; ++kk) fs += Rm(ms, i * N + kk) * s_tro[le][f][ms][v][kk];
          s_tr[le][f][0][v][i] = fs;
        }
      }
    } else if constexpr (XM) {
      // pairs of element t / NP on lanes [0, EPB NP), sub-face-0 face items of element
      // (t - EPB NP) / NF0 on the rest; the items of other sub-faces (coarse sides only) after
      constexpr int NF0 = NFC * NF, NFX = NFI - NF0;
      static_assert(EPB * (NP + NF0) == T * EPB, "cross-element flux mapping fills the block");
      const int t = threadIdx.x;
      if (t < EPB * NP) {
        const int q = t / NP;
        if (blk * EPB + q < a.n_act) pair_flux(q, t - q * NP);
      } else {
        const int r = t - EPB * NP, q = r / NF0;
        if (blk * EPB + q < a.n_act) face_flux(q, r - q * NF0);
      }
      for (int x = t; x < EPB * NFX; x += T * EPB) {
        const int q = x / NFX;
        if (blk * EPB + q < a.n_act) face_flux(q, NF0 + x - q * NFX);
      }
    } else if (K::PLN) {
      constexpr int NFL = T - K::PLN;   // face lanes
      if (lane < K::PLN) {
        for (int w = lane; w < NP; w += K::PLN) pair_flux(le, w);
      } else if (lane - K::PLN < NFI) {
        face_flux(le, lane - K::PLN);
      }
      // face items beyond the face lanes exist only on the sub-faces of coarse sides; every lane
      // takes part (on other blocks each returns at once)
      for (int r = NFL + lane; r < NFI; r += T) face_flux(le, r);
    } else {
      for (int w = lane; w < NP + NFI; w += T) {
        if (w < NP) pair_flux(le, w);
        else face_flux(le, w - NP);
      }
    }
    if constexpr (SC) {
      // HLL fluxes between neighbouring nodes of every coordinate line (subcell faces) of
      // elements with alpha > 0: on the lanes with the fewest flux items above (split body:
      // after the face lanes; one element per wave: after the last item; XM: the face wave,
      // after the face fluxes, whose code path they share)
      auto subcell_flux = [&](int q, int w) {
        const int k = w % (N - 1), line = (w / (N - 1)) % K::NLINE, d = w / ((N - 1) * K::NLINE);
        const int nl = node_on_line<DIM, N>(d, line, k), nr = node_on_line<DIM, N>(d, line, k + 1);
        double uL[NV], uR[NV], fl[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          uL[v] = s_u[q][v][nl];
          uR[v] = s_u[q][v][nr];
        }
        hll_flux<DIM>(uL, uR, d, gamma, fl);
#pragma unroll
        for (int v = 0; v < NV; ++v) s_fvs[q][w][v] = fl[v];
      };
      if constexpr (XM) {
        constexpr int NFW = NFC * NF * EPB;   // lanes of the face wave
        for (int x = (int)threadIdx.x - EPB * NP; x >= 0 && x < EPB * NFVI; x += NFW) {
          const int q = x / NFVI;
          if (blk * EPB + q < a.n_act && s_alpha[q] > 0.0) subcell_flux(q, x - q * NFVI);
        }
      } else if (alpha > 0.0) {
        constexpr int FVB = K::PLN ? K::PLN + NFI : (NP + NFI) % T;
        for (int w = (lane + T - FVB) % T; w < NFVI; w += T) subcell_flux(le, w);
      }
    }
  }
  __syncthreads();

  // ---- E0: coarse sides: sub-face fluxes projected back to the coarse face nodes with R_m.
  //      2D: inviscid into s_tro[..][0], viscous into s_tro[..][1] (the own sub-face traces
  //      there are no longer needed).  3D: held in registers over a barrier, then written over
  //      sub-face 0 of s_tr (inviscid) and s_trv (viscous).
  constexpr int NE0 = (NFC * NV * NF + T - 1) / T;
  double e0_fs[NE0], e0_fsv[NE0];
  bool e0_has[NE0];
#pragma unroll
  for (int k = 0; k < NE0; ++k) {
    e0_has[k] = false;
    e0_fs[k] = e0_fsv[k] = 0.0;
    const int w = lane + k * T;
    if (EARLYF || !act || w >= NFC * NV * NF) continue;
    const int i = w % NF;
    const int v = (w / NF) % NV;
    const int f = w / (NF * NV);
    if (face_kind(s_fk[le][f]) != kCoarseSide) continue;
    double fs = 0.0, fsv = 0.0;
    if (DIM == 2) {
#pragma unroll
      for (int ms = 0; ms < 2; ++ms)
#pragma unroll
        for (int kk = 0; kk < N; ++kk) {
          const double r = Rm(ms, i * N + kk);
          fs += r * s_tr[le][f][ms][v][kk];
          if (VISC) fsv += r * s_trv[le][f][ms][v][kk];
        }
    } else {
      const int ia = i % N, ib = i / N;
#pragma unroll
      for (int ms = 0; ms < 4; ++ms) {
        const int m0 = ms & 1, m1 = (ms >> 1) & 1;
#pragma unroll
        for (int kb = 0; kb < N; ++kb) {
          double row = 0.0, rowv = 0.0;
#pragma unroll
          for (int ka = 0; ka < N; ++ka) {
            const double r = Rm(m0, ia * N + ka);
            row += r * s_tr[le][f][ms][v][ka + N * kb];
            if (VISC && !ALIAS) rowv += r * s_trv[le][f][ms][v][ka + N * kb];
          }
          const double rb = Rm(m1, ib * N + kb);
          fs += rb * row;
          if (VISC && !ALIAS) fsv += rb * rowv;
        }
      }
    }
    if (LDS_OWN) {
      s_tro[le][f][0][v][i] = fs;
      if (VISC) s_tro[le][f][LDS_OWN ? 1 : 0][v][i] = fsv;
    } else {
      e0_has[k] = true;
      e0_fs[k] = fs;
      e0_fsv[k] = fsv;
    }
  }
  if (!LDS_OWN) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NE0; ++k) {
      if (!e0_has[k]) continue;
      const int w = lane + k * T;
      const int i = w % NF, v = (w / NF) % NV, f = w / (NF * NV);
      s_tr[le][f][0][v][i] = e0_fs[k];
      if (VISC && !ALIAS) s_trv[le][f][0][v][i] = e0_fsv[k];
    }
  }
  if (!EARLYF) __syncthreads();
  if (!act) return;

  // ---- E: sums, lifting, Jacobian, stage combination
  const double iw0 = op.iw[0], iwN = op.iw[N - 1], iw1 = op.iw[1];
#pragma unroll
  for (int it = 0; it < NITEM; ++it) {
    const int w = lane + it * T;
    if (w >= NV * ND) continue;
    const int v = w / ND, nd = w - v * ND;
    double du = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int line, pos;
      line_of<DIM, N>(nd, d, line, pos);
      const int base = (d * K::NLINE + line) * NPL;
      // branch-free: every lane reads an operand for every term and weighs the terms that do
      // not apply by zero (the pair (pos, pos) reads pair 0 of the line; interior nodes read
      // the flux of face 2d), so that the reads issue together instead of one branch at a time
      double acc = 0.0;
#pragma unroll
      for (int mm = 0; mm < N; ++mm) {
        const int pi = (int)((PairNodes<N>::kIndexOf >> (4 * (pos * N + mm))) & 15);
        acc += s_D2[pos * N + mm] * s_pf[le][(base + pi) * NV + v];
      }
      if constexpr (SC) {
        if (alpha > 0.0) {
          // (1 - alpha) flux differencing + alpha finite volumes on the LGL subcells (no subcell
          // flux at the element's faces: the surface term below brings the face flux)
          const int fb = (d * K::NLINE + line) * (N - 1);
          const double fr = pos < N - 1 ? s_fvs[le][fb + pos][v] : 0.0;
          const double fl = pos > 0 ? s_fvs[le][fb + pos - 1][v] : 0.0;
          const double iwp = pos == 0 || pos == N - 1 ? iw0 : iw1;
          acc = (1.0 - alpha) * acc + alpha * iwp * (fr - fl);
        }
      }
      const int f = 2 * d + (pos == N - 1 ? 1 : 0);
      const int fi = face_index<DIM, N>(nd, d);
      const bool coarse = LDS_OWN && face_kind(s_fk[le][f]) == kCoarseSide;
      const double lift = pos == N - 1 ? iwN : (pos == 0 ? -iw0 : 0.0);
      // (EARLYF: face fluxes in s_tro, projected coarse sides in s_tr)
      acc += lift * ((coarse != EARLYF) ? s_tro[le][f][0][v][fi] : s_tr[le][f][0][v][fi]);
      du -= J[d] * acc;
      if (VISC) {
        double vacc = 0.0;
#pragma unroll
        for (int mm = 0; mm < N; ++mm) vacc += s_D[pos * N + mm] * fv_own(d, v, node_on_line<DIM, N>(d, line, mm));
        const double fs = coarse ? s_tro[le][f][LDS_OWN ? 1 : 0][v][fi] : s_trv[le][f][0][v][fi];
        vacc += lift * (fs - fv_own(d, v, nd));
        du += J[d] * vacc;
      }
    }
    const int64_t idx = ((int64_t)v * ld + e) * ND + nd;
    if (a.Kout) {
      a.Kout[idx] = du;
      continue;
    }
    const double K1v = a.first ? du : (HOLD_OPS ? k1[it] : a.K1[idx]);
    const double accv = HOLD_OPS ? acc[it] : (a.read_acc ? a.ACC[idx] : 0.0);
    if (a.first) a.K1[idx] = du;
    if (a.acc_mode == 1) a.ACC[idx] = a.bi * du;
    else if (a.acc_mode == 2) a.ACC[idx] = accv + a.bi * du;
    if (a.last) {
      const double inc = a.use_acc_last ? (a.acc_mode == 0 ? accv : a.ACC[idx]) + a.bS * du : a.bS * du;
      a.Uout[idx] = (HOLD_OPS ? un[it] : a.U[idx]) + a.dt * inc;
    } else if (a.wr[my_mem]) {
      a.Yw[my_mem][idx] = (HOLD_OPS ? un[it] : a.U[idx]) + a.dt * (a.a1[my_mem] * K1v + a.a2[my_mem] * du);
    }
  }
}

// Waves per SIMD the register allocation must allow.  3D p=3 blocks (7 waves; 34 KB of LDS for
// Euler, 38 KB for Navier-Stokes) at 72 VGPRs (7 waves per SIMD, no spill since the element
// index is uniform) fit four blocks per CU; the step from three to four blocks took the
// Taylor-Green launch from 90 to 72.5 us (and from two to three, 105 to 90).  The one-wave 2D p=3
// bodies (large launches) are held to 5 waves per SIMD (at most 102 VGPRs): with one element per
// wave and block that meant 96 VGPRs and a 20-byte spill instead of 102-106, 2-6 % less on uniform
// meshes of 128^2-1024^2 elements (6 waves spilled 72-88 bytes and ran slower); the four-element
// body stays below that by itself (62 VGPRs for Euler, 65 with shock capturing, 81 for
// Navier-Stokes).
template <int DIM, int N, bool VISC, bool SPLIT>
constexpr int stage_waves_per_simd() {
  if (DIM == 3 && N == 4) return 7;
  if (DIM == 2 && N == 4 && !SPLIT) return 5;
  return SK<DIM, N, SPLIT>::MINW;
}

template <int DIM, int N, bool VISC, bool SPLIT, bool SC>
__global__ __launch_bounds__((SK<DIM, N, SPLIT>::T * SK<DIM, N, SPLIT>::epb()),
                             (stage_waves_per_simd<DIM, N, VISC, SPLIT>())) void k_stage(StageArgs a, Mesh m, Ops op,
                                                                                       Physics ph) {
  // Workgroups go to the 8 XCDs round-robin (block b to XCD b mod 8); give XCD x the
  // contiguous block range [x G, (x+1) G), G = gridDim / 8, so that neighbouring slots (sorted
  // by member, Morton order inside) share an L2 and neighbour-trace reads can hit there.  (A
  // mapping that keeps each slot on one XCD in every launch, in chunks of 16 blocks, fetched
  // 20 % more from beyond L2: within a launch the neighbours matter, across launches the L2
  // does not keep a slot's data.)
  const int g8 = (int)gridDim.x >> 3;
  const int b = (int)blockIdx.x;
  stage_block<DIM, N, VISC, SK<DIM, N, SPLIT>::epb(), SPLIT, SC>(a, m, op, ph, (b & 7) * g8 + (b >> 3));
}

// ------------------------------------------------------------------------------------------
// Batched stage tick: many independent 2D Euler runs of one polynomial degree, each advanced by
// one of its own stages.  The tiles of the tick (EPB elements of one run each) are the
// concatenated active prefixes of the unfinished runs k0 <= k < k1, tile_off[k] the first tile
// of run k; block b takes tiles b, b + gridDim.x, ... (persistent when the grid is smaller
// than the tile count).  One instantiation per degree keeps the register allocation of a
// single body (both bodies in one kernel double it).
// ------------------------------------------------------------------------------------------
template <int N, int EPB>
__device__ __forceinline__ void batch_tile(const BatchRun* __restrict__ runs, const StageArgs* __restrict__ sargs,
                                           const int32_t* __restrict__ tile_off, int k0, int k1, int64_t tick, int t) {
  int lo = k0, hi = k1 - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_off[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  const int k = __builtin_amdgcn_readfirstlane(lo);
  const BatchRun& r = runs[k];
  const StageArgs& a = sargs[r.sarg0 + (int)(tick % r.S)];
  stage_block<2, N, false, EPB>(a, r.m, r.op, r.ph, t - tile_off[k]);
}

// one block per tile (the grid padded to a multiple of 8), no loop: the register allocation of the
// single-run kernel
template <int N, int EPB>
__global__ __launch_bounds__((SK<2, N>::T * EPB)) void k_stage_batch_flat(const BatchRun* __restrict__ runs,
                                                                          const StageArgs* __restrict__ sargs,
                                                                          const int32_t* __restrict__ tile_off,
                                                                          int k0, int k1, int64_t tick) {
  // XCD-aware as the single-run kernel: XCD x takes the contiguous tile range [x G, (x+1) G)
  // (G = gridDim / 8, the grid padded to a multiple of the 8 XCDs), so that the neighbouring
  // tiles of a run share an L2 (64 runs of the C4 batch: 108.8 -> 106.1 us per tick)
  const int n_tiles = tile_off[k1] - tile_off[k0];
  const int g8 = (int)gridDim.x >> 3;
  const int bb = ((int)blockIdx.x & 7) * g8 + ((int)blockIdx.x >> 3);
  if (bb >= n_tiles) return;
  batch_tile<N, EPB>(runs, sargs, tile_off, k0, k1, tick, tile_off[k0] + bb);
}

// persistent: a fixed grid loops over the tiles (values hoisted out of the loop raise the
// register count, so the autotuner weighs it against the flat form)
template <int N, int EPB>
__global__ __launch_bounds__((SK<2, N>::T * EPB)) void k_stage_batch(const BatchRun* __restrict__ runs,
                                                                     const StageArgs* __restrict__ sargs,
                                                                     const int32_t* __restrict__ tile_off, int k0,
                                                                     int k1, int64_t tick) {
  const int t0 = tile_off[k0];
  const int n_tiles = tile_off[k1] - t0;
  for (int tt = blockIdx.x; tt < n_tiles; tt += gridDim.x) {
    batch_tile<N, EPB>(runs, sargs, tile_off, k0, k1, tick, t0 + tt);
    __syncthreads();
  }
}

template <int DIM, int N>
struct GKc {
  using g = G<DIM, N>;
  static constexpr int ND = g::ND, NF = g::NF, NFC = g::NFC, NV = g::NV, NSUB = g::NSUB, NW = DIM + 1;
  static constexpr int T = DIM == 2 ? 64 : 256;
  // 3D p=3: 256 lanes, at most 64 VGPRs (8 waves per SIMD, without a spill since the trace
  // loads issue together with the own values): eight 15 KB blocks per CU, 36.2 -> 34.7 us per
  // Taylor-Green launch against seven at 72 VGPRs (128-lane blocks: 39 us)
  static constexpr int WPS = DIM == 3 && N == 4 ? 8 : 1;
};

template <int DIM>
__device__ __forceinline__ void grad_vars(const double* u, double gamma, double* w) {
  double rho, v[DIM], p;
  cons_to_prim<DIM>(u, gamma, rho, v, p);
#pragma unroll
  for (int d = 0; d < DIM; ++d) w[d] = v[d];
  w[DIM] = p / rho;
}

template <int DIM, int N>
__global__ __launch_bounds__((GKc<DIM, N>::T), (GKc<DIM, N>::WPS)) void k_grad(StageArgs a, Mesh m, Ops op,
                                                                              Physics ph) {
  using K = GKc<DIM, N>;
  constexpr int ND = K::ND, NF = K::NF, NFC = K::NFC, NV = K::NV, NSUB = K::NSUB, NW = K::NW, T = K::T;
  __shared__ double s_w[NW][ND];
  // neighbour w traces, then central face values; after their last read the lifted gradients
  // take the same LDS (held in registers across one barrier): 15 KB per 3D p=3 block
  constexpr int NTRW = NFC * NSUB * NW * NF, NQ = DIM * NW * ND;
  static_assert(NQ <= NTRW, "gradients fit the trace storage");
  __shared__ double s_trq[NTRW];
  auto s_tr = reinterpret_cast<double (*)[NSUB][NW][NF]>(s_trq);
  auto s_q = reinterpret_cast<double (*)[NW][ND]>(s_trq);
  __shared__ int s_fk[NFC];
  // D, P_0, P_1, R_0, R_1 from the device copy (lane-indexed reads from kernel-argument memory
  // would each be a slow memory round)
  __shared__ double s_op[5][N * N];
  // XCD-aware: the first Ga blocks (the active count rounded up to the 8 XCDs) take the active
  // elements exactly as the stage kernel's blocks do, XCD x the contiguous range [x Ga/8,
  // (x+1) Ga/8), so that a block's neighbours' traces and the stage values the previous stage
  // launch wrote are mostly in its own XCD's L2, and the stage launch after it finds this
  // kernel's viscous flux there; the halo follows in a padded range of its own.  Taylor-Green:
  // 34.3 -> 33.2 us per launch against block b on element b.
  const int Ga = (a.n_act + 7) & ~7;
  const int bx = (int)blockIdx.x;
  int b;
  if (bx < Ga) {
    const int g8 = Ga >> 3;
    b = (bx & 7) * g8 + (bx >> 3);
    if (b >= a.n_act) return;
  } else {
    const int h = bx - Ga, g8 = ((int)gridDim.x - Ga) >> 3;
    const int hh = (h & 7) * g8 + (h >> 3);
    if (hh >= a.n_halo) return;
    b = a.n_act + hh;
  }
  const int e = b < a.n_act ? active_slot(a, b) : a.halo[b - a.n_act];
  const int lane = threadIdx.x;
  const int ld = m.ld;
  const double gamma = ph.gamma;
  const int my_src = src_of(a, member_of_slot(m, e));
  const int lev = m.lev[e];
  // own values and neighbour traces in one memory round: each trace lane reads its face's kind
  // and neighbour slot itself and issues the trace loads right behind them, before the own
  // values are converted (through LDS they would wait for a barrier: a second round)
  constexpr int NTRI = NSUB * NFC * NF, NTR = (NTRI + T - 1) / T;
  int tr_nb[NTR], tr_pk[NTR];
#pragma unroll
  for (int q = 0; q < NTR; ++q) {
    const int it = lane + q * T;
    tr_pk[q] = -1;
    tr_nb[q] = 0;
    if (it < NTRI) {
      const int f = (it / NF) % NFC, sub = it / (NF * NFC);
      tr_pk[q] = m.fk[(int64_t)e * NFC + f];
      tr_nb[q] = m.fn[((int64_t)e * NFC + f) * 4 + sub];
    }
  }
  if (lane < NFC) s_fk[lane] = m.fk[(int64_t)e * NFC + lane];
  double tu[NTR][NV];
  bool tr_on[NTR];
#pragma unroll
  for (int q = 0; q < NTR; ++q) {
    const int it = lane + q * T;
    const int j = it % NF, f = (it / NF) % NFC, sub = it / (NF * NFC);
    tr_on[q] = it < NTRI && (sub == 0 || face_kind(tr_pk[q]) == kCoarseSide);
    if (!tr_on[q]) continue;
    const int nb = tr_nb[q];
    const int src = src_of(a, member_of_slot(m, nb));
    const int nn = face_node<DIM, N>(f >> 1, 1 - (f & 1), j);
#pragma unroll
    for (int v = 0; v < NV; ++v) tu[q][v] = stage_value(a, src, ((int64_t)v * ld + nb) * ND + nn);
  }
  for (int nd = lane; nd < ND; nd += T) {
    double u[NV], w[NW];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = stage_value(a, my_src, ((int64_t)v * ld + e) * ND + nd);
    grad_vars<DIM>(u, gamma, w);
#pragma unroll
    for (int k = 0; k < NW; ++k) s_w[k][nd] = w[k];
  }
  for (int t = lane; t < 5 * N * N; t += T) s_op[t / (N * N)][t % (N * N)] = op.dD[N * N + t];
  // neighbour traces, converted to w at the trace node
#pragma unroll
  for (int q = 0; q < NTR; ++q) {
    if (!tr_on[q]) continue;
    const int it = lane + q * T;
    const int j = it % NF, f = (it / NF) % NFC, sub = it / (NF * NFC);
    double w[NW];
    grad_vars<DIM>(tu[q], gamma, w);
#pragma unroll
    for (int k = 0; k < NW; ++k) s_tr[f][sub][k][j] = w[k];
  }
  __syncthreads();
  // fine sides: coarse w trace interpolated to the sub-face (into sub-slot 1)
  for (int it = lane; it < NFC * NW * NF; it += T) {
    const int j = it % NF, k = (it / NF) % NW, f = it / (NF * NW);
    const int32_t pk = s_fk[f];
    if (face_kind(pk) != kFineSide) continue;
    const int s0 = face_sub0(pk), s1 = face_sub1(pk);
    double val = 0.0;
    if (DIM == 2) {
#pragma unroll
      for (int q = 0; q < N; ++q) val += s_op[1 + s0][j * N + q] * s_tr[f][0][k][q];
    } else {
      const int ja = j % N, jb = j / N;
#pragma unroll
      for (int kb = 0; kb < N; ++kb) {
        double row = 0.0;
#pragma unroll
        for (int ka = 0; ka < N; ++ka) row += s_op[1 + s0][ja * N + ka] * s_tr[f][0][k][ka + N * kb];
        val += s_op[1 + s1][jb * N + kb] * row;
      }
    }
    s_tr[f][1][k][j] = val;
  }
  __syncthreads();
  // central face values w* on every (sub-)face node, in place
  for (int it = lane; it < NSUB * NFC * NF; it += T) {
    const int j = it % NF;
    const int f = (it / NF) % NFC;
    const int sub = it / (NF * NFC);
    const int kind = face_kind(s_fk[f]);
    if (sub > 0 && kind != kCoarseSide) continue;
    const int d = f >> 1, side = f & 1;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      double own;
      if (kind == kCoarseSide) {
        const int m0 = sub & 1, m1 = (sub >> 1) & 1;
        own = 0.0;
        if (DIM == 2) {
#pragma unroll
          for (int q = 0; q < N; ++q) own += s_op[1 + m0][j * N + q] * s_w[k][face_node<DIM, N>(d, side, q)];
        } else {
          const int ja = j % N, jb = j / N;
#pragma unroll
          for (int kb = 0; kb < N; ++kb) {
            double row = 0.0;
#pragma unroll
            for (int ka = 0; ka < N; ++ka) row += s_op[1 + m0][ja * N + ka] * s_w[k][face_node<DIM, N>(d, side, ka + N * kb)];
            own += s_op[1 + m1][jb * N + kb] * row;
          }
        }
      } else {
        own = s_w[k][face_node<DIM, N>(d, side, j)];
      }
      const int ts = kind == kFineSide ? 1 : sub;
      s_tr[f][sub][k][j] = 0.5 * (own + s_tr[f][ts][k][j]);
    }
  }
  __syncthreads();
  // lifted gradients
  const double iw0 = op.iw[0], iwN = op.iw[N - 1];
  constexpr int NQL = (NQ + T - 1) / T;   // per lane
  double qv[NQL];
#pragma unroll
  for (int q = 0; q < NQL; ++q) {
    const int it = lane + q * T;
    if (it >= NQ) continue;
    const int nd = it % ND, k = (it / ND) % NW, d = it / (ND * NW);
    int line, pos;
    line_of<DIM, N>(nd, d, line, pos);
    double acc = 0.0;
#pragma unroll
    for (int mm = 0; mm < N; ++mm) acc += s_op[0][pos * N + mm] * s_w[k][node_on_line<DIM, N>(d, line, mm)];
    if (pos == N - 1 || pos == 0) {
      const int f = 2 * d + (pos == N - 1 ? 1 : 0);
      const int fi = face_index<DIM, N>(nd, d);
      double ws;
      if (face_kind(s_fk[f]) == kCoarseSide) {
        ws = 0.0;
        if (DIM == 2) {
#pragma unroll
          for (int ms = 0; ms < 2; ++ms)
#pragma unroll
            for (int q = 0; q < N; ++q) ws += s_op[3 + ms][fi * N + q] * s_tr[f][ms][k][q];
        } else {
          const int ja = fi % N, jb = fi / N;
#pragma unroll
          for (int ms = 0; ms < 4; ++ms) {
            const int m0 = ms & 1, m1 = (ms >> 1) & 1;
#pragma unroll
            for (int kb = 0; kb < N; ++kb) {
              double row = 0.0;
#pragma unroll
              for (int ka = 0; ka < N; ++ka) row += s_op[3 + m0][ja * N + ka] * s_tr[f][ms][k][ka + N * kb];
              ws += s_op[3 + m1][jb * N + kb] * row;
            }
          }
        }
      } else {
        ws = s_tr[f][0][k][fi];
      }
      const double jump = ws - s_w[k][nd];
      acc += pos == N - 1 ? iwN * jump : -iw0 * jump;
    }
    qv[q] = m.jac[lev][d] * acc;
  }
  __syncthreads();   // every read of the face values is done: the gradients take their place
#pragma unroll
  for (int q = 0; q < NQL; ++q) {
    const int it = lane + q * T;
    if (it < NQ) s_q[it / (NW * ND)][(it / ND) % NW][it % ND] = qv[q];
  }
  __syncthreads();
  // viscous flux at every node, one direction per item (DIM ND items: 3D p=3 uses three of
  // the four waves instead of one)
  for (int it = lane; it < DIM * ND; it += T) {
    const int nd = it % ND, d = it / ND;
    double divv = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) divv += s_q[k][k][nd];
    double f[NV];
    f[0] = 0.0;
    double en = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      double tau = ph.mu * (s_q[d][k][nd] + s_q[k][d][nd]);
      if (k == d) tau -= 2.0 / 3.0 * ph.mu * divv;
      f[1 + k] = tau;
      en += tau * s_w[k][nd];
    }
    f[DIM + 1] = en + ph.kappa * s_q[d][DIM][nd];
#pragma unroll
    for (int v = 0; v < NV; ++v) a.Fv[(((int64_t)d * NV + v) * ld + e) * ND + nd] = f[v];
  }
}

template <int DIM, int N>
hipError_t launch_grad_t(const StageArgs& a, const Mesh& m, const Ops& op, const Physics& ph, hipStream_t s,
                         hipEvent_t ev0, hipEvent_t ev1) {
  const int nb = a.n_act + a.n_halo;
  if (nb <= 0) return hipSuccess;
  const int blocks = ((a.n_act + 7) & ~7) + ((a.n_halo + 7) & ~7);   // active and halo parts, each a multiple of 8
  if (ev0)
    hipExtLaunchKernelGGL((k_grad<DIM, N>), dim3(blocks), dim3(GKc<DIM, N>::T), 0, s, ev0, ev1, 0, a, m, op, ph);
  else
    hipLaunchKernelGGL((k_grad<DIM, N>), dim3(blocks), dim3(GKc<DIM, N>::T), 0, s, a, m, op, ph);
  return hipGetLastError();
}

template <int DIM, int N, bool VISC, bool SPLIT, bool SC>
hipError_t launch_stage_v(const StageArgs& a, const Mesh& m, const Ops& op, const Physics& ph, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1) {
  using K = SK<DIM, N, SPLIT>;
  constexpr int EPB = K::epb();
  const int blocks = ((a.n_act + EPB - 1) / EPB + 7) & ~7;   // a multiple of the 8 XCDs
  if (ev0)
    hipExtLaunchKernelGGL((k_stage<DIM, N, VISC, SPLIT, SC>), dim3(blocks), dim3(K::T * EPB), 0, s, ev0, ev1, 0,
                          a, m, op, ph);
  else
    hipLaunchKernelGGL((k_stage<DIM, N, VISC, SPLIT, SC>), dim3(blocks), dim3(K::T * EPB), 0, s, a, m, op, ph);
  return hipGetLastError();
}

// 2D p=3 launches with few active elements are latency-bound: two waves per element (pair and
// face fluxes side by side) finish sooner; with many elements the launch is throughput-bound
// and the one-wave body (four elements per block, flux phase across the block) issues fewer
// instructions per element.  Measured on uniform meshes: the split body is faster up to 1024
// elements (5.8 vs 6.5 us per launch) and on the adaptive KH launches (~1400: 7.4 vs 7.8 us),
// the one-wave body from 2304 on (7.1 vs 7.9 us); with shock capturing (the paper's KH state)
// likewise, 1024: 7.8 vs 8.4 us, 2304: 8.6 vs 7.7 us, 4096: 12.0 vs 8.8 us.
constexpr int kSplitMaxElements = STAGE_SPLIT_MAX;

template <int DIM, int N, bool VISC, bool SC = false>
hipError_t launch_stage_t(const StageArgs& a, const Mesh& m, const Ops& op, const Physics& ph, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1) {
  if (a.n_act <= 0) return hipSuccess;
  if constexpr (DIM == 2 && N == 4) {
    if (a.n_act <= kSplitMaxElements)
      return launch_stage_v<DIM, N, VISC, true, SC>(a, m, op, ph, s, ev0, ev1);
  }
  return launch_stage_v<DIM, N, VISC, false, SC>(a, m, op, ph, s, ev0, ev1);
}

}  // namespace

template <int N, int EPB>
hipError_t launch_batch_t(bool persistent, int grid, const BatchRun* runs, const StageArgs* sargs,
                          const int32_t* tile_off, int k0, int k1, int64_t tick, hipStream_t s) {
  const dim3 b(SK<2, N>::T * EPB);
  if (persistent)
    hipLaunchKernelGGL((k_stage_batch<N, EPB>), dim3(grid), b, 0, s, runs, sargs, tile_off, k0, k1, tick);
  else
    hipLaunchKernelGGL((k_stage_batch_flat<N, EPB>), dim3((grid + 7) & ~7), b, 0, s, runs, sargs, tile_off, k0, k1,
                       tick);
  return hipGetLastError();
}

hipError_t launch_stage_batch(int N, int M, int grid, bool persistent, const BatchRun* runs, const StageArgs* sargs,
                              const int32_t* tile_off, int k0, int k1, int64_t tick, hipStream_t s) {
  if (grid <= 0 || k1 <= k0) return hipSuccess;
  // M elements of degree 3 per tile (64 M lanes), 2 M of degree 2 (32 lanes each)
  if (N == 4 && M == 1) return launch_batch_t<4, 1>(persistent, grid, runs, sargs, tile_off, k0, k1, tick, s);
  if (N == 4 && M == 2) return launch_batch_t<4, 2>(persistent, grid, runs, sargs, tile_off, k0, k1, tick, s);
  if (N == 4 && M == 4) return launch_batch_t<4, 4>(persistent, grid, runs, sargs, tile_off, k0, k1, tick, s);
  if (N == 3 && M == 1) return launch_batch_t<3, 2>(persistent, grid, runs, sargs, tile_off, k0, k1, tick, s);
  if (N == 3 && M == 2) return launch_batch_t<3, 4>(persistent, grid, runs, sargs, tile_off, k0, k1, tick, s);
  if (N == 3 && M == 4) return launch_batch_t<3, 8>(persistent, grid, runs, sargs, tile_off, k0, k1, tick, s);
  return hipErrorNotSupported;
}

int stage_body_id(int dim, int N, int n_act, bool sc) {
  return ((dim == 2 && N == 4 && n_act > 0 && n_act <= kSplitMaxElements) ? 1 : 0) + (sc ? 2 : 0);
}

hipError_t launch_stage(int dim, int N, bool viscous, const StageArgs& a, const Mesh& m, const Ops& op,
                        const Physics& ph, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (!viscous && a.sc) {
    if (dim == 2 && N == 4) return launch_stage_t<2, 4, false, true>(a, m, op, ph, s, e0, e1);
    if (dim == 2 && N == 3) return launch_stage_t<2, 3, false, true>(a, m, op, ph, s, e0, e1);
    return hipErrorNotSupported;
  }
  if (!viscous) {
    if (dim == 2 && N == 4) return launch_stage_t<2, 4, false>(a, m, op, ph, s, e0, e1);
    if (dim == 2 && N == 3) return launch_stage_t<2, 3, false>(a, m, op, ph, s, e0, e1);
    if (dim == 3 && N == 4) return launch_stage_t<3, 4, false>(a, m, op, ph, s, e0, e1);
    if (dim == 3 && N == 3) return launch_stage_t<3, 3, false>(a, m, op, ph, s, e0, e1);
  } else {
    if (dim == 2 && N == 4) return launch_stage_t<2, 4, true>(a, m, op, ph, s, e0, e1);
    if (dim == 2 && N == 3) return launch_stage_t<2, 3, true>(a, m, op, ph, s, e0, e1);
    if (dim == 3 && N == 4) return launch_stage_t<3, 4, true>(a, m, op, ph, s, e0, e1);
    if (dim == 3 && N == 3) return launch_stage_t<3, 3, true>(a, m, op, ph, s, e0, e1);
  }
  return hipErrorNotSupported;
}

hipError_t launch_gradients(int dim, int N, const StageArgs& a, const Mesh& m, const Ops& op, const Physics& ph,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (dim == 2 && N == 4) return launch_grad_t<2, 4>(a, m, op, ph, s, e0, e1);
  if (dim == 2 && N == 3) return launch_grad_t<2, 3>(a, m, op, ph, s, e0, e1);
  if (dim == 3 && N == 4) return launch_grad_t<3, 4>(a, m, op, ph, s, e0, e1);
  if (dim == 3 && N == 3) return launch_grad_t<3, 3>(a, m, op, ph, s, e0, e1);
  return hipErrorNotSupported;
}

}  // namespace perk
