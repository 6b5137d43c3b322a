// Adjoint (vector-Jacobian product) of the DGSEM Euler right-hand side for gfx950, and the
// stage-wise reverse sweep of the partitioned P-ERK step built on it.
//
// For a cotangent W and the stage state Y the kernel forms G = F'(Y)^T W element by element
// ("gather" form: each element writes only its own rows of G, so there are no atomics):
//   * volume: every unordered node pair (a, b) of a coordinate line carries one two-point
//     flux f#(u_a, u_b) that enters du_a with -J 2 D_ab and du_b with -J 2 D_ba; its cotangent
//     P = -J (2 D_ab W_a + 2 D_ba W_b) is pulled back through the local Jacobians of f#;
//   * faces: the HLL flux of a face node enters the lifting of both neighbours; the element
//     collects the flux cotangent of both sides (its own W and the neighbour's W, projected
//     with R_m^T across a 2:1 mortar) and pulls it back through the derivative with respect to
//     its own trace only (the neighbour does the same for its trace); on the coarse side of a
//     mortar the result lives on the sub-face nodes and is taken back with P_m^T.
// The local flux Jacobians are the derivative of the computed map along the branches it takes,
// in reverse mode written out (one forward and one backward pass per flux): the
// entropy-conserving pair flux (logarithmic mean and its series branch) and the HLL face flux
// (Davis wave speeds, ties resolved towards the first argument).
//
// Block layout: one element per block; in 2D the pair pull-backs run on the first wave and the
// face pull-backs on the second, so that neither waits for the other inside a wave.  The
// derivative and mortar tables come from the device operator table into LDS (lane-indexed
// reads of kernel-argument memory are slow).
//
// Reverse sweep of one step (Sec. 3.1: Y_i = U_n + dt (a_{i,1} K_1 + a_{i,i-1} K_{i-1}),
// K_i = I_i F(Y_i), U_{n+1} = U_n + dt sum_i b_i K_i), from the stage values stored by a
// forward recomputation: with K~_i the cotangent of K_i,
//   Ybar_i = F'(Y_i)^T (I_i K~_i);  Ubar += Ybar_i;  K~_1 += dt a_{i,1} Ybar_i;
//   K~_{i-1} = dt b_{i-1} lam + dt a_{i,i-1} Ybar_i,
// per element with its member's coefficients; only active elements and their face
// neighbours are launched (everything else has Ybar_i = 0).

#include "perk_device.h"

namespace perk {
namespace {

// ------------------------------------------------------------ reverse mode for the pair flux
// Value and both partial derivatives of the logarithmic mean along the branch the dual form
// takes (same u, same threshold): series (a+b)/(2F(u)) or (b-a)/ln(b/a).  ia, ib: 1/a, 1/b.
__device__ __forceinline__ void log_mean_d(double a, double b, double ia, double ib, double& lm, double& da,
                                           double& db) {
  const double s = a + b, t = b - a;
  const double is = rcp(s);
  const double f = t * is, u = f * f;
  if (u < 1e-2) {
    // F(u) = sum_k u^k / (2k+1), k = 0..7, and F'(u), in Horner form (constant reciprocals, no
    // divisions)
    constexpr double c1 = 1.0 / 3, c2 = 1.0 / 5, c3 = 1.0 / 7, c4 = 1.0 / 9, c5 = 1.0 / 11, c6 = 1.0 / 13,
                     c7 = 1.0 / 15;
    const double F = 1.0 + u * (c1 + u * (c2 + u * (c3 + u * (c4 + u * (c5 + u * (c6 + u * c7))))));
    const double Fp =
        c1 + u * (2.0 * c2 + u * (3.0 * c3 + u * (4.0 * c4 + u * (5.0 * c5 + u * (6.0 * c6 + u * (7.0 * c7))))));
    const double iF = rcp(F);
    const double h = 0.5 * iF;
    lm = s * h;
    const double c = Fp * f * iF * iF * is;
    da = h + 2.0 * c * b;
    db = h - 2.0 * c * a;
  } else {
    const double L = log(b * ia);
    const double iL = rcp(L), iL2 = iL * iL;
    lm = t * iL;
    da = (t * ia - L) * iL2;
    db = (L - t * ib) * iL2;
  }
}
// P^T (d f#/d u_L) and P^T (d f#/d u_R) of the entropy-conserving flux in one forward and one
// backward pass (the dual form needs 2 n_v forward passes); one reciprocal per denominator
// (densities, pressures, the logarithmic means).  The same derivative as the dual form up to
// rounding (host check on random states of both branches: 5e-14 relative).
template <int DIM>
__device__ __forceinline__ void ec_flux_vjp(const double* uL, const double* uR, int d, double gamma,
                                            const double* P, double* gL, double* gR) {
  constexpr int NV = DIM + 2;
  const double gm1 = gamma - 1.0;
  const double rL = uL[0], rR = uR[0];
  const double irL = rcp(rL), irR = rcp(rR);
  double vL[DIM], vR[DIM], keL = 0.0, keR = 0.0;
  for (int k = 0; k < DIM; ++k) {
    vL[k] = uL[1 + k] * irL;
    vR[k] = uR[1 + k] * irR;
    keL = keL + 0.5 * (uL[1 + k] * vL[k]);
    keR = keR + 0.5 * (uR[1 + k] * vR[k]);
  }
  const double pL = gm1 * (uL[NV - 1] - keL), pR = gm1 * (uR[NV - 1] - keR);
  const double ipL = rcp(pL), ipR = rcp(pR);
  double rho_ln, dra, drb, beta_ln, dba, dbb;
  log_mean_d(rL, rR, irL, irR, rho_ln, dra, drb);
  const double bL = rL * ipL, bR = rR * ipR;
  log_mean_d(bL, bR, pL * irL, pR * irR, beta_ln, dba, dbb);
  const double vd = 0.5 * (vL[d] + vR[d]);
  double vLvR = 0.0;
  for (int k = 0; k < DIM; ++k) vLvR = vLvR + vL[k] * vR[k];
  const double f0 = rho_ln * vd;
  const double ib = rcp(gm1 * beta_ln);
  const double Q = 0.5 * vLvR + ib;
  const double PE = P[NV - 1];
  double vLb[DIM], vRb[DIM];
  double f0b = P[0] + PE * Q;
  const double Qb = PE * f0;
  for (int k = 0; k < DIM; ++k) {
    f0b += P[1 + k] * (0.5 * (vL[k] + vR[k]));
    vLb[k] = 0.5 * f0 * P[1 + k] + 0.5 * Qb * vR[k];
    vRb[k] = 0.5 * f0 * P[1 + k] + 0.5 * Qb * vL[k];
  }
  double pLb = 0.5 * PE * vR[d] + 0.5 * P[1 + d];
  double pRb = 0.5 * PE * vL[d] + 0.5 * P[1 + d];
  vRb[d] += 0.5 * PE * pL;
  vLb[d] += 0.5 * PE * pR;
  const double beta_lnb = -Qb * gm1 * ib * ib;
  const double rho_lnb = f0b * vd, vdb = f0b * rho_ln;
  vLb[d] += 0.5 * vdb;
  vRb[d] += 0.5 * vdb;
  double rLb = rho_lnb * dra, rRb = rho_lnb * drb;
  const double bLb = beta_lnb * dba * ipL, bRb = beta_lnb * dbb * ipR;
  rLb += bLb;
  pLb -= bLb * bL;
  rRb += bRb;
  pRb -= bRb * bR;
  // p = (gamma-1)(E - ke), ke = sum 1/2 m_k v_k, v_k = m_k / r
  const double kLb = -gm1 * pLb, kRb = -gm1 * pRb;
  gL[NV - 1] = gm1 * pLb;
  gR[NV - 1] = gm1 * pRb;
  for (int k = 0; k < DIM; ++k) {
    const double vbl = (vLb[k] + 0.5 * uL[1 + k] * kLb) * irL, vbr = (vRb[k] + 0.5 * uR[1 + k] * kRb) * irR;
    gL[1 + k] = 0.5 * vL[k] * kLb + vbl;
    gR[1 + k] = 0.5 * vR[k] * kRb + vbr;
    rLb -= vbl * vL[k];
    rRb -= vbr * vR[k];
  }
  gL[0] = rLb;
  gR[0] = rRb;
}

// (d f*/d u_L)^T Hb and (d f*/d u_R)^T Hb of the HLL flux with Davis wave speeds (normal +e_d
// from L to R) in one forward and one backward pass.  Branches as in the forward flux:
// s_L >= 0 takes the left Euler flux, s_R <= 0 the right one, otherwise the HLL average; the
// min / max of the wave speeds pass their cotangent to the argument they took (ties: left).
// One reciprocal per denominator.  Same derivative as forward-mode dual numbers up to rounding
// (host check on random sub- and supersonic states: 4e-15 relative).
template <int DIM>
__device__ __forceinline__ void hll_flux_vjp(const double* uL, const double* uR, int d, double gamma,
                                             const double* Hb, double* gL, double* gR) {
  constexpr int NV = DIM + 2;
  const double gm1 = gamma - 1.0;
  const double* us[2] = {uL, uR};
  double irho[2], v[2][DIM], p[2], c[2], fx[2][NV];
  for (int s = 0; s < 2; ++s) {
    const double* u = us[s];
    irho[s] = rcp(u[0]);
    double ke = 0.0;
    for (int k = 0; k < DIM; ++k) {
      v[s][k] = u[1 + k] * irho[s];
      ke = ke + 0.5 * (u[1 + k] * v[s][k]);
    }
    p[s] = gm1 * (u[NV - 1] - ke);
    c[s] = sqrt(gamma * p[s] * irho[s]);
    fx[s][0] = u[1 + d];
    for (int k = 0; k < DIM; ++k) fx[s][1 + k] = u[1 + k] * v[s][d];
    fx[s][1 + d] = fx[s][1 + d] + p[s];
    fx[s][NV - 1] = (u[NV - 1] + p[s]) * v[s][d];
  }
  const double aL = v[0][d] - c[0], aR = v[1][d] - c[1];
  const double bL = v[0][d] + c[0], bR = v[1][d] + c[1];
  const bool sl_r = aR < aL, sr_r = bR > bL;   // ties go to the left state
  const double sL = sl_r ? aR : aL, sR = sr_r ? bR : bL;
  double fb[2][NV], ub[2][NV];
  double sLb = 0.0, sRb = 0.0;
  for (int k = 0; k < NV; ++k) {
    ub[0][k] = 0.0;
    ub[1][k] = 0.0;
  }
  if (sL >= 0.0) {
    for (int k = 0; k < NV; ++k) {
      fb[0][k] = Hb[k];
      fb[1][k] = 0.0;
    }
  } else if (sR <= 0.0) {
    for (int k = 0; k < NV; ++k) {
      fb[0][k] = 0.0;
      fb[1][k] = Hb[k];
    }
  } else {
    const double id = rcp(sR - sL);
    for (int k = 0; k < NV; ++k) {
      const double du = uR[k] - uL[k];
      const double f = (sR * fx[0][k] - sL * fx[1][k] + sL * sR * du) * id;
      const double h = Hb[k] * id;
      fb[0][k] = h * sR;
      fb[1][k] = -h * sL;
      ub[1][k] += h * sL * sR;
      ub[0][k] -= h * sL * sR;
      sRb += h * (fx[0][k] + sL * du - f);
      sLb += h * (sR * du - fx[1][k] + f);
    }
  }
  // wave speeds: s = v_d -+ c
  double vdb[2], cb[2];
  vdb[0] = (sl_r ? 0.0 : sLb) + (sr_r ? 0.0 : sRb);
  vdb[1] = (sl_r ? sLb : 0.0) + (sr_r ? sRb : 0.0);
  cb[0] = (sr_r ? 0.0 : sRb) - (sl_r ? 0.0 : sLb);
  cb[1] = (sr_r ? sRb : 0.0) - (sl_r ? sLb : 0.0);
  double* gs[2] = {gL, gR};
  for (int s = 0; s < 2; ++s) {
    const double* u = us[s];
    double* g = ub[s];
    const double* f = fb[s];
    double vb[DIM];
    for (int k = 0; k < DIM; ++k) vb[k] = 0.0;
    double pb = 0.0, rb = 0.0;
    // c = sqrt(x), x = gamma p / rho
    const double xb = cb[s] * 0.5 * rcp(c[s]) * gamma * irho[s];
    pb += xb;
    rb -= xb * p[s] * irho[s];
    vb[d] += vdb[s];
    // Euler flux in direction d
    g[1 + d] += f[0];
    for (int k = 0; k < DIM; ++k) {
      g[1 + k] += f[1 + k] * v[s][d];
      vb[d] += f[1 + k] * u[1 + k];
    }
    pb += f[1 + d];
    g[NV - 1] += f[NV - 1] * v[s][d];
    pb += f[NV - 1] * v[s][d];
    vb[d] += f[NV - 1] * (u[NV - 1] + p[s]);
    // p = (gamma-1)(E - ke), ke = sum 1/2 m_k v_k, v_k = m_k / rho
    g[NV - 1] += gm1 * pb;
    const double keb = -gm1 * pb;
    for (int k = 0; k < DIM; ++k) {
      g[1 + k] += 0.5 * v[s][k] * keb;
      vb[k] += 0.5 * u[1 + k] * keb;
      g[1 + k] += vb[k] * irho[s];
      rb -= vb[k] * v[s][k] * irho[s];
    }
    g[0] += rb;
    for (int k = 0; k < NV; ++k) gs[s][k] = g[k];
  }
}

// stage value of slot data: 0 U_n, 1 Yin, 2 U_n + dt c_i K_1 (as in the stage kernel)
__device__ __forceinline__ double vstage(const VjpArgs& a, int src, int64_t idx) {
  if (src == 0) return a.U[idx];
  if (src == 1) return a.Yin[idx];
  return a.U[idx] + a.dt * a.ci * a.K1[idx];
}

template <int DIM, int N>
struct AK {
  using g = G<DIM, N>;
  static constexpr int ND = g::ND, NF = g::NF, NFC = g::NFC, NV = g::NV, NSUB = g::NSUB;
  static constexpr int NPL = N * (N - 1) / 2;
  static constexpr int NLINE = DIM == 2 ? N : N * N;
  static constexpr int NP = DIM * NLINE * NPL;
  static constexpr int NFI = NSUB * NFC * NF;          // face items (sub-faces on coarse sides)
  static constexpr bool SPLIT = DIM == 2;              // pairs on wave 0, faces on wave 1
  static constexpr int T = DIM == 2 ? 128 : (N == 4 ? 384 : 192);
};

// Operator tables staged in LDS: t[0] 2 D with a zero diagonal, t[1] D, t[2 + m] P_m,
// t[4 + m] R_m (N x N, row-major).
// R_m[i, k] (coarse node i, sub-face node k) and P_m[k, i] of a 2:1 mortar, tensor products in 3D
template <int DIM, int N>
__device__ __forceinline__ double Rm(const double (*t)[N * N], int m, int i, int k) {
  if (DIM == 2) return t[4 + m][i * N + k];
  return t[4 + (m & 1)][(i % N) * N + (k % N)] * t[4 + ((m >> 1) & 1)][(i / N) * N + (k / N)];
}
template <int DIM, int N>
__device__ __forceinline__ double Pm(const double (*t)[N * N], int m0, int m1, int k, int i) {
  if (DIM == 2) return t[2 + m0][k * N + i];
  return t[2 + m0][(k % N) * N + (i % N)] * t[2 + m1][(k / N) * N + (i / N)];
}

template <int DIM, int N>
__global__ __launch_bounds__((AK<DIM, N>::T)) void k_rhs_vjp(VjpArgs a, Mesh m, Ops op, Physics ph) {
  using K = AK<DIM, N>;
  constexpr int ND = K::ND, NF = K::NF, NFC = K::NFC, NV = K::NV, NSUB = K::NSUB, T = K::T;
  constexpr int NP = K::NP, NPL = K::NPL, NFI = K::NFI;
  __shared__ double s_u[NV][ND];                 // own stage state
  __shared__ double s_w[NV][ND];                 // own cotangent
  __shared__ double s_tr[NFC][NSUB][NV][NF];     // neighbour stage traces (fine side: interpolated in sub 1)
  __shared__ double s_tw[NFC][NSUB][NV][NF];     // neighbour cotangent traces (raw)
  __shared__ double s_jn[NFC][NSUB];             // neighbour 2/h in the face direction
  __shared__ double s_ga[NP][NV], s_gb[NP][NV];  // pair pull-backs to the first / second node
  __shared__ double s_gf[NFC][NSUB][NV][NF];     // face pull-backs (coarse side: on sub-face nodes)
  __shared__ double s_op[6][N * N];              // 2D (zero diagonal), D, P_0, P_1, R_0, R_1
  __shared__ int s_fk[NFC];
  __shared__ int s_fn[NFC][4];

  const int lane = threadIdx.x;
  const int b = blockIdx.x;
  const int e = b < a.n_act ? b : a.halo[b - a.n_act];
  const int ld = m.ld;
  const double gamma = ph.gamma;
  const int mem = member_of_slot(m, e);
  const int lev = m.lev[e];
  double J[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) J[d] = m.jac[lev][d];
  // the members' stage-value codes packed two bits each (a member-indexed read of the argument
  // array from a lane-dependent neighbour would be a gather from kernel-argument memory)
  int src_bits = 0;
#pragma unroll
  for (int r = 0; r < kMaxMembers; ++r) src_bits |= a.src[r] << (2 * r);
  auto src_m = [&](int r) { return (src_bits >> (2 * r)) & 3; };

  // ---- A: own state and cotangent, connectivity, operator tables; then neighbour traces
  if (lane < NFC) s_fk[lane] = m.fk[(int64_t)e * NFC + lane];
  if (lane < NFC * 4) s_fn[lane / 4][lane % 4] = m.fn[(int64_t)e * NFC * 4 + lane];
  for (int t = lane; t < 6 * N * N; t += T) s_op[t / (N * N)][t % (N * N)] = op.dD[t];
  const int my_src = src_m(mem);
  const bool w_own = e < a.n_w;
  for (int w = lane; w < NV * ND; w += T) {
    const int v = w / ND, nd = w - v * ND;
    const int64_t idx = ((int64_t)v * ld + e) * ND + nd;
    s_u[v][nd] = vstage(a, my_src, idx);
    s_w[v][nd] = w_own ? a.W[idx] : 0.0;
  }
  // 2D: the epilogue operands of the lane's (variable, node) item come in with the first loads
  // (no memory round after the last barrier); 3D reads them at the end (its registers are full)
  constexpr bool PRE = DIM == 2;
  static_assert(!PRE || NV * ND <= T, "one epilogue item per lane");
  double pre_ubar = 0.0, pre_k1bar = 0.0, pre_lam = 0.0;
  if (PRE && lane < NV * ND) {
    const int v = lane / ND, nd = lane - v * ND;
    const int64_t idx = ((int64_t)v * ld + e) * ND + nd;
    if (a.Ubar) pre_ubar = a.Ubar[idx];
    if (a.K1bar) pre_k1bar = a.K1bar[idx];
    if (a.Kprev) pre_lam = a.lam[idx];
  }
  __syncthreads();
  for (int w = lane; w < NFI * NV; w += T) {
    const int j = w % NF;
    const int v = (w / NF) % NV;
    const int f = (w / (NF * NV)) % NFC;
    const int sub = w / (NF * NV * NFC);
    const int kind = face_kind(s_fk[f]);
    if (sub > 0 && kind != kCoarseSide) continue;
    const int nb = s_fn[f][sub];
    const int d = f >> 1, side = f & 1;
    const int nn = face_node<DIM, N>(d, 1 - side, j);
    const int64_t idx = ((int64_t)v * ld + nb) * ND + nn;
    s_tr[f][sub][v][j] = vstage(a, src_m(member_of_slot(m, nb)), idx);
    s_tw[f][sub][v][j] = nb < a.n_w ? a.W[idx] : 0.0;
    if (v == 0 && j == 0) s_jn[f][sub] = m.jac[m.lev[nb]][d];
  }
  __syncthreads();
  // fine side: coarse trace interpolated to this sub-face into sub-slot 1
  for (int w = lane; w < NFC * NV * NF; w += T) {
    const int j = w % NF;
    const int v = (w / NF) % NV;
    const int f = w / (NF * NV);
    const int32_t pk = s_fk[f];
    if (face_kind(pk) != kFineSide) continue;
    const int s0 = face_sub0(pk), s1 = face_sub1(pk);
    double val = 0.0;
    for (int k = 0; k < NF; ++k) val += Pm<DIM, N>(s_op, s0, s1, j, k) * s_tr[f][0][v][k];
    s_tr[f][1][v][j] = val;
  }
  __syncthreads();

  // ---- D: pull-backs through the local flux Jacobians, one flux per lane
  auto pair_vjp = [&](int w) {
    const int pl = w % NPL;
    const int line = (w / NPL) % K::NLINE;
    const int d = w / (NPL * K::NLINE);
    int pa = 0, pb = 1, cnt = 0;
    for (int x = 0; x < N; ++x)
      for (int y = x + 1; y < N; ++y) {
        if (cnt == pl) { pa = x; pb = y; }
        ++cnt;
      }
    const int na = node_on_line<DIM, N>(d, line, pa), nb = node_on_line<DIM, N>(d, line, pb);
    const double dab = s_op[0][pa * N + pb], dba = s_op[0][pb * N + pa];
    double Pb[NV], uA[NV], uB[NV], gA[NV], gB[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Pb[v] = -J[d] * (dab * s_w[v][na] + dba * s_w[v][nb]);
      uA[v] = s_u[v][na];
      uB[v] = s_u[v][nb];
    }
    ec_flux_vjp<DIM>(uA, uB, d, gamma, Pb, gA, gB);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      s_ga[w][v] = gA[v];
      s_gb[w][v] = gB[v];
    }
  };
  const double iw0 = op.iw[0], iwN = op.iw[N - 1];
  auto face_vjp = [&](int r) {
    const int j = r % NF;
    const int f = (r / NF) % NFC;
    const int sub = r / (NF * NFC);
    const int32_t pk = s_fk[f];
    const int kind = face_kind(pk);
    if (sub > 0 && kind != kCoarseSide) return;
    const int d = f >> 1, side = f & 1;
    const double lift_own = side == 1 ? -iwN : iw0;
    const double lift_nb = side == 1 ? iw0 : -iwN;
    double own[NV], oth[NV], Hb[NV];
    if (kind == kCoarseSide) {
      const int m0 = sub & 1, m1 = (sub >> 1) & 1;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double x = 0.0, h = 0.0;
#pragma unroll 2
        for (int i = 0; i < NF; ++i) {
          const int on = face_node<DIM, N>(d, side, i);
          x += Pm<DIM, N>(s_op, m0, m1, j, i) * s_u[v][on];
          h += Rm<DIM, N>(s_op, sub, i, j) * s_w[v][on];
        }
        own[v] = x;
        oth[v] = s_tr[f][sub][v][j];
        Hb[v] = J[d] * lift_own * h + s_jn[f][sub] * lift_nb * s_tw[f][sub][v][j];
      }
    } else {
      const int on = face_node<DIM, N>(d, side, j);
      const int ts = kind == kFineSide ? 1 : 0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        own[v] = s_u[v][on];
        oth[v] = s_tr[f][ts][v][j];
        double hn;
        if (kind == kFineSide) {
          const int s0 = face_sub0(pk), s1 = face_sub1(pk);
          const int ms = DIM == 2 ? s0 : s0 + 2 * s1;
          hn = 0.0;
#pragma unroll 2
          for (int i = 0; i < NF; ++i) hn += Rm<DIM, N>(s_op, ms, i, j) * s_tw[f][0][v][i];
        } else {
          hn = s_tw[f][0][v][j];
        }
        Hb[v] = J[d] * lift_own * s_w[v][on] + s_jn[f][0] * lift_nb * hn;
      }
    }
    // the own trace is the left state on a +d face (side 1), the right state on a -d face
    double uL[NV], uR[NV], gL[NV], gR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uL[v] = side == 1 ? own[v] : oth[v];
      uR[v] = side == 1 ? oth[v] : own[v];
    }
    hll_flux_vjp<DIM>(uL, uR, d, gamma, Hb, gL, gR);
#pragma unroll
    for (int v = 0; v < NV; ++v) s_gf[f][sub][v][j] = side == 1 ? gL[v] : gR[v];
  };
  if (K::SPLIT) {
    if (lane < 64) {
      for (int w = lane; w < NP; w += 64) pair_vjp(w);
    } else {
      for (int r = lane - 64; r < NFI; r += T - 64) face_vjp(r);
    }
  } else {
    for (int w = lane; w < NP + NFI; w += T) {
      if (w < NP) pair_vjp(w);
      else face_vjp(w - NP);
    }
  }
  __syncthreads();

  // ---- E: per (variable, node): gather the pull-backs, stage-combination epilogue
  for (int w = lane; w < NV * ND; w += T) {
    const int v = w / ND, nd = w - v * ND;
    double g = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int line, pos;
      line_of<DIM, N>(nd, d, line, pos);
      const int base = (d * K::NLINE + line) * NPL;
      for (int mm = 0; mm < N; ++mm) {
        if (mm == pos) continue;
        g += mm > pos ? s_ga[base + pair_index<N>(pos, mm)][v] : s_gb[base + pair_index<N>(mm, pos)][v];
      }
      if (pos == 0 || pos == N - 1) {
        const int f = 2 * d + (pos == N - 1 ? 1 : 0);
        const int fi = face_index<DIM, N>(nd, d);
        if (face_kind(s_fk[f]) == kCoarseSide) {
          for (int ms = 0; ms < NSUB; ++ms) {
            const int m0 = ms & 1, m1 = (ms >> 1) & 1;
#pragma unroll 4
            for (int k = 0; k < NF; ++k) g += Pm<DIM, N>(s_op, m0, m1, k, fi) * s_gf[f][ms][v][k];
          }
        } else {
          g += s_gf[f][0][v][fi];
        }
      }
    }
    const int64_t idx = ((int64_t)v * ld + e) * ND + nd;
    if (a.Gout) a.Gout[idx] = g;
    if (a.Ubar) a.Ubar[idx] = (PRE ? pre_ubar : a.Ubar[idx]) + g;
    if (a.K1bar) a.K1bar[idx] = (PRE ? pre_k1bar : a.K1bar[idx]) + a.dt * a.A1[mem] * g;
    if (a.Kprev) a.Kprev[idx] = a.dt * (a.bprev * (PRE ? pre_lam : a.lam[idx]) + a.A2[mem] * g);
  }
}

// y = alpha x (n doubles), the start of the reverse sweep
__global__ void k_scale(double* y, const double* x, double alpha, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = alpha * x[i];
}

template <int DIM, int N>
hipError_t launch_vjp_t(const VjpArgs& a, const Mesh& m, const Ops& op, const Physics& ph, hipStream_t s) {
  const int blocks = a.n_act + a.n_halo;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_rhs_vjp<DIM, N>), dim3(blocks), dim3(AK<DIM, N>::T), 0, s, a, m, op, ph);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rhs_vjp(int dim, int N, const VjpArgs& a, const Mesh& m, const Ops& op, const Physics& ph,
                          hipStream_t s) {
  if (dim == 2 && N == 4) return launch_vjp_t<2, 4>(a, m, op, ph, s);
  if (dim == 2 && N == 3) return launch_vjp_t<2, 3>(a, m, op, ph, s);
  if (dim == 3 && N == 4) return launch_vjp_t<3, 4>(a, m, op, ph, s);
  if (dim == 3 && N == 3) return launch_vjp_t<3, 3>(a, m, op, ph, s);
  return hipErrorNotSupported;
}

hipError_t launch_scale(double* y, const double* x, double alpha, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n, 256)), dim3(256), 0, s, y, x, alpha, n);
  return hipGetLastError();
}

}  // namespace perk
