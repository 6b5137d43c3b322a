// Tangent of the Euler right-hand side on the GPU (gfx950): F'(u) v in forward mode, with every
// quantity carried as a (value, derivative) pair through the operator of the stage kernel --
// primitives, node logarithms, the entropy-conserving two-point flux, the HLL flux with Davis
// wave speeds, the 2:1 mortar interpolation and projection, lifting and the Jacobian factor.
// Branches (the logarithmic-mean series, the min / max of the wave speeds, the HLL cases) follow
// the values; at an exact tie of the min / max the first argument's derivative is taken.  One
// element per block of one wave.  Used by the spectrum estimation of Sec. 4.1 (products with the
// Jacobian at the real mesh) and checked against dual-number tangents.

#include "perk_device.h"

namespace perk {
namespace {

struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual dual_rcp(Dual a) {
  const double r = rcp(a.v);
  return {r, -a.d * r * r};
}
__device__ __forceinline__ Dual dual_log(Dual a) { return {log_pos(a.v), a.d * rcp(a.v)}; }
__device__ __forceinline__ Dual dual_sqrt(Dual a) {
  const double s = sqrt_pos(a.v);
  return {s, a.d * 0.5 * rcp(s)};
}
// ties take the first argument (its derivative), as the flux's own min / max does
__device__ __forceinline__ Dual dual_min(Dual a, Dual b) { return b.v < a.v ? b : a; }
__device__ __forceinline__ Dual dual_max(Dual a, Dual b) { return b.v > a.v ? b : a; }

template <int DIM>
struct DQ {
  Dual rho, v[DIM], p, lrho, beta, lbeta;
};

template <int DIM>
__device__ void dual_prim(const Dual* u, double gamma, Dual& rho, Dual* v, Dual& p) {
  rho = u[0];
  const Dual ir = dual_rcp(rho);
  Dual ke = {0.0, 0.0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    v[d] = u[1 + d] * ir;
    ke = ke + u[1 + d] * v[d];
  }
  p = (gamma - 1.0) * (u[DIM + 1] - 0.5 * ke);
}

// logarithmic mean (a - b)/(ln a - ln b): the series (a + b)/(2 F(f^2)), f = (a-b)/(a+b), where
// f^2 < 1e-2, else the quotient of the logarithms (the branch the value takes)
__device__ Dual dual_log_mean(Dual a, Dual b, Dual la, Dual lb) {
  const Dual dd = a - b, ss = a + b;
  if (dd.v * dd.v < 1e-2 * ss.v * ss.v) {
    const Dual f = dd * dual_rcp(ss);
    const Dual u = f * f;
    // 1/F(u) through u^7 (coefficients of the series inversion of F(u) = sum u^k/(2k+1))
    const double c[8] = {1.0, -1.0 / 3.0, -4.0 / 45.0, -44.0 / 945.0, -428.0 / 14175.0, -10196.0 / 467775.0,
                         -10719068.0 / 638512875.0, -25865068.0 / 1915538625.0};
    Dual s = {c[7], 0.0};
#pragma unroll
    for (int k = 6; k >= 0; --k) s = s * u + Dual{c[k], 0.0};
    return 0.5 * (ss * s);
  }
  return dd * dual_rcp(la - lb);
}

// 1 / logarithmic mean
__device__ Dual dual_inv_log_mean(Dual a, Dual b, Dual la, Dual lb) {
  const Dual dd = a - b, ss = a + b;
  if (dd.v * dd.v < 1e-2 * ss.v * ss.v) {
    const Dual iss = dual_rcp(ss);
    const Dual f = dd * iss;
    const Dual u = f * f;
    Dual s = {1.0 / 15.0, 0.0};
#pragma unroll
    for (int k = 6; k >= 0; --k) s = s * u + Dual{1.0 / (2 * k + 1), 0.0};
    return 2.0 * (s * iss);
  }
  return (la - lb) * dual_rcp(dd);
}

// the direction d differs from lane to lane: components along d are taken by selects (an
// indexed register array would live in scratch memory)
template <int DIM>
__device__ Dual along(const Dual* x, int d) {
  Dual r = x[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) r = k == d ? x[k] : r;
  return r;
}

template <int DIM>
__device__ void dual_ec_flux(const DQ<DIM>& L, const DQ<DIM>& R, int d, double inv_gm1, Dual* f) {
  const Dual rho_ln = dual_log_mean(L.rho, R.rho, L.lrho, R.lrho);
  const Dual ibeta_ln = dual_inv_log_mean(L.beta, R.beta, L.lbeta, R.lbeta);
  const Dual vdL = along<DIM>(L.v, d), vdR = along<DIM>(R.v, d);
  const Dual vd = 0.5 * (vdL + vdR);
  Dual vv = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) vv = vv + L.v[k] * R.v[k];
  const Dual fr = rho_ln * vd;
  const Dual pm = 0.5 * (L.p + R.p);
  f[0] = fr;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const Dual fk = fr * (0.5 * (L.v[k] + R.v[k]));
    f[1 + k] = k == d ? fk + pm : fk;
  }
  f[DIM + 1] = fr * (0.5 * vv + inv_gm1 * ibeta_ln) + 0.5 * (L.p * vdR + R.p * vdL);
}

template <int DIM>
__device__ void dual_hll(const Dual* uL, const Dual* uR, int d, double gamma, Dual* f) {
  Dual rl, vl[DIM], pl, rr, vr[DIM], pr;
  dual_prim<DIM>(uL, gamma, rl, vl, pl);
  dual_prim<DIM>(uR, gamma, rr, vr, pr);
  const Dual vnl = along<DIM>(vl, d), vnr = along<DIM>(vr, d);
  const Dual mnl = along<DIM>(uL + 1, d), mnr = along<DIM>(uR + 1, d);
  const Dual cl = dual_sqrt(gamma * (pl * dual_rcp(rl))), cr = dual_sqrt(gamma * (pr * dual_rcp(rr)));
  const Dual sl = dual_min(vnl - cl, vnr - cr);
  const Dual sr = dual_max(vnl + cl, vnr + cr);
  Dual fl[DIM + 2], fr[DIM + 2];
  fl[0] = mnl;
  fr[0] = mnr;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const Dual al = uL[1 + k] * vnl, ar = uR[1 + k] * vnr;
    fl[1 + k] = k == d ? al + pl : al;
    fr[1 + k] = k == d ? ar + pr : ar;
  }
  fl[DIM + 1] = (uL[DIM + 1] + pl) * vnl;
  fr[DIM + 1] = (uR[DIM + 1] + pr) * vnr;
  if (sl.v >= 0.0) {
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) f[v] = fl[v];
  } else if (sr.v <= 0.0) {
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) f[v] = fr[v];
  } else {
    const Dual inv = dual_rcp(sr - sl);
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) f[v] = (sr * fl[v] - sl * fr[v] + (sl * sr) * (uR[v] - uL[v])) * inv;
  }
}

template <int DIM, int N>
__global__ __launch_bounds__(64) void k_rhs_jvp(const double* __restrict__ U, const double* __restrict__ V,
                                                double* __restrict__ Tout, double* __restrict__ Fout, Mesh m, Ops op,
                                                Physics ph) {
  using g = G<DIM, N>;
  constexpr int ND = g::ND, NF = g::NF, NFC = g::NFC, NV = g::NV, NSUB = g::NSUB, T = 64;
  __shared__ Dual s_u[NV][ND];
  // neighbour traces (fine sides: the coarse trace interpolated into sub 1), then the numerical
  // fluxes on the (sub-)face nodes in place
  __shared__ Dual s_tr[NFC][NSUB][NV][NF];
  __shared__ Dual s_fc[NFC][NV][NF];         // face flux at the element's own face nodes
  __shared__ DQ<DIM> s_q[ND];
  __shared__ double s_op[6][N * N];          // 2 D (zero diagonal), D, P_0, P_1, R_0, R_1
  __shared__ int s_fk[NFC], s_fn[NFC][4];
  const int e = blockIdx.x;
  const int lane = threadIdx.x;
  const int ld = m.ld;
  const double gamma = ph.gamma, inv_gm1 = 1.0 / (gamma - 1.0);
  const int lev = m.lev[e];
  auto P = [&](int mm, int idx) { return s_op[2 + mm][idx]; };
  auto Rp = [&](int mm, int idx) { return s_op[4 + mm][idx]; };

  // ---- own state and tangent, connectivity, operator tables
  if (lane < NFC) s_fk[lane] = m.fk[(int64_t)e * NFC + lane];
  for (int t = lane; t < NFC * 4; t += T) s_fn[t / 4][t % 4] = m.fn[(int64_t)e * NFC * 4 + t];
  for (int t = lane; t < 6 * N * N; t += T) s_op[t / (N * N)][t % (N * N)] = op.dD[t];
  for (int w = lane; w < NV * ND; w += T) {
    const int v = w / ND, nd = w - v * ND;
    const int64_t idx = ((int64_t)v * ld + e) * ND + nd;
    s_u[v][nd] = Dual{U[idx], V[idx]};
  }
  __syncthreads();
  // ---- neighbour traces; node quantities
  for (int w = lane; w < NSUB * NFC * NV * NF; w += T) {
    const int j = w % NF, v = (w / NF) % NV, f = (w / (NF * NV)) % NFC, sub = w / (NF * NV * NFC);
    if (sub > 0 && face_kind(s_fk[f]) != kCoarseSide) continue;
    const int nb = s_fn[f][sub];
    const int d = f >> 1, side = f & 1;
    const int64_t idx = ((int64_t)v * ld + nb) * ND + face_node<DIM, N>(d, 1 - side, j);
    s_tr[f][sub][v][j] = Dual{U[idx], V[idx]};
  }
  for (int nd = lane; nd < ND; nd += T) {
    Dual uu[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uu[v] = s_u[v][nd];
    DQ<DIM> q;
    dual_prim<DIM>(uu, gamma, q.rho, q.v, q.p);
    q.lrho = dual_log(q.rho);
    q.beta = q.rho * dual_rcp(q.p);
    q.lbeta = dual_log(q.beta);
    s_q[nd] = q;
  }
  __syncthreads();
  // ---- fine sides: the coarse neighbour's trace interpolated to this sub-face
  for (int w = lane; w < NFC * NV * NF; w += T) {
    const int j = w % NF, v = (w / NF) % NV, f = w / (NF * NV);
    const int32_t pk = s_fk[f];
    if (face_kind(pk) != kFineSide) continue;
    const int s0 = face_sub0(pk), s1 = face_sub1(pk);
    Dual val = {0.0, 0.0};
    if (DIM == 2) {
      for (int k = 0; k < N; ++k) val = val + P(s0, j * N + k) * s_tr[f][0][v][k];
    } else {
      const int ja = j % N, jb = j / N;
      for (int kb = 0; kb < N; ++kb) {
        Dual row = {0.0, 0.0};
        for (int ka = 0; ka < N; ++ka) row = row + P(s0, ja * N + ka) * s_tr[f][0][v][ka + N * kb];
        val = val + P(s1, jb * N + kb) * row;
      }
    }
    s_tr[f][1][v][j] = val;
  }
  __syncthreads();
  // ---- numerical fluxes on every (sub-)face node
  for (int r = lane; r < NSUB * NFC * NF; r += T) {
    const int j = r % NF, f = (r / NF) % NFC, sub = r / (NF * NFC);
    const int kind = face_kind(s_fk[f]);
    if (sub > 0 && kind != kCoarseSide) continue;
    const int d = f >> 1, side = f & 1;
    Dual mine[NV], oth[NV], fl[NV];
    if (kind == kCoarseSide) {
      // own trace interpolated to sub-face `sub`
      const int m0 = sub & 1, m1 = (sub >> 1) & 1;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Dual x = {0.0, 0.0};
        if (DIM == 2) {
          for (int k = 0; k < N; ++k) x = x + P(m0, j * N + k) * s_u[v][face_node<DIM, N>(d, side, k)];
        } else {
          const int ja = j % N, jb = j / N;
          for (int kb = 0; kb < N; ++kb) {
            Dual row = {0.0, 0.0};
            for (int ka = 0; ka < N; ++ka)
              row = row + P(m0, ja * N + ka) * s_u[v][face_node<DIM, N>(d, side, ka + N * kb)];
            x = x + P(m1, jb * N + kb) * row;
          }
        }
        mine[v] = x;
        oth[v] = s_tr[f][sub][v][j];
      }
    } else {
      const int on = face_node<DIM, N>(d, side, j);
      const int ts = kind == kFineSide ? 1 : 0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        mine[v] = s_u[v][on];
        oth[v] = s_tr[f][ts][v][j];
      }
    }
    if (side == 1) dual_hll<DIM>(mine, oth, d, gamma, fl);
    else dual_hll<DIM>(oth, mine, d, gamma, fl);
#pragma unroll
    for (int v = 0; v < NV; ++v) s_tr[f][sub][v][j] = fl[v];
  }
  __syncthreads();
  // ---- coarse sides: sub-face fluxes projected back to the face nodes
  for (int w = lane; w < NFC * NV * NF; w += T) {
    const int i = w % NF, v = (w / NF) % NV, f = w / (NF * NV);
    if (face_kind(s_fk[f]) != kCoarseSide) {
      s_fc[f][v][i] = s_tr[f][0][v][i];
      continue;
    }
    Dual fs = {0.0, 0.0};
    if (DIM == 2) {
      for (int ms = 0; ms < 2; ++ms)
        for (int k = 0; k < N; ++k) fs = fs + Rp(ms, i * N + k) * s_tr[f][ms][v][k];
    } else {
      const int ia = i % N, ib = i / N;
      for (int ms = 0; ms < 4; ++ms) {
        const int m0 = ms & 1, m1 = (ms >> 1) & 1;
        for (int kb = 0; kb < N; ++kb) {
          Dual row = {0.0, 0.0};
          for (int ka = 0; ka < N; ++ka) row = row + Rp(m0, ia * N + ka) * s_tr[f][ms][v][ka + N * kb];
          fs = fs + Rp(m1, ib * N + kb) * row;
        }
      }
    }
    s_fc[f][v][i] = fs;
  }
  __syncthreads();
  // ---- per node: flux differencing along every direction, lifting, Jacobian factor
  const double iw0 = op.iw[0], iwN = op.iw[N - 1];
  for (int nd = lane; nd < ND; nd += T) {
    Dual du[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) du[v] = Dual{0.0, 0.0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int line, pos;
      line_of<DIM, N>(nd, d, line, pos);
      Dual acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = Dual{0.0, 0.0};
#pragma unroll
      for (int mm = 0; mm < N; ++mm) {
        if (mm == pos) continue;
        Dual f[NV];
        dual_ec_flux<DIM>(s_q[nd], s_q[node_on_line<DIM, N>(d, line, mm)], d, inv_gm1, f);
        const double c = s_op[0][pos * N + mm];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = acc[v] + c * f[v];
      }
      if (pos == N - 1 || pos == 0) {
        const int f = 2 * d + (pos == N - 1 ? 1 : 0);
        const int fi = face_index<DIM, N>(nd, d);
        const double lift = pos == N - 1 ? iwN : -iw0;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = acc[v] + lift * s_fc[f][v][fi];
      }
      const double J = m.jac[lev][d];
#pragma unroll
      for (int v = 0; v < NV; ++v) du[v] = du[v] - J * acc[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t idx = ((int64_t)v * ld + e) * ND + nd;
      Tout[idx] = du[v].d;
      if (Fout) Fout[idx] = du[v].v;
    }
  }
}

template <int DIM, int N>
hipError_t launch_jvp_t(int n, const double* U, const double* V, double* T, double* F, const Mesh& m, const Ops& op,
                        const Physics& ph, hipStream_t s) {
  hipLaunchKernelGGL((k_rhs_jvp<DIM, N>), dim3(n), dim3(64), 0, s, U, V, T, F, m, op, ph);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rhs_jvp(int dim, int N, int n, const double* U, const double* V, double* T, double* F,
                          const Mesh& m, const Ops& op, const Physics& ph, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dim == 2 && N == 4) return launch_jvp_t<2, 4>(n, U, V, T, F, m, op, ph, s);
  if (dim == 2 && N == 3) return launch_jvp_t<2, 3>(n, U, V, T, F, m, op, ph, s);
  if (dim == 3 && N == 4) return launch_jvp_t<3, 4>(n, U, V, T, F, m, op, ph, s);
  if (dim == 3 && N == 3) return launch_jvp_t<3, 3>(n, U, V, T, F, m, op, ph, s);
  return hipErrorNotSupported;
}

}  // namespace perk
