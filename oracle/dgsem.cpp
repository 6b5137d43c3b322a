// Oracle: serial DGSEM for the compressible Euler and Navier-Stokes equations on a periodic
// Cartesian forest of quad/octrees with 2:1 mortars, plus the dense masked partitioned RK step.
//
// TEST INFRASTRUCTURE ONLY.  Plain loops, fp64, no blocking, no fusion, no reordering beyond
// what each formula states.  Shares no code with the HIP library.
//
// Paper passages and readings followed (section / equation names of the paper):
//  * Conservation law u_t + div f(u, grad u) = 0, eq. (ConservationLaw), Sec. 1.
//  * DGSEM with flux differencing on Legendre-Gauss-Lobatto nodes (Sec. 6.1, citing Black,
//    Kopriva, Gassner-Winters-Kopriva).  Strong form per direction x (y, z alike):
//      du_i += -(2/h) [ sum_{m != i} 2 D_im f#(u_i, u_m) + delta_iN f*_E / w_N
//                       - delta_i0 f*_W / w_0 ]
//    which is the split form with the diagonal terms 2 D_NN f(u_N) = f(u_N)/w_N cancelled.
//  * Entropy-conserving two-point volume flux (Ranocha, cited in Sec. 4.1 and Sec. 7.2.1),
//    logarithmic means with a series branch for nearly equal arguments (the paper does not
//    say how the logarithmic mean is evaluated).
//  * HLL surface flux (Harten-Lax-van Leer) with Davis wave-speed estimates.
//  * Mortars for 2:1 non-conforming faces (Kopriva 1996, cited in Sec. 6.2): interpolate the
//    coarse trace to each fine sub-face, evaluate the flux there, project back with the L2
//    projection R_m = 1/2 M^{-1} B_m, M and B_m with exact integrals (tensor product, factor
//    1/4, in 3D).  Exact integrals make R_0 P_0 + R_1 P_1 = I (a coarse polynomial survives the
//    round trip); LGL quadrature in place of them would not, and would cost one order of the
//    truncation error at mortars.
//  * BR1 viscous terms (Bassi-Rebay, cited in Sec. 7.1): gradients of w = (v, T) with central
//    face values, viscous flux, divergence with the central average of the viscous flux.
//  * Subcell shock capturing (Hennemann, Rueda-Ramirez, Hindenlang, Gassner 2021, which the
//    paper uses for its inviscid runs: Sec. 4.1 and Sec. 7.2.1), optional, Euler: per element a
//    blending factor alpha from the modal energy of the density in the L2-orthonormal Legendre
//    basis (the share of the highest modes, E = max(E_1, E_2)), alpha = 1/(1 + exp(-s/T (E - T)))
//    with T = a 10^(-c (p+1)^(1/4)), s = ln((1 - 1e-4)/1e-4), set to 0 below alpha_min and capped
//    at alpha_max; the volume term becomes (1 - alpha) [flux differencing] + alpha [first-order
//    finite volumes on the LGL subcells: (F_{i+1/2} - F_{i-1/2}) / w_i, F = the HLL flux of the
//    neighbouring nodes, F = 0 at the element's own faces, whose flux the surface term brings].
//  * Partitioned RK step (eq. PartitionedRKSystem): K_i^(r) = I^(r) F(U_n + dt sum_j sum_k
//    a_ij^(k) K_j^(k)), U_{n+1} = U_n + dt sum_i b_i K_i.  Evaluated densely: F on the whole
//    mesh at every stage, every element combined with its own member's Butcher row.
//
// Layout of a state array: u[(e * nv + v) * Nd + node], node = i + N j (+ N^2 k), element
// order = order of the leaf list passed in.  Variables: rho, rho v_1..rho v_d, E.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

namespace {

// ------------------------------------------------------------------------------------------
// Forward-mode dual number v + d eps (eps^2 = 0): evaluating a function on duals yields its
// value and its derivative along the seeded direction, following the branches the value takes.
// Used only for the tangent-linear and adjoint checks of the Euler operator.
// ------------------------------------------------------------------------------------------
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() = default;
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
inline Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
inline bool operator<(Dual a, double b) { return a.v < b; }
inline bool operator>=(Dual a, double b) { return a.v >= b; }
inline bool operator<=(Dual a, double b) { return a.v <= b; }
inline Dual log(Dual a) { return {std::log(a.v), a.d / a.v}; }
inline Dual sqrt(Dual a) {
  const double r = std::sqrt(a.v);
  return {r, 0.5 * a.d / r};
}
inline Dual fmin(Dual a, Dual b) { return b.v < a.v ? b : a; }
inline Dual fmax(Dual a, Dual b) { return b.v > a.v ? b : a; }
using std::fmax;
using std::fmin;
using std::log;
using std::sqrt;
inline double value_of(double x) { return x; }
inline double value_of(Dual x) { return x.v; }

// ------------------------------------------------------------------------------------------
// Legendre-Gauss-Lobatto nodes and weights, Lagrange basis, differentiation matrix.
// ------------------------------------------------------------------------------------------
void legendre_and_derivative(int n, double x, double& P, double& dP) {
  // three-term recurrence for P_n and its derivative
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

// Nodes are -1, 1 and the roots of P'_p; weights 2 / (p (p+1) P_p(x)^2).
void lgl(int N, std::vector<double>& x, std::vector<double>& w) {
  const int p = N - 1;
  x.assign(N, 0.0);
  w.assign(N, 0.0);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int j = 1; j < p; ++j) {
    // Chebyshev-Gauss-Lobatto start, Newton on q(x) = P'_p(x) using
    // (1 - x^2) P''_p = 2 x P'_p - p (p+1) P_p.
    double xi = -std::cos(M_PI * j / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre_and_derivative(p, xi, P, dP);
      double d2P = (2.0 * xi * dP - p * (p + 1.0) * P) / (1.0 - xi * xi);
      double dx = dP / d2P;
      xi -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    x[j] = xi;
  }
  for (int j = 0; j < N; ++j) {
    double P, dP;
    if (j == 0 || j == p) {
      // P_p(+-1) = (+-1)^p
      P = (j == 0 && (p % 2 == 1)) ? -1.0 : 1.0;
    } else {
      legendre_and_derivative(p, x[j], P, dP);
    }
    w[j] = 2.0 / (p * (p + 1.0) * P * P);
  }
}

// Gauss-Legendre nodes and weights (n points, exact for degree 2n-1): roots of P_n by Newton
// from Chebyshev starts, weights 2 / ((1 - x^2) P'_n(x)^2).
void gauss_legendre(int n, std::vector<double>& g, std::vector<double>& gw) {
  g.assign(n, 0.0);
  gw.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double xi = -std::cos(M_PI * (j + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre_and_derivative(n, xi, P, dP);
      const double dx = P / dP;
      xi -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double P, dP;
    legendre_and_derivative(n, xi, P, dP);
    g[j] = xi;
    gw[j] = 2.0 / ((1.0 - xi * xi) * dP * dP);
  }
}

// Solve A X = B for X (A n x n, B n x m, row-major) by Gaussian elimination with partial pivoting.
std::vector<double> dense_solve(std::vector<double> A, std::vector<double> B, int n, int m) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
    for (int k = 0; k < m; ++k) std::swap(B[c * m + k], B[piv * m + k]);
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      for (int k = 0; k < m; ++k) B[r * m + k] -= f * B[c * m + k];
    }
  }
  for (int c = n - 1; c >= 0; --c)
    for (int k = 0; k < m; ++k) {
      double v = B[c * m + k];
      for (int j = c + 1; j < n; ++j) v -= A[c * n + j] * B[j * m + k];
      B[c * m + k] = v / A[c * n + c];
    }
  return B;
}

double lagrange(const std::vector<double>& x, int j, double xi) {
  double v = 1.0;
  for (size_t m = 0; m < x.size(); ++m)
    if ((int)m != j) v *= (xi - x[m]) / (x[j] - x[m]);
  return v;
}

// D_ij = l'_j(x_i) from the barycentric formula.
std::vector<double> diff_matrix(const std::vector<double>& x) {
  const int N = (int)x.size();
  std::vector<double> lam(N, 1.0), D(N * N, 0.0);
  for (int j = 0; j < N; ++j)
    for (int m = 0; m < N; ++m)
      if (m != j) lam[j] /= (x[j] - x[m]);
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int j = 0; j < N; ++j)
      if (j != i) {
        D[i * N + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
        s += D[i * N + j];
      }
    D[i * N + i] = -s;
  }
  return D;
}

// ------------------------------------------------------------------------------------------
// Physics
// ------------------------------------------------------------------------------------------
struct Phys {
  int dim;
  double gamma;
  double mu;      // dynamic viscosity (constant); 0 for Euler
  double kappa;   // heat conductivity gamma mu / ((gamma-1) Pr), gas constant 1
  bool viscous;
  int surface_ec;  // 0: HLL surface flux; 1: entropy-conserving flux on faces (entropy pin)
};

template <class T>
struct PrimT {
  T rho, v[3], p;
};
using Prim = PrimT<double>;

template <class T>
PrimT<T> cons2prim(const Phys& ph, const T* u) {
  PrimT<T> q;
  q.rho = u[0];
  T ke = 0.0;
  for (int d = 0; d < 3; ++d) q.v[d] = 0.0;
  for (int d = 0; d < ph.dim; ++d) {
    q.v[d] = u[1 + d] / u[0];
    ke += 0.5 * u[1 + d] * q.v[d];
  }
  q.p = (ph.gamma - 1.0) * (u[1 + ph.dim] - ke);
  return q;
}

// physical flux in direction d
template <class T>
void euler_flux(const Phys& ph, const T* u, int d, T* f) {
  PrimT<T> q = cons2prim(ph, u);
  const int nv = ph.dim + 2;
  f[0] = u[1 + d];
  for (int k = 0; k < ph.dim; ++k) f[1 + k] = u[1 + k] * q.v[d];
  f[1 + d] += q.p;
  f[nv - 1] = (u[nv - 1] + q.p) * q.v[d];
}

// logarithmic mean (b - a) / (ln b - ln a).  With f = (b-a)/(b+a), u = f^2 it equals
// (a+b) / (2 F(u)), F(u) = ln(b/a)/(2f) = sum_k u^k/(2k+1); for u < 1e-2 the series through
// u^7/15 is used (truncation below u^8/17 < 1e-17), so the logarithm is only evaluated where
// |ln(b/a)| > 0.2 and the quotient loses little to cancellation.
template <class T>
T log_mean(T a, T b) {
  T f = (b - a) / (b + a);
  T u = f * f;
  if (u < 1e-2) {
    T F = 1.0 + u / 3.0 + u * u / 5.0 + u * u * u / 7.0 + u * u * u * u / 9.0 +
          u * u * u * u * u / 11.0 + u * u * u * u * u * u / 13.0 + u * u * u * u * u * u * u / 15.0;
    return (a + b) / (2.0 * F);
  }
  return (b - a) / log(b / a);
}

// Entropy-conserving and kinetic-energy-preserving two-point flux (Ranocha), direction d:
//   f^rho = rho_ln {{v_d}},  f^{rho v_k} = f^rho {{v_k}} + {{p}} delta_kd,
//   f^E = f^rho (1/2 v_L . v_R + 1/((gamma-1) (rho/p)_ln)) + 1/2 (p_L v_{d,R} + p_R v_{d,L}).
template <class T>
void ec_flux(const Phys& ph, const T* uL, const T* uR, int d, T* f) {
  PrimT<T> L = cons2prim(ph, uL), R = cons2prim(ph, uR);
  const int nv = ph.dim + 2;
  T rho_ln = log_mean(L.rho, R.rho);
  T beta_ln = log_mean(L.rho / L.p, R.rho / R.p);
  T vd = 0.5 * (L.v[d] + R.v[d]);
  T p_avg = 0.5 * (L.p + R.p);
  T vLvR = 0.0;
  for (int k = 0; k < ph.dim; ++k) vLvR += L.v[k] * R.v[k];
  f[0] = rho_ln * vd;
  for (int k = 0; k < ph.dim; ++k) f[1 + k] = f[0] * 0.5 * (L.v[k] + R.v[k]);
  f[1 + d] += p_avg;
  f[nv - 1] = f[0] * (0.5 * vLvR + 1.0 / ((ph.gamma - 1.0) * beta_ln)) +
              0.5 * (L.p * R.v[d] + R.p * L.v[d]);
}

// Branches taken by the plain (double) HLL flux since the last reset: sL >= 0 (left state's
// flux), sR <= 0 (right state's flux), subsonic (HLL average).  For tests that must reach them.
static long long g_hll_branch[3] = {0, 0, 0};

// HLL flux with Davis wave speeds; normal +e_d from L to R.
template <class T>
void hll_flux(const Phys& ph, const T* uL, const T* uR, int d, T* f) {
  const int nv = ph.dim + 2;
  PrimT<T> L = cons2prim(ph, uL), R = cons2prim(ph, uR);
  T cL = sqrt(ph.gamma * L.p / L.rho);
  T cR = sqrt(ph.gamma * R.p / R.rho);
  T sL = fmin(L.v[d] - cL, R.v[d] - cR);
  T sR = fmax(L.v[d] + cL, R.v[d] + cR);
  T fL[5], fR[5];
  euler_flux(ph, uL, d, fL);
  euler_flux(ph, uR, d, fR);
  const int branch = sL >= 0.0 ? 0 : (sR <= 0.0 ? 1 : 2);
  if (std::is_same<T, double>::value) ++g_hll_branch[branch];
  if (branch == 0) {
    for (int v = 0; v < nv; ++v) f[v] = fL[v];
  } else if (branch == 1) {
    for (int v = 0; v < nv; ++v) f[v] = fR[v];
  } else {
    for (int v = 0; v < nv; ++v)
      f[v] = (sR * fL[v] - sL * fR[v] + sL * sR * (uR[v] - uL[v])) / (sR - sL);
  }
}

// Gradient variables of BR1: w = (v_1..v_d, T), T = p / rho (gas constant 1).
void grad_vars(const Phys& ph, const double* u, double* w) {
  Prim q = cons2prim(ph, u);
  for (int k = 0; k < ph.dim; ++k) w[k] = q.v[k];
  w[ph.dim] = q.p / q.rho;
}

// Viscous flux in direction d from w and its gradients g[dir][var] (var over w):
//   tau = mu (grad v + grad v^T) - 2/3 mu (div v) I,  F_v = (0, tau_{:,d}, tau_{:,d}.v + kappa dT/dx_d)
void viscous_flux(const Phys& ph, const double* w, const double (*g)[4], int d, double* f) {
  const int D = ph.dim;
  double divv = 0.0;
  for (int k = 0; k < D; ++k) divv += g[k][k];
  f[0] = 0.0;
  double e = 0.0;
  for (int k = 0; k < D; ++k) {
    double tau = ph.mu * (g[d][k] + g[k][d]);
    if (k == d) tau -= 2.0 / 3.0 * ph.mu * divv;
    f[1 + k] = tau;
    e += tau * w[k];
  }
  f[D + 1] = e + ph.kappa * g[d][D];
}

// ------------------------------------------------------------------------------------------
// Mesh: periodic Cartesian forest of n_root[d] trees per direction on [lo, hi].
// ------------------------------------------------------------------------------------------
enum FaceKind { CONFORMING = 0, FINE_SIDE = 1, COARSE_SIDE = 2 };

struct Face {
  int kind;
  int nbr[4];     // neighbour element(s): 1 for conforming / fine side, 2^{dim-1} for coarse side
  int sub[2];     // FINE_SIDE: position of this element's face on the coarse face per tangential axis
};

struct Solver {
  Phys ph;
  int dim, N, Nd, Nf, nv;
  int nroot[3];
  double lo[3], hi[3];
  std::vector<std::array<int, 4>> leaves;   // level, i, j, k
  std::map<std::array<int, 4>, int> index;
  std::vector<std::vector<Face>> faces;    // [e][2*dim]
  std::vector<double> x, w, D;
  std::vector<double> Pm[2];   // [j*N + i] = l_i(xi_j^m), xi^0 = (xi-1)/2, xi^1 = (xi+1)/2
  // [i*N + j]: L2 projection of the fine data on sub-face m back to the coarse face (Kopriva's
  // conservative mortars): with exact integrals, M R_m = 1/2 B_m, M_ik = int l_i l_k,
  // (B_m)_ij = int_{-1}^{1} l_i(xi^m(s)) l_j(s) ds
  std::vector<double> Rm[2];

  // subcell shock capturing (see the header); off unless set
  struct ShockCapturing {
    bool on = false;
    double alpha_max = 0.5, alpha_min = 0.001;
    double a = 0.5, c = 1.8;
    double alpha_fixed = -1.0;   // >= 0: every element takes this blending factor (checks)
  } sc;
  // [k*N + i]: coefficient of the k-th L2-orthonormal Legendre polynomial sqrt(k + 1/2) P_k of the
  // interpolant of nodal values f_i: sum_i Vinv[k][i] f_i (the inverse of the Vandermonde matrix
  // V[i][k] = sqrt(k + 1/2) P_k(x_i))
  std::vector<double> Vinv;

  int ncell(int level, int d) const { return nroot[d] << level; }
  double h(int e, int d) const { return (hi[d] - lo[d]) / ncell(leaves[e][0], d); }

  int find(int level, int i, int j, int k) const {
    if (level < 0) return -1;
    auto it = index.find({level, i, j, k});
    return it == index.end() ? -1 : it->second;
  }

  void build() {
    Nd = dim == 2 ? N * N : N * N * N;
    Nf = dim == 2 ? N : N * N;
    nv = dim + 2;
    lgl(N, x, w);
    D = diff_matrix(x);
    for (int m = 0; m < 2; ++m) {
      Pm[m].assign(N * N, 0.0);
      Rm[m].assign(N * N, 0.0);
      for (int j = 0; j < N; ++j) {
        double xi = m == 0 ? 0.5 * (x[j] - 1.0) : 0.5 * (x[j] + 1.0);
        for (int i = 0; i < N; ++i) Pm[m][j * N + i] = lagrange(x, i, xi);
      }
    }
    {
      // exact integrals of products of two degree-p polynomials: Gauss-Legendre with N points
      std::vector<double> g, gw;
      gauss_legendre(N, g, gw);
      std::vector<double> M(N * N, 0.0);
      for (int i = 0; i < N; ++i)
        for (int k = 0; k < N; ++k)
          for (int q = 0; q < N; ++q) M[i * N + k] += gw[q] * lagrange(x, i, g[q]) * lagrange(x, k, g[q]);
      for (int m = 0; m < 2; ++m) {
        std::vector<double> B(N * N, 0.0);
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j)
            for (int q = 0; q < N; ++q) {
              const double xi = m == 0 ? 0.5 * (g[q] - 1.0) : 0.5 * (g[q] + 1.0);
              B[i * N + j] += 0.5 * gw[q] * lagrange(x, i, xi) * lagrange(x, j, g[q]);
            }
        Rm[m] = dense_solve(M, B, N, N);
      }
    }
    {
      std::vector<double> V(N * N), I(N * N, 0.0);
      for (int i = 0; i < N; ++i) {
        for (int k = 0; k < N; ++k) {
          double P, dP;
          legendre_and_derivative(k, x[i], P, dP);
          V[i * N + k] = std::sqrt(k + 0.5) * P;
        }
        I[i * N + i] = 1.0;
      }
      Vinv = dense_solve(V, I, N, N);
    }
    index.clear();
    for (size_t e = 0; e < leaves.size(); ++e) {
      if (index.count(leaves[e])) throw std::runtime_error("duplicate leaf");
      index[leaves[e]] = (int)e;
    }
    faces.assign(leaves.size(), std::vector<Face>(2 * dim));
    for (size_t e = 0; e < leaves.size(); ++e) {
      const auto& L = leaves[e];
      int lev = L[0];
      for (int d = 0; d < dim; ++d)
        for (int s = 0; s < 2; ++s) {
          Face& F = faces[e][2 * d + s];
          int c[3] = {L[1], L[2], L[3]};
          c[d] += s ? 1 : -1;
          int n = ncell(lev, d);
          c[d] = (c[d] % n + n) % n;
          int same = find(lev, c[0], c[1], dim == 3 ? c[2] : 0);
          if (same >= 0) {
            F.kind = CONFORMING;
            F.nbr[0] = same;
            continue;
          }
          int parent = find(lev - 1, c[0] >> 1, c[1] >> 1, dim == 3 ? (c[2] >> 1) : 0);
          if (parent >= 0) {
            F.kind = FINE_SIDE;
            F.nbr[0] = parent;
            int t = 0;
            for (int a = 0; a < dim; ++a)
              if (a != d) F.sub[t++] = L[1 + a] & 1;
            continue;
          }
          // children of the same-level neighbour cell adjacent to this face
          F.kind = COARSE_SIDE;
          int tang[2], nt = 0;
          for (int a = 0; a < dim; ++a)
            if (a != d) tang[nt++] = a;
          int nsub = 1 << (dim - 1);
          for (int m = 0; m < nsub; ++m) {
            int cc[3] = {2 * c[0], 2 * c[1], dim == 3 ? 2 * c[2] : 0};
            cc[d] += s ? 0 : 1;   // the child touching this face
            cc[tang[0]] += m & 1;
            if (dim == 3) cc[tang[1]] += (m >> 1) & 1;
            int ch = find(lev + 1, cc[0], cc[1], dim == 3 ? cc[2] : 0);
            if (ch < 0) throw std::runtime_error("mesh is not 2:1 balanced or has a hole");
            F.nbr[m] = ch;
          }
        }
    }
  }

  // volume node index of face node (a, b) on face (d, s)
  int face_node(int d, int s, int a, int b) const {
    int side = s ? N - 1 : 0;
    if (dim == 2) return d == 0 ? side + N * a : a + N * side;
    if (d == 0) return side + N * a + N * N * b;
    if (d == 1) return a + N * side + N * N * b;
    return a + N * b + N * N * side;
  }

  // trace (all variables) of a nodal field with nvar components on face (d, s) of element e
  template <class T>
  void trace(const T* f, int nvar, int e, int d, int s, std::vector<T>& out) const {
    out.assign(nvar * Nf, T(0.0));
    int nb = dim == 3 ? N : 1;
    for (int b = 0; b < nb; ++b)
      for (int a = 0; a < N; ++a) {
        int nd = face_node(d, s, a, b);
        for (int v = 0; v < nvar; ++v) out[v * Nf + a + N * b] = f[((size_t)e * nvar + v) * Nd + nd];
      }
  }

  // interpolate a face field (nvar components) to sub-face (sub[0], sub[1]) with P_m
  template <class T>
  void to_subface(const std::vector<T>& in, int nvar, const int* sub, std::vector<T>& out) const {
    out.assign(nvar * Nf, T(0.0));
    if (dim == 2) {
      const auto& P = Pm[sub[0]];
      for (int v = 0; v < nvar; ++v)
        for (int j = 0; j < N; ++j) {
          T acc = 0.0;
          for (int i = 0; i < N; ++i) acc += P[j * N + i] * in[v * Nf + i];
          out[v * Nf + j] = acc;
        }
    } else {
      const auto& P1 = Pm[sub[0]];
      const auto& P2 = Pm[sub[1]];
      for (int v = 0; v < nvar; ++v)
        for (int j2 = 0; j2 < N; ++j2)
          for (int j1 = 0; j1 < N; ++j1) {
            T acc = 0.0;
            for (int i2 = 0; i2 < N; ++i2)
              for (int i1 = 0; i1 < N; ++i1)
                acc += P1[j1 * N + i1] * P2[j2 * N + i2] * in[v * Nf + i1 + N * i2];
            out[v * Nf + j1 + N * j2] = acc;
          }
    }
  }

  // project a sub-face field back to the coarse face with R_m and add
  template <class T>
  void add_projection(const std::vector<T>& in, int nvar, int m, std::vector<T>& acc) const {
    if (dim == 2) {
      const auto& R = Rm[m];
      for (int v = 0; v < nvar; ++v)
        for (int i = 0; i < N; ++i) {
          T s = 0.0;
          for (int j = 0; j < N; ++j) s += R[i * N + j] * in[v * Nf + j];
          acc[v * Nf + i] += s;
        }
    } else {
      const auto& R1 = Rm[m & 1];
      const auto& R2 = Rm[(m >> 1) & 1];
      for (int v = 0; v < nvar; ++v)
        for (int i2 = 0; i2 < N; ++i2)
          for (int i1 = 0; i1 < N; ++i1) {
            T s = 0.0;
            for (int j2 = 0; j2 < N; ++j2)
              for (int j1 = 0; j1 < N; ++j1)
                s += R1[i1 * N + j1] * R2[i2 * N + j2] * in[v * Nf + j1 + N * j2];
            acc[v * Nf + i1 + N * i2] += s;
          }
    }
  }

  // Numerical face values on face (d, s) of element e, as seen by e, for a two-sided rule
  // rule(left_values, right_values, d, out) applied node by node.  `field` holds nvar
  // components per node.  Conforming: rule on the shared nodes.  Fine side: the coarse trace
  // is interpolated to this sub-face.  Coarse side: rule on every sub-face, projected back.
  template <class T, class Rule>
  void face_values(const T* field, int nvar, int e, int d, int s, Rule rule, std::vector<T>& out) const {
    const Face& F = faces[e][2 * d + s];
    std::vector<T> mine, other, tmp, res(nvar * Nf);
    trace(field, nvar, e, d, s, mine);
    auto apply = [&](const std::vector<T>& own, const std::vector<T>& nb, std::vector<T>& r) {
      std::vector<T> a(nvar), b(nvar), o(nvar);
      for (int n = 0; n < Nf; ++n) {
        for (int v = 0; v < nvar; ++v) {
          a[v] = own[v * Nf + n];
          b[v] = nb[v * Nf + n];
        }
        if (s == 1) rule(a.data(), b.data(), d, o.data());   // this element is on the left
        else rule(b.data(), a.data(), d, o.data());
        for (int v = 0; v < nvar; ++v) r[v * Nf + n] = o[v];
      }
    };
    if (F.kind == CONFORMING) {
      trace(field, nvar, F.nbr[0], d, 1 - s, other);
      apply(mine, other, res);
      out = res;
    } else if (F.kind == FINE_SIDE) {
      trace(field, nvar, F.nbr[0], d, 1 - s, tmp);
      to_subface(tmp, nvar, F.sub, other);
      apply(mine, other, res);
      out = res;
    } else {
      out.assign(nvar * Nf, T(0.0));
      int nsub = 1 << (dim - 1);
      for (int m = 0; m < nsub; ++m) {
        int sub[2] = {m & 1, (m >> 1) & 1};
        std::vector<T> mine_m;
        to_subface(mine, nvar, sub, mine_m);
        trace(field, nvar, F.nbr[m], d, 1 - s, other);
        apply(mine_m, other, res);
        add_projection(res, nvar, m, out);
      }
    }
  }

  void node_ijk(int nd, int* ijk) const {
    ijk[0] = nd % N;
    ijk[1] = (nd / N) % N;
    ijk[2] = dim == 3 ? nd / (N * N) : 0;
  }
  int node_of(const int* ijk) const {
    return dim == 2 ? ijk[0] + N * ijk[1] : ijk[0] + N * ijk[1] + N * N * ijk[2];
  }

  // share of the highest modes in the density's modal energy on element e:
  // E = max((total - clip_1) / total, (clip_1 - clip_2) / clip_1), clip_k the energy of the modes
  // whose degree in every direction is at most p - k
  double sc_energy(const double* u, size_t e) const {
    const int p = N - 1;
    const int nc = dim == 3 ? N : 1;
    double total = 0.0, clip1 = 0.0, clip2 = 0.0;
    for (int c3 = 0; c3 < nc; ++c3)
      for (int b = 0; b < N; ++b)
        for (int a = 0; a < N; ++a) {
          double m = 0.0;
          for (int k = 0; k < nc; ++k)
            for (int j = 0; j < N; ++j)
              for (int i = 0; i < N; ++i) {
                const double vk = dim == 3 ? Vinv[c3 * N + k] : 1.0;
                const int nd = dim == 3 ? i + N * j + N * N * k : i + N * j;
                m += Vinv[a * N + i] * Vinv[b * N + j] * vk * u[(e * nv + 0) * Nd + nd];
              }
          const double m2 = m * m;
          const int deg = std::max(a, std::max(b, c3));
          total += m2;
          if (deg <= p - 1) clip1 += m2;
          if (deg <= p - 2) clip2 += m2;
        }
    const double e1 = total > 0.0 ? (total - clip1) / total : 0.0;
    const double e2 = clip1 > 0.0 ? (clip1 - clip2) / clip1 : 0.0;
    return std::max(e1, e2);
  }

  double sc_alpha_of_energy(double E) const {
    const double T = sc.a * std::pow(10.0, -sc.c * std::pow((double)N, 0.25));
    const double s = std::log((1.0 - 1e-4) / 1e-4);
    double alpha = 1.0 / (1.0 + std::exp(-s / T * (E - T)));
    if (alpha < sc.alpha_min) return 0.0;
    return std::min(alpha, sc.alpha_max);
  }

  double sc_alpha(const double* u, size_t e) const {
    if (!sc.on) return 0.0;
    if (sc.alpha_fixed >= 0.0) return sc.alpha_fixed;
    return sc_alpha_of_energy(sc_energy(u, e));
  }

  // inviscid part of du = F(u): volume flux differencing and surface flux (scalar type T:
  // double, or Dual for the tangent of the Euler operator, which has no shock capturing)
  template <class T>
  void rhs_inviscid(const T* u, T* du) const {
    const size_t ne = leaves.size();
    for (size_t q = 0; q < ne * nv * Nd; ++q) du[q] = 0.0;
    for (size_t e = 0; e < ne; ++e) {
      double alpha = 0.0;
      if constexpr (std::is_same<T, double>::value) alpha = sc_alpha(u, e);
      for (int d = 0; d < dim; ++d) {
        double J = 2.0 / h((int)e, d);
        for (int nd = 0; nd < Nd; ++nd) {
          int ijk[3];
          node_ijk(nd, ijk);
          int a = ijk[d];
          T ui[5], um[5], f[5];
          for (int v = 0; v < nv; ++v) ui[v] = u[(e * nv + v) * Nd + nd];
          for (int m = 0; m < N; ++m) {
            if (m == a) continue;
            int jk[3] = {ijk[0], ijk[1], ijk[2]};
            jk[d] = m;
            int n2 = node_of(jk);
            for (int v = 0; v < nv; ++v) um[v] = u[(e * nv + v) * Nd + n2];
            ec_flux(ph, ui, um, d, f);
            for (int v = 0; v < nv; ++v) du[(e * nv + v) * Nd + nd] -= J * (1.0 - alpha) * 2.0 * D[a * N + m] * f[v];
          }
          if (alpha > 0.0) {
            // first-order finite volumes on the LGL subcells: subcell interfaces between the
            // node and its neighbours along d; none at the element's own faces
            T fp[5], fm[5];
            for (int v = 0; v < nv; ++v) fp[v] = fm[v] = 0.0;
            for (int side = 0; side < 2; ++side) {
              const int m = side ? a + 1 : a - 1;
              if (m < 0 || m >= N) continue;
              int jk[3] = {ijk[0], ijk[1], ijk[2]};
              jk[d] = m;
              const int n2 = node_of(jk);
              for (int v = 0; v < nv; ++v) um[v] = u[(e * nv + v) * Nd + n2];
              if (side) hll_flux(ph, ui, um, d, fp);
              else hll_flux(ph, um, ui, d, fm);
            }
            for (int v = 0; v < nv; ++v) du[(e * nv + v) * Nd + nd] -= J * alpha * (fp[v] - fm[v]) / w[a];
          }
        }
        for (int s = 0; s < 2; ++s) {
          std::vector<T> fs;
          face_values(u, nv, (int)e, d, s,
                      [&](const T* L, const T* R, int dd, T* o) {
                        if (ph.surface_ec) ec_flux(ph, L, R, dd, o);
                        else hll_flux(ph, L, R, dd, o);
                      },
                      fs);
          int nb = dim == 3 ? N : 1;
          for (int b = 0; b < nb; ++b)
            for (int a2 = 0; a2 < N; ++a2) {
              int nd = face_node(d, s, a2, b);
              for (int v = 0; v < nv; ++v) {
                T val = fs[v * Nf + a2 + N * b];
                if (s == 1) du[(e * nv + v) * Nd + nd] -= J * val / w[N - 1];
                else du[(e * nv + v) * Nd + nd] += J * val / w[0];
              }
            }
        }
      }
    }
  }

  // du = F(u)
  void rhs(const double* u, double* du) const {
    const size_t ne = leaves.size();
    rhs_inviscid(u, du);
    if (!ph.viscous) return;
    // ---- BR1: gradients of w, viscous flux, divergence
    const int nw = dim + 1;
    std::vector<double> W(ne * nw * Nd), G((size_t)dim * ne * nw * Nd, 0.0);
    for (size_t e = 0; e < ne; ++e)
      for (int nd = 0; nd < Nd; ++nd) {
        double ue[5], we[4];
        for (int v = 0; v < nv; ++v) ue[v] = u[(e * nv + v) * Nd + nd];
        grad_vars(ph, ue, we);
        for (int v = 0; v < nw; ++v) W[(e * nw + v) * Nd + nd] = we[v];
      }
    auto central = [&](const double* L, const double* R, int, double* o) {
      for (int v = 0; v < nw; ++v) o[v] = 0.5 * (L[v] + R[v]);
    };
    for (size_t e = 0; e < ne; ++e)
      for (int d = 0; d < dim; ++d) {
        double J = 2.0 / h((int)e, d);
        double* g = &G[((size_t)d * ne) * nw * Nd];
        for (int nd = 0; nd < Nd; ++nd) {
          int ijk[3];
          node_ijk(nd, ijk);
          for (int v = 0; v < nw; ++v) {
            double acc = 0.0;
            for (int m = 0; m < N; ++m) {
              int jk[3] = {ijk[0], ijk[1], ijk[2]};
              jk[d] = m;
              acc += D[ijk[d] * N + m] * W[(e * nw + v) * Nd + node_of(jk)];
            }
            g[(e * nw + v) * Nd + nd] += J * acc;
          }
        }
        for (int s = 0; s < 2; ++s) {
          std::vector<double> ws;
          face_values(W.data(), nw, (int)e, d, s, central, ws);
          int nb = dim == 3 ? N : 1;
          for (int b = 0; b < nb; ++b)
            for (int a2 = 0; a2 < N; ++a2) {
              int nd = face_node(d, s, a2, b);
              for (int v = 0; v < nw; ++v) {
                double jump = ws[v * Nf + a2 + N * b] - W[(e * nw + v) * Nd + nd];
                if (s == 1) g[(e * nw + v) * Nd + nd] += J * jump / w[N - 1];
                else g[(e * nw + v) * Nd + nd] -= J * jump / w[0];
              }
            }
        }
      }
    // viscous flux at every node, per direction: Fv[d][e][v][node]
    std::vector<double> Fv((size_t)dim * ne * nv * Nd);
    for (size_t e = 0; e < ne; ++e)
      for (int nd = 0; nd < Nd; ++nd) {
        double we[4], gg[3][4];
        for (int v = 0; v < nw; ++v) we[v] = W[(e * nw + v) * Nd + nd];
        for (int d = 0; d < dim; ++d)
          for (int v = 0; v < nw; ++v) gg[d][v] = G[(((size_t)d * ne + e) * nw + v) * Nd + nd];
        for (int d = 0; d < dim; ++d) {
          double f[5];
          viscous_flux(ph, we, gg, d, f);
          for (int v = 0; v < nv; ++v) Fv[(((size_t)d * ne + e) * nv + v) * Nd + nd] = f[v];
        }
      }
    auto central_u = [&](const double* L, const double* R, int, double* o) {
      for (int v = 0; v < nv; ++v) o[v] = 0.5 * (L[v] + R[v]);
    };
    for (size_t e = 0; e < ne; ++e)
      for (int d = 0; d < dim; ++d) {
        double J = 2.0 / h((int)e, d);
        const double* fv = &Fv[((size_t)d * ne) * nv * Nd];
        for (int nd = 0; nd < Nd; ++nd) {
          int ijk[3];
          node_ijk(nd, ijk);
          for (int v = 0; v < nv; ++v) {
            double acc = 0.0;
            for (int m = 0; m < N; ++m) {
              int jk[3] = {ijk[0], ijk[1], ijk[2]};
              jk[d] = m;
              acc += D[ijk[d] * N + m] * fv[(e * nv + v) * Nd + node_of(jk)];
            }
            du[(e * nv + v) * Nd + nd] += J * acc;
          }
        }
        for (int s = 0; s < 2; ++s) {
          std::vector<double> fs;
          face_values(fv, nv, (int)e, d, s, central_u, fs);
          int nb = dim == 3 ? N : 1;
          for (int b = 0; b < nb; ++b)
            for (int a2 = 0; a2 < N; ++a2) {
              int nd = face_node(d, s, a2, b);
              for (int v = 0; v < nv; ++v) {
                double jump = fs[v * Nf + a2 + N * b] - fv[(e * nv + v) * Nd + nd];
                if (s == 1) du[(e * nv + v) * Nd + nd] += J * jump / w[N - 1];
                else du[(e * nv + v) * Nd + nd] -= J * jump / w[0];
              }
            }
        }
      }
  }
};

thread_local std::string g_err;

}  // namespace

extern "C" {

const char* orc_last_error() { return g_err.c_str(); }

// leaves: n_leaves x 4 int32 (level, i, j, k); k ignored in 2D.
void* orc_create(int dim, int N, int viscous, int surface_ec, double gamma, double mu,
                 double prandtl, const int* nroot, const double* lo, const double* hi, int n_leaves,
                 const int32_t* leaves) {
  try {
    Solver* s = new Solver();
    s->dim = dim;
    s->N = N;
    s->ph.dim = dim;
    s->ph.gamma = gamma;
    s->ph.viscous = viscous != 0;
    s->ph.surface_ec = surface_ec;
    s->ph.mu = viscous ? mu : 0.0;
    s->ph.kappa = viscous ? gamma * mu / ((gamma - 1.0) * prandtl) : 0.0;
    for (int d = 0; d < 3; ++d) {
      s->nroot[d] = d < dim ? nroot[d] : 1;
      s->lo[d] = d < dim ? lo[d] : 0.0;
      s->hi[d] = d < dim ? hi[d] : 1.0;
    }
    s->leaves.resize(n_leaves);
    for (int e = 0; e < n_leaves; ++e)
      s->leaves[e] = {leaves[4 * e], leaves[4 * e + 1], leaves[4 * e + 2], dim == 3 ? leaves[4 * e + 3] : 0};
    s->build();
    return s;
  } catch (const std::exception& ex) {
    g_err = ex.what();
    return nullptr;
  }
}

void orc_destroy(void* h) { delete static_cast<Solver*>(h); }

int orc_sizes(void* h, int* out) {
  Solver* s = static_cast<Solver*>(h);
  out[0] = (int)s->leaves.size();
  out[1] = s->nv;
  out[2] = s->Nd;
  return 0;
}

void orc_rhs(void* h, const double* u, double* du) { static_cast<Solver*>(h)->rhs(u, du); }

// physical coordinates of all nodes: x[(e*dim + d)*Nd + node]
void orc_node_coords(void* h, double* xout) {
  Solver* s = static_cast<Solver*>(h);
  for (size_t e = 0; e < s->leaves.size(); ++e)
    for (int nd = 0; nd < s->Nd; ++nd) {
      int ijk[3];
      s->node_ijk(nd, ijk);
      for (int d = 0; d < s->dim; ++d) {
        double hd = s->h((int)e, d);
        double x0 = s->lo[d] + hd * s->leaves[e][1 + d];
        xout[(e * s->dim + d) * s->Nd + nd] = x0 + 0.5 * hd * (1.0 + s->x[ijk[d]]);
      }
    }
}

void orc_lgl(int N, double* x, double* w, double* D) {
  std::vector<double> xx, ww;
  lgl(N, xx, ww);
  auto DD = diff_matrix(xx);
  for (int i = 0; i < N; ++i) {
    x[i] = xx[i];
    w[i] = ww[i];
  }
  for (int i = 0; i < N * N; ++i) D[i] = DD[i];
}

void orc_mortar_ops(void* h, double* P0, double* P1, double* R0, double* R1) {
  Solver* s = static_cast<Solver*>(h);
  for (int i = 0; i < s->N * s->N; ++i) {
    P0[i] = s->Pm[0][i];
    P1[i] = s->Pm[1][i];
    R0[i] = s->Rm[0][i];
    R1[i] = s->Rm[1][i];
  }
}

void orc_ec_flux(int dim, double gamma, const double* uL, const double* uR, int d, double* f) {
  Phys ph{dim, gamma, 0.0, 0.0, false, 0};
  ec_flux(ph, uL, uR, d, f);
}
void orc_hll_flux(int dim, double gamma, const double* uL, const double* uR, int d, double* f) {
  Phys ph{dim, gamma, 0.0, 0.0, false, 0};
  hll_flux(ph, uL, uR, d, f);
}
void orc_euler_flux(int dim, double gamma, const double* u, int d, double* f) {
  Phys ph{dim, gamma, 0.0, 0.0, false, 0};
  euler_flux(ph, u, d, f);
}
double orc_log_mean(double a, double b) { return log_mean(a, b); }
void orc_hll_branch_counts(long long* out, int reset) {
  for (int k = 0; k < 3; ++k) {
    if (out) out[k] = g_hll_branch[k];
    if (reset) g_hll_branch[k] = 0;
  }
}

// Face kinds for inspection: kinds[e*2dim + f], nbrs[(e*2dim + f)*4 + m]
void orc_faces(void* h, int32_t* kinds, int32_t* nbrs) {
  Solver* s = static_cast<Solver*>(h);
  int nf = 2 * s->dim;
  for (size_t e = 0; e < s->leaves.size(); ++e)
    for (int f = 0; f < nf; ++f) {
      const Face& F = s->faces[e][f];
      kinds[e * nf + f] = F.kind;
      for (int m = 0; m < 4; ++m) nbrs[(e * nf + f) * 4 + m] = (F.kind == COARSE_SIDE || m == 0) ? F.nbr[m] : -1;
      if (F.kind == COARSE_SIDE && s->dim == 2)
        for (int m = 2; m < 4; ++m) nbrs[(e * nf + f) * 4 + m] = -1;
    }
}

// One partitioned RK step, dense form (eq. PartitionedRKSystem) with masks from member[e].
// A: R x S x S full Butcher matrices, b: S shared weights (eq. Conservation), c unused
// (autonomous problem).  u is overwritten with U_{n+1}.  Returns 0 on success.
int orc_prk_step(void* h, double* u, double dt, int R, int S, const double* A, const double* b,
                 const int32_t* member) {
  Solver* s = static_cast<Solver*>(h);
  const size_t ne = s->leaves.size();
  const size_t n = ne * s->nv * s->Nd;
  const size_t per = (size_t)s->nv * s->Nd;
  for (size_t e = 0; e < ne; ++e)
    if (member[e] < 0 || member[e] >= R) {
      g_err = "member index out of range";
      return -1;
    }
  std::vector<std::vector<double>> K(S, std::vector<double>(n));
  std::vector<double> Y(n);
  for (int i = 0; i < S; ++i) {
    for (size_t e = 0; e < ne; ++e) {
      const double* Ar = A + (size_t)member[e] * S * S;
      for (size_t q = 0; q < per; ++q) {
        size_t idx = e * per + q;
        double acc = 0.0;
        for (int j = 0; j < i; ++j) acc += Ar[i * S + j] * K[j][idx];
        Y[idx] = u[idx] + dt * acc;
      }
    }
    s->rhs(Y.data(), K[i].data());
  }
  for (size_t idx = 0; idx < n; ++idx) {
    double acc = 0.0;
    for (int i = 0; i < S; ++i) acc += b[i] * K[i][idx];
    u[idx] += dt * acc;
  }
  return 0;
}

}  // extern "C"

extern "C" {
// Plain explicit RK step with a full S x S Butcher matrix (no partitioning), for the
// single-level comparisons: Y_i = U + dt sum_{j<i} A_ij K_j, K_i = F(Y_i), U += dt sum b_i K_i.
int orc_rk_step(void* h, double* u, double dt, int S, const double* A, const double* b) {
  Solver* s = static_cast<Solver*>(h);
  const size_t n = s->leaves.size() * (size_t)s->nv * s->Nd;
  std::vector<std::vector<double>> K(S, std::vector<double>(n));
  std::vector<double> Y(n);
  for (int i = 0; i < S; ++i) {
    for (size_t q = 0; q < n; ++q) {
      double acc = 0.0;
      for (int j = 0; j < i; ++j) acc += A[i * S + j] * K[j][q];
      Y[q] = u[q] + dt * acc;
    }
    s->rhs(Y.data(), K[i].data());
  }
  for (size_t q = 0; q < n; ++q) {
    double acc = 0.0;
    for (int i = 0; i < S; ++i) acc += b[i] * K[i][q];
    u[q] += dt * acc;
  }
  return 0;
}
}

// ------------------------------------------------------------------------------------------
// Tangent-linear and adjoint of the Euler operator and of the partitioned RK step.
//
// The discrete adjoint of a map G is G'(u)^T.  Here G' is formed column by column from the
// forward-mode dual evaluation of G itself (the exact derivative of the computed map, each
// branch taken as the value takes it), and the adjoint applied to lam is the vector of
// <lam, G'(u) e_j>.  Dense and slow (one dual evaluation per unknown): for small meshes only.
// ------------------------------------------------------------------------------------------
namespace {

template <class T>
void prk_step_t(const Solver* s, T* u, double dt, int R, int S, const double* A, const double* b,
                const int32_t* member) {
  const size_t ne = s->leaves.size();
  const size_t n = ne * s->nv * s->Nd;
  const size_t per = (size_t)s->nv * s->Nd;
  std::vector<std::vector<T>> K(S, std::vector<T>(n));
  std::vector<T> Y(n);
  for (int i = 0; i < S; ++i) {
    for (size_t e = 0; e < ne; ++e) {
      const double* Ar = A + (size_t)member[e] * S * S;
      for (size_t q = 0; q < per; ++q) {
        size_t idx = e * per + q;
        T acc = 0.0;
        for (int j = 0; j < i; ++j) acc += Ar[i * S + j] * K[j][idx];
        Y[idx] = u[idx] + dt * acc;
      }
    }
    s->rhs_inviscid(Y.data(), K[i].data());
  }
  for (size_t idx = 0; idx < n; ++idx) {
    T acc = 0.0;
    for (int i = 0; i < S; ++i) acc += b[i] * K[i][idx];
    u[idx] += dt * acc;
  }
}

bool check_euler(const Solver* s) {
  if (s->ph.viscous) {
    g_err = "tangent and adjoint: Euler operator only";
    return false;
  }
  if (s->sc.on) {
    g_err = "tangent and adjoint: not with shock capturing";
    return false;
  }
  return true;
}

}  // namespace

extern "C" {

// Subcell shock capturing: on != 0 switches it on with the given parameters; alpha_fixed >= 0
// gives every element that blending factor instead of the indicator's (checks).  Euler only.
int orc_set_shock_capturing(void* h, int on, double alpha_max, double alpha_min, double alpha_fixed) {
  Solver* s = static_cast<Solver*>(h);
  if (on && s->ph.viscous) {
    g_err = "shock capturing: Euler only";
    return -1;
  }
  s->sc.on = on != 0;
  s->sc.alpha_max = alpha_max;
  s->sc.alpha_min = alpha_min;
  s->sc.alpha_fixed = alpha_fixed;
  return 0;
}

// Per element: the modal energy share E of the density and the blending factor alpha of the
// current parameters (alpha regardless of whether shock capturing is on); Vinv [N*N] if not null.
int orc_sc_indicator(void* h, const double* u, double* energy, double* alpha, double* vinv) {
  Solver* s = static_cast<Solver*>(h);
  for (size_t e = 0; e < s->leaves.size(); ++e) {
    const double E = s->sc_energy(u, e);
    if (energy) energy[e] = E;
    if (alpha) alpha[e] = s->sc.alpha_fixed >= 0.0 ? s->sc.alpha_fixed : s->sc_alpha_of_energy(E);
  }
  if (vinv)
    for (int i = 0; i < s->N * s->N; ++i) vinv[i] = s->Vinv[i];
  return 0;
}

// f = F(u) and t = F'(u) du (Euler)
int orc_rhs_jvp(void* h, const double* u, const double* du, double* f, double* t) {
  const Solver* s = static_cast<Solver*>(h);
  if (!check_euler(s)) return -1;
  const size_t n = s->leaves.size() * (size_t)s->nv * s->Nd;
  std::vector<Dual> x(n), y(n);
  for (size_t q = 0; q < n; ++q) x[q] = Dual(u[q], du[q]);
  s->rhs_inviscid(x.data(), y.data());
  for (size_t q = 0; q < n; ++q) {
    if (f) f[q] = y[q].v;
    t[q] = y[q].d;
  }
  return 0;
}

// out = F'(u)^T w (Euler), column by column
int orc_rhs_vjp(void* h, const double* u, const double* w, double* out) {
  const Solver* s = static_cast<Solver*>(h);
  if (!check_euler(s)) return -1;
  const size_t n = s->leaves.size() * (size_t)s->nv * s->Nd;
  std::vector<Dual> x(n), y(n);
  for (size_t j = 0; j < n; ++j) {
    for (size_t q = 0; q < n; ++q) x[q] = Dual(u[q], q == j ? 1.0 : 0.0);
    s->rhs_inviscid(x.data(), y.data());
    double acc = 0.0;
    for (size_t q = 0; q < n; ++q) acc += w[q] * y[q].d;
    out[j] = acc;
  }
  return 0;
}

// One dense masked partitioned RK step on duals: u_out = Phi(u), t_out = Phi'(u) du (Euler)
int orc_prk_step_jvp(void* h, const double* u, const double* du, double dt, int R, int S, const double* A,
                     const double* b, const int32_t* member, double* u_out, double* t_out) {
  const Solver* s = static_cast<Solver*>(h);
  if (!check_euler(s)) return -1;
  const size_t ne = s->leaves.size();
  for (size_t e = 0; e < ne; ++e)
    if (member[e] < 0 || member[e] >= R) {
      g_err = "member index out of range";
      return -1;
    }
  const size_t n = ne * (size_t)s->nv * s->Nd;
  std::vector<Dual> x(n);
  for (size_t q = 0; q < n; ++q) x[q] = Dual(u[q], du[q]);
  prk_step_t(s, x.data(), dt, R, S, A, b, member);
  for (size_t q = 0; q < n; ++q) {
    if (u_out) u_out[q] = x[q].v;
    t_out[q] = x[q].d;
  }
  return 0;
}

// out = Phi'(u)^T lam for one partitioned RK step (Euler), column by column
int orc_prk_step_vjp(void* h, const double* u, const double* lam, double dt, int R, int S, const double* A,
                     const double* b, const int32_t* member, double* out) {
  const Solver* s = static_cast<Solver*>(h);
  if (!check_euler(s)) return -1;
  const size_t ne = s->leaves.size();
  for (size_t e = 0; e < ne; ++e)
    if (member[e] < 0 || member[e] >= R) {
      g_err = "member index out of range";
      return -1;
    }
  const size_t n = ne * (size_t)s->nv * s->Nd;
  std::vector<Dual> x(n);
  for (size_t j = 0; j < n; ++j) {
    for (size_t q = 0; q < n; ++q) x[q] = Dual(u[q], q == j ? 1.0 : 0.0);
    prk_step_t(s, x.data(), dt, R, S, A, b, member);
    double acc = 0.0;
    for (size_t q = 0; q < n; ++q) acc += lam[q] * x[q].d;
    out[j] = acc;
  }
  return 0;
}

}  // extern "C"
