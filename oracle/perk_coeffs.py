"""Oracle: P-ERK Butcher tableaux, their stability polynomials and order conditions.

Test infrastructure only (see oracle/__init__.py).  Everything here is fp64 numpy/scipy.

Paper passages followed
  * Partitioned RK in Butcher form, eq. (PartitionedRKSystem), Sec. 2.
  * Order conditions for shared b and c, eq. (PRKOrderCondsSimplified), Sec. 2.1.
  * Internal consistency, eq. (InternalConsistency), Sec. 2.3; shared b, eq. (Conservation).
  * Second-order P-ERK tableau structure, eq. (PERK_ButcherTableauClassic), Sec. 3.1;
    abscissae shown by example there (c_i = (i-1)/10 for S=6) and in the S=16 table
    eq. (PERK_8_16_CompactForm): c_i = (i-1)/(2(S-1)), b = e_S.
  * Third-order base scheme (Shu-Osher), eq. (PERK_ThirdOrderShuOsher), and the free
    abscissae c_i = (i-1)/(S-3), i <= S-2, eq. (Free_Timesteps), Sec. 3.3.
  * Stability polynomial of a tableau P(z) = 1 + z b^T (I - zA)^{-1} 1, Sec. 4.3.
  * Monomial form of P_{p;E}, Sec. 4.3; second-order construction eq. (PERKCoeffsConstruction);
    third-order construction by a nonlinear solve with the 1/6 constraint and positivity, Sec. 4.3.2.
  * Optimisation problem eq. (OptimizationProblem), Sec. 4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------------------
# Tableau container.  a_sub[i] is a_{i,i-1} (0-based row i, so a_sub[0] = a_sub[1] = 0);
# a_{i,1} = c_i - a_{i,i-1} by internal consistency.
# ----------------------------------------------------------------------------------------
@dataclass
class PerkFamily:
    order: int
    S: int
    E: list                      # stage evaluations per member, ascending
    c: np.ndarray                # [S]
    b: np.ndarray                # [S]
    a_sub: np.ndarray            # [R, S]
    alpha: list = field(default_factory=list)   # optimised monomial coefficients per member

    def to_json(self):
        return {"order": self.order, "S": self.S, "E": list(map(int, self.E)),
                "c": [float(x) for x in self.c], "b": [float(x) for x in self.b],
                "a_sub": [[float(x) for x in row] for row in self.a_sub]}

    @staticmethod
    def from_json(d):
        return PerkFamily(d["order"], d["S"], list(d["E"]), np.array(d["c"], float),
                          np.array(d["b"], float), np.array(d["a_sub"], float))


def perk2_abscissae(S: int) -> np.ndarray:
    """c_i = (i-1)/(2(S-1)), i = 1..S (the S=6 and S=16 tableaux of Sec. 3.1)."""
    return np.array([(i - 1) / (2.0 * (S - 1)) for i in range(1, S + 1)])


def perk2_weights(S: int) -> np.ndarray:
    """b = e_S (explicit-midpoint type choice, Sec. 3.1)."""
    b = np.zeros(S)
    b[-1] = 1.0
    return b


def perk3_abscissae(S: int) -> np.ndarray:
    """c_i = (i-1)/(S-3) for i <= S-2 (eq. Free_Timesteps); c_{S-1} = 1, c_S = 1/2 from the
    Shu-Osher base (eq. PERK_ThirdOrderShuOsher)."""
    if S < 3:
        raise ValueError("third-order P-ERK needs S >= 3")
    c = np.zeros(S)
    if S > 3:
        for i in range(1, S - 1):
            c[i - 1] = (i - 1) / (S - 3.0)
    c[S - 2] = 1.0
    c[S - 1] = 0.5
    return c


def perk3_weights(S: int) -> np.ndarray:
    """b_1 = b_{S-1} = 1/6, b_S = 2/3 (Shu-Osher weights, eq. PERK_ThirdOrderShuOsher)."""
    b = np.zeros(S)
    b[0] += 1.0 / 6.0
    b[S - 2] += 1.0 / 6.0
    b[S - 1] += 2.0 / 3.0
    return b


def dense_A(c: np.ndarray, a_sub_row: np.ndarray) -> np.ndarray:
    """Full S x S Butcher matrix of one member: A[i,0] = c_i - a_{i,i-1}, A[i,i-1] = a_{i,i-1}.
    Row 2 (0-based 1) holds only a_{2,1} = c_2."""
    S = len(c)
    A = np.zeros((S, S))
    for i in range(1, S):
        if i == 1:
            A[1, 0] = c[1]
        else:
            A[i, i - 1] = a_sub_row[i]
            A[i, 0] = c[i] - a_sub_row[i]
    return A


def stability_poly(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Monomial coefficients of P(z) = 1 + z b^T (I - zA)^{-1} 1 = 1 + sum_k z^{k+1} b^T A^k 1
    (Sec. 4.3).  A is strictly lower triangular, so the series ends at k = S-1."""
    S = len(b)
    coef = np.zeros(S + 1)
    coef[0] = 1.0
    v = np.ones(S)
    for k in range(S):
        coef[k + 1] = b @ v
        v = A @ v
    return coef


def member_stage_evaluations(a_sub_row: np.ndarray, c: np.ndarray, b: np.ndarray) -> list:
    """Stages i (1-based) whose K_i enters the solution of this member when it is integrated
    alone: K_1, and every K_j used with a nonzero coefficient (Sec. 3.1, reducible methods)."""
    return stage_evaluations(dense_A(c, a_sub_row), b)


def stage_evaluations(A: np.ndarray, b: np.ndarray) -> list:
    """The same for a full Butcher matrix A: the stages reachable from the nonzero weights
    through nonzero entries of A."""
    S = len(b)
    needed = set()
    frontier = [j for j in range(S) if b[j] != 0.0]
    while frontier:
        j = frontier.pop()
        if j in needed:
            continue
        needed.add(j)
        frontier.extend(k for k in range(S) if A[j, k] != 0.0)
    return sorted(j + 1 for j in needed)


def order_condition_residuals(fam: PerkFamily) -> np.ndarray:
    """Residuals of eq. (PRKOrderCondsSimplified) up to fam.order, for every member."""
    c, b = fam.c, fam.b
    res = [b.sum() - 1.0]
    if fam.order >= 2:
        res.append(b @ c - 0.5)
    if fam.order >= 3:
        res.append(b @ (c * c) - 1.0 / 3.0)
        for r in range(len(fam.E)):
            A = dense_A(c, fam.a_sub[r])
            res.append(b @ (A @ c) - 1.0 / 6.0)
    return np.array(res)


def internal_consistency_residuals(fam: PerkFamily) -> np.ndarray:
    """sum_j a_ij^(r) - c_i, eq. (InternalConsistency)."""
    out = []
    for r in range(len(fam.E)):
        A = dense_A(fam.c, fam.a_sub[r])
        out.append(A.sum(axis=1) - fam.c)
    return np.array(out)


# ----------------------------------------------------------------------------------------
# Second order: closed-form construction from the monomial coefficients
# (eq. PERK2_StabPnom and eq. PERKCoeffsConstruction).
# ----------------------------------------------------------------------------------------
def perk2_a_from_alpha(alpha: dict, E: int, S: int) -> np.ndarray:
    """a_{S-i} = alpha_{3+i} / (c_{S-i-1} prod_{j<i} a_{S-j}), i = 0..E-3.
    alpha maps degree k (3..E) to the monomial coefficient of z^k."""
    c = perk2_abscissae(S)
    a = np.zeros(S)
    prod = 1.0
    for i in range(0, E - 2):
        row = S - i                         # 1-based row index S-i
        a[row - 1] = alpha[3 + i] / (c[row - 2] * prod)   # c_{S-i-1}
        prod *= a[row - 1]
    return a


def disk_optimal_alpha_p2(E: int) -> dict:
    """Second-order polynomial of degree E that is optimal for the disk of radius E-1 centred
    at -(E-1): P(z) = 1/E + (E-1)/E (1 + z/(E-1))^E (Owren & Seip, cited in Sec. 3.2.2).
    |1 + z/(E-1)| <= 1 on that disk, so |P| <= 1/E + (E-1)/E = 1 there."""
    s = E
    return {k: (s - 1) / s * math.comb(s, k) / (s - 1) ** k for k in range(3, E + 1)}


def disk_optimal_alpha_p1(E: int) -> dict:
    """First-order optimum for the disk of radius E: P(z) = (1 + z/E)^E."""
    return {k: math.comb(E, k) / E ** k for k in range(2, E + 1)}


def perk2_family(E_list, alphas=None) -> PerkFamily:
    E_list = sorted(E_list)
    S = E_list[-1]
    c = perk2_abscissae(S)
    b = perk2_weights(S)
    rows, al = [], []
    for E in E_list:
        alpha = alphas[E] if alphas is not None else disk_optimal_alpha_p2(E)
        rows.append(perk2_a_from_alpha(alpha, E, S))
        al.append(alpha)
    return PerkFamily(2, S, E_list, c, b, np.array(rows), al)


# ----------------------------------------------------------------------------------------
# Third order: nonlinear solve (Sec. 4.3.2).  Unknowns a_{i,i-1} for the E-2 rows
# i = S-E+3..S; equations: the z^3..z^E coefficients of P from the dense tableau equal
# (1/6, alpha_4..alpha_E).  The z^3 equation is b_S a_S + b_{S-1} a_{S-1} = 1/6.
# Positivity 0 < a_i < c_i; random starting points of a trust-region solver.  The unknowns are
# solved for as log a_i (positivity by construction, upper bound log c_i) and every equation
# is scaled by its target (coefficients of high degree are tiny), i.e. residuals
# coef_k(a) / alpha_k - 1.
# ----------------------------------------------------------------------------------------
def perk3_member(alpha: dict, E: int, S: int, seeds=range(200), tol=1e-12):
    from scipy.optimize import least_squares

    c = perk3_abscissae(S)
    b = perk3_weights(S)
    rows = list(range(S - E + 3, S + 1))          # 1-based rows with a free a_{i,i-1}
    if E == 3:
        a = np.zeros(S)
        a[S - 1] = (1.0 / 6.0) / b[S - 1]
        return a
    target = np.array([1.0 / 6.0] + [alpha[k] for k in range(4, E + 1)])

    def full(logx):
        a = np.zeros(S)
        for r, v in zip(rows, np.exp(logx)):
            a[r - 1] = v
        return a

    def resid(logx):
        coef = stability_poly(dense_A(c, full(logx)), b)
        return coef[3:E + 1] / target - 1.0

    hi = np.log(np.array([c[r - 1] for r in rows]))
    lo = np.full(len(rows), -60.0)
    for seed in seeds:
        x0 = hi + np.log(np.random.default_rng(seed).random(len(rows)))
        sol = least_squares(resid, x0, bounds=(lo, hi), xtol=1e-15, ftol=1e-15, gtol=1e-15,
                            method="trf", max_nfev=2000)
        a = full(sol.x)
        if np.max(np.abs(sol.fun)) < tol and all(0 < a[r - 1] < c[r - 1] for r in rows):
            return a
    raise RuntimeError(f"no positive third-order P-ERK tableau found for E={E}, S={S}")


def perk3_family(E_list, alphas: dict) -> PerkFamily:
    E_list = sorted(E_list)
    S = E_list[-1]
    c = perk3_abscissae(S)
    b = perk3_weights(S)
    rows = [perk3_member(alphas.get(E, {}), E, S) for E in E_list]
    return PerkFamily(3, S, E_list, c, b, np.array(rows), [alphas.get(E, {}) for E in E_list])


# ----------------------------------------------------------------------------------------
# Optimisation of the stability polynomial (eq. OptimizationProblem, Sec. 4.2):
# max h such that |P(h lambda)| <= 1 for all supplied eigenvalues.  For fixed h the
# constraint set is convex in alpha; it is replaced by the circumscribed regular M-gon
# Re(exp(-i theta_k) P) <= 1, a linear feasibility problem, and h is bisected.  The polygon
# touches the unit circle at P = 1, so eigenvalues near the origin (where P ~ exp(z) has
# modulus close to 1) stay feasible; elsewhere |P| <= 1/cos(pi/M) is guaranteed.
# ----------------------------------------------------------------------------------------
def _feasible(eigs, h, p, E, M):
    from scipy.optimize import linprog

    rho = np.max(np.abs(eigs))
    mu = eigs / rho                   # |mu| <= 1
    z = h * eigs
    fixed = sum(z ** j / math.factorial(j) for j in range(p + 1))
    # scaled unknowns g_j = alpha_j (h rho)^j multiply mu^j (all of modulus <= 1)
    basis = np.stack([mu ** j for j in range(p + 1, E + 1)], axis=1)   # [n, E-p]
    th = 2 * np.pi * np.arange(M) / M
    rot = np.exp(-1j * th)
    A_ub = np.concatenate([(rot[k] * basis).real for k in range(M)], axis=0)
    b_ub = np.concatenate([1.0 - (rot[k] * fixed).real for k in range(M)])
    res = linprog(np.zeros(E - p), A_ub=A_ub, b_ub=b_ub, bounds=[(None, None)] * (E - p),
                  method="highs")
    if res.status != 0:
        return None
    g = res.x
    return {j: g[j - p - 1] / (h * rho) ** j for j in range(p + 1, E + 1)}


def optimize_alpha(eigs, p: int, E: int, M: int = 128, rtol: float = 1e-6):
    """Return (h_max, alpha) with alpha the monomial coefficients of degree p+1..E."""
    eigs = np.asarray(eigs, dtype=complex)
    eigs = eigs[np.abs(eigs) > 0]
    rho = np.max(np.abs(eigs))
    if E <= p:
        # no free coefficient: the truncated Taylor polynomial
        coef = np.array([1.0 / math.factorial(j) for j in range(p + 1)])
        return max_stable_step(coef, eigs), {}
    lo, hi = 0.0, 2.0 * E * E / rho          # |P| <= 1 cannot hold beyond ~E^2/rho
    best = None
    # find a feasible lower bound first
    h = 0.5 / rho
    a = _feasible(eigs, h, p, E, M)
    while a is None and h > 1e-12:
        h *= 0.5
        a = _feasible(eigs, h, p, E, M)
    if a is None:
        raise RuntimeError("no feasible step")
    lo, best = h, a
    while hi - lo > rtol * lo:
        mid = 0.5 * (lo + hi)
        a = _feasible(eigs, mid, p, E, M)
        if a is None:
            hi = mid
        else:
            lo, best = mid, a
    return lo, best


def max_stable_step(coef: np.ndarray, eigs, rtol: float = 1e-10) -> float:
    """Largest h with |P(h lambda)| <= 1 + 1e-12 for every lambda, by bisection (continuous
    scan from 0; used to check optimiser output)."""
    eigs = np.asarray(eigs, dtype=complex)
    P = np.polynomial.Polynomial(coef)

    def ok(h):
        return np.all(np.abs(P(h * eigs)) <= 1 + 1e-12)

    hi = 1.0 / np.max(np.abs(eigs))
    while ok(hi):
        hi *= 2
    lo = 0.0
    while hi - lo > rtol * hi:
        mid = 0.5 * (lo + hi)
        if ok(mid):
            lo = mid
        else:
            hi = mid
    return lo


# ----------------------------------------------------------------------------------------
# Alternative stage-evaluation patterns (Sec. 3.2.4, eq. PERK_ButcherTableauAlternating and
# eq. PERK_ButcherTableauEarlyShared).  A second-order member with E evaluations is given by its
# chain of evaluated stages s_0 = 0 < s_1 < ... < s_{E-1} = S-1 (0-based): row s_1 is
# Y = U + dt c K_1, row s_m (m >= 2) couples K_1 and K_{s_{m-1}}, and b = e_S.  For the linear
# test equation the stage polynomials are y_1 = 1 + c_{s_1} z and
# y_m = 1 + c_{s_m} z + a_m z (y_{m-1} - 1), so
#   P(z) = 1 + z y_{E-1} = 1 + z + c_{S-1} z^2 + a_{E-1} c_{s_{E-2}} z^3
#          + a_{E-1} a_{E-2} c_{s_{E-3}} z^4 + ... + (a_{E-1} ... a_2) c_{s_1} z^E,
# and matching the monomial coefficients alpha_3 .. alpha_E fixes a_{E-1}, a_{E-2}, ... in turn
# (the classic chain s_m = S-E+m gives the construction of eq. PERKCoeffsConstruction).
# ----------------------------------------------------------------------------------------
PAPER_CHAINS_S6_E4 = {
    # 0-based evaluated stages of the S = 6, E = 4 tableaux printed in Sec. 3.1 and 3.2.4
    "classic": [0, 3, 4, 5],        # K_1, K_4, K_5, K_6
    "alternating": [0, 2, 3, 5],    # K_1, K_3, K_4, K_6
    "early_shared": [0, 1, 2, 5],   # K_1, K_2, K_3, K_6
}


def chain_member(alpha: dict, chain, S: int):
    """Coupling column (0-based, -1 for none) and coefficient a_{i,j} of every row of a
    second-order member evaluating the stages `chain` (0-based, starting at 0, ending at S-1),
    from the monomial coefficients alpha[3..E] of its stability polynomial."""
    chain = list(chain)
    E = len(chain)
    if chain[0] != 0 or chain[-1] != S - 1 or any(b <= a for a, b in zip(chain, chain[1:])):
        raise ValueError("chain must rise strictly from stage 0 to stage S-1")
    c = perk2_abscissae(S)
    coupling = -np.ones(S, dtype=np.int64)
    a = np.zeros(S)
    prod = 1.0
    for k in range(3, E + 1):
        m = E + 2 - k                    # chain position whose coefficient alpha_k fixes
        row, col = chain[m], chain[m - 1]
        a[row] = alpha[k] / (c[chain[m - 1]] * prod)
        coupling[row] = col
        prod *= a[row]
    return coupling, a


def dense_A_coupled(c: np.ndarray, coupling_row, a_row) -> np.ndarray:
    """Full S x S Butcher matrix of one member with one coupling per row: A[i,0] = c_i - a_i and
    A[i, j] = a_i for j = coupling_row[i] >= 1, else A[i,0] = c_i."""
    S = len(c)
    A = np.zeros((S, S))
    for i in range(1, S):
        j = int(coupling_row[i])
        if j >= 1:
            A[i, j] = a_row[i]
            A[i, 0] = c[i] - a_row[i]
        else:
            A[i, 0] = c[i]
    return A


@dataclass
class PatternFamily:
    """Second-order P-ERK family whose members evaluate their stages along chains of their own
    (Sec. 3.2.4); c and b = e_S shared.  coupling[r][i] is the 0-based column j >= 1 of the one
    coupling of row i (-1: none), a_val[r][i] the coefficient a_{i,j}."""
    order: int
    S: int
    E: list
    c: np.ndarray
    b: np.ndarray
    coupling: np.ndarray     # [R, S] int
    a_val: np.ndarray        # [R, S]
    chains: list = field(default_factory=list)

    def dense(self, r):
        return dense_A_coupled(self.c, self.coupling[r], self.a_val[r])

    @property
    def a_sub(self):
        """The coefficient of every row's coupling (the per-row table a solver takes)."""
        return self.a_val


def pattern_family(chains, S: int, alphas=None) -> PatternFamily:
    """Members given by their chains of evaluated stages, each with the disk-optimal
    second-order polynomial of its degree unless alphas[E] is given."""
    chains = sorted((list(ch) for ch in chains), key=len)
    c = perk2_abscissae(S)
    b = perk2_weights(S)
    cp, av, E = [], [], []
    for ch in chains:
        e = len(ch)
        alpha = alphas[e] if alphas is not None and e in alphas else disk_optimal_alpha_p2(e)
        j, a = chain_member(alpha, ch, S)
        cp.append(j)
        av.append(a)
        E.append(e)
    return PatternFamily(2, S, E, c, b, np.array(cp), np.array(av), chains)
