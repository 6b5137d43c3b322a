"""P-ERK coefficient generation (offline host tool): spectrum -> optimised stability
polynomials -> Butcher coefficients of the family.

Paper passages
  * Spectrum of a reduced-resolution semidiscretisation, scaled by h_reduced / h (Sec. 4.1,
    steps 1 and 4): here the Jacobian is formed column by column from central differences of
    libperk's right-hand side on the GPU, then eigenvalues by dense LAPACK.
  * Optimisation max dt s.t. |P(dt lambda)| <= 1 (eq. OptimizationProblem, Sec. 4.2): for a
    fixed dt the admissible set of free monomial coefficients is convex; |P| <= 1 is imposed
    on a circumscribed polygon of the unit disk (a linear programme) and dt is bisected.
  * Second-order construction in closed form, eq. (PERKCoeffsConstruction) with
    c_i = (i-1)/(2(S-1)), b = e_S (Sec. 3.1, 4.3.1).
  * Third-order construction by a bounded nonlinear least-squares solve with positivity
    0 < a_{i,i-1} < c_i from seeded random starts (Sec. 4.3.2), abscissae eq. (Free_Timesteps),
    Shu-Osher weights (eq. PERK_ThirdOrderShuOsher).
"""
from __future__ import annotations

import ctypes
import json
import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Family:
    order: int
    S: int
    E: list
    c: np.ndarray
    b: np.ndarray
    a_sub: np.ndarray             # [R, S], a_{i,i-1} (or a_{i,j} of row i's coupling column j)
    dt_opt: list = None           # optimal step per member for the spectrum it was built on
    h_ref: float = None           # element size that spectrum belongs to
    coupling: np.ndarray = None   # [R, S] coupling column per row (-1 none); None: classic pattern

    def to_dict(self):
        return {"order": self.order, "S": self.S, "E": [int(e) for e in self.E],
                "c": self.c.tolist(), "b": self.b.tolist(), "a_sub": self.a_sub.tolist(),
                "dt_opt": None if self.dt_opt is None else [float(x) for x in self.dt_opt],
                "h_ref": self.h_ref,
                "coupling": None if self.coupling is None else np.asarray(self.coupling).tolist()}

    @staticmethod
    def from_dict(d):
        cp = d.get("coupling")
        return Family(d["order"], d["S"], list(d["E"]), np.asarray(d["c"], float), np.asarray(d["b"], float),
                      np.asarray(d["a_sub"], float), d.get("dt_opt"), d.get("h_ref"),
                      None if cp is None else np.asarray(cp, np.int32))

    def save(self, path):
        with open(path, "w") as f:
            json.dump(self.to_dict(), f, indent=1)

    @staticmethod
    def load(path):
        with open(path) as f:
            return Family.from_dict(json.load(f))


# ------------------------------------------------------------------ tableau structure
def abscissae(order, S):
    if order == 2:
        return np.arange(S) / (2.0 * (S - 1)) if S > 1 else np.zeros(1)
    c = np.zeros(S)
    free = S - 2
    for i in range(free):
        c[i] = i / (S - 3.0) if S > 3 else 0.0
    c[S - 2], c[S - 1] = 1.0, 0.5
    return c


def weights(order, S):
    b = np.zeros(S)
    if order == 2:
        b[-1] = 1.0
    else:
        b[0] += 1 / 6
        b[S - 2] += 1 / 6
        b[S - 1] += 2 / 3
    return b


def member_matrix(c, a_row):
    """Full Butcher matrix of one member from its a_{i,i-1} and internal consistency."""
    S = len(c)
    A = np.zeros((S, S))
    if S > 1:
        A[1, 0] = c[1]
    for i in range(2, S):
        A[i, i - 1] = a_row[i]
        A[i, 0] = c[i] - a_row[i]
    return A


def poly_of(A, b):
    """Coefficients of 1 + z b^T (I - z A)^{-1} 1 (A strictly lower triangular)."""
    S = len(b)
    out = [1.0]
    v = np.ones(S)
    for _ in range(S):
        out.append(float(b @ v))
        v = A @ v
    return np.array(out)


# ------------------------------------------------------------------ optimisation
def _lp_feasible(lam, dt, p, E, n_poly):
    from scipy.optimize import linprog
    r = np.max(np.abs(lam))
    mu = lam / r
    z = dt * lam
    base = np.zeros_like(z)
    term = np.ones_like(z)
    for j in range(p + 1):
        base = base + term
        term = term * z / (j + 1)
    cols = np.stack([mu ** j for j in range(p + 1, E + 1)], axis=1)
    rows, rhs = [], []
    for k in range(n_poly):
        rot = np.exp(-2j * np.pi * k / n_poly)
        rows.append((rot * cols).real)
        rhs.append(1.0 - (rot * base).real)
    res = linprog(np.zeros(E - p), A_ub=np.vstack(rows), b_ub=np.concatenate(rhs),
                  bounds=[(None, None)] * (E - p), method="highs")
    if res.status != 0:
        return None
    scale = dt * r
    return {j: res.x[j - p - 1] / scale ** j for j in range(p + 1, E + 1)}


def optimise(lam, p, E, n_poly=128, rtol=1e-6):
    """Largest dt (and the polynomial) with |P(dt lam)| <= 1 on the circumscribed n_poly-gon."""
    lam = np.asarray(lam, complex)
    lam = lam[np.abs(lam) > 1e-12 * np.max(np.abs(lam))]
    r = np.max(np.abs(lam))
    if E <= p:
        coef = np.array([1 / math.factorial(j) for j in range(p + 1)])
        return stable_step(coef, lam), {}
    lo = 0.5 / r
    sol = _lp_feasible(lam, lo, p, E, n_poly)
    while sol is None:
        lo *= 0.5
        sol = _lp_feasible(lam, lo, p, E, n_poly)
    hi = 2.0 * E * E / r
    while hi - lo > rtol * lo:
        mid = 0.5 * (lo + hi)
        s = _lp_feasible(lam, mid, p, E, n_poly)
        if s is None:
            hi = mid
        else:
            lo, sol = mid, s
    return lo, sol


def stable_step(coef, lam, tol=1e-12):
    P = np.polynomial.Polynomial(coef)
    ok = lambda h: np.all(np.abs(P(h * lam)) <= 1 + tol)
    hi = 1.0 / np.max(np.abs(lam))
    while ok(hi):
        hi *= 2
    lo = 0.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if ok(mid) else (lo, mid)
    return lo


# ------------------------------------------------------------------ construction
def perk2_row(alpha, E, S):
    c = abscissae(2, S)
    a = np.zeros(S)
    prod = 1.0
    for i in range(E - 2):
        row = S - 1 - i                     # 0-based row S-i
        a[row] = alpha[3 + i] / (c[row - 1] * prod)
        prod *= a[row]
    return a


def perk3_row(alpha, E, S, n_starts=200):
    """Solve for the free a_{i,i-1} of a third-order member: unknowns log a_i (positive, below
    log c_i), residuals scaled by their targets (poly coefficient / target - 1)."""
    from scipy.optimize import least_squares
    c = abscissae(3, S)
    b = weights(3, S)
    if E == 3:
        a = np.zeros(S)
        a[S - 1] = (1 / 6) / b[S - 1]
        return a
    free = np.arange(S - E + 2, S)           # 0-based rows with a free a_{i,i-1}
    target = np.array([1 / 6] + [alpha[k] for k in range(4, E + 1)])

    def assemble(y):
        a = np.zeros(S)
        a[free] = np.exp(y)
        return a

    def res(y):
        return poly_of(member_matrix(c, assemble(y)), b)[3:E + 1] / target - 1.0

    upper = np.log(c[free])
    lower = np.full(len(free), -60.0)
    for seed in range(n_starts):
        y0 = upper + np.log(np.random.default_rng(1000 + seed).random(len(free)))
        s = least_squares(res, y0, bounds=(lower, upper), xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=2000)
        a = assemble(s.x)
        if np.max(np.abs(s.fun)) < 1e-12 and np.all(a[free] > 0) and np.all(a[free] < c[free]):
            return a
    raise RuntimeError(f"no positive third-order tableau for E={E}")


def coupled_matrix(c, coupling_row, a_row):
    """Full Butcher matrix of one member whose row i couples K_1 and K_j, j = coupling_row[i]."""
    S = len(c)
    A = np.zeros((S, S))
    for i in range(1, S):
        j = int(coupling_row[i])
        A[i, 0] = c[i] - (a_row[i] if j >= 1 else 0.0)
        if j >= 1:
            A[i, j] = a_row[i]
    return A


def rechain(fam, r, chain):
    """Member r of a second-order family moved onto another chain of evaluated stages (0-based,
    from stage 0 to S-1; Sec. 3.2.4), keeping its stability polynomial.  The couplings are found
    one at a time from the last row backwards: each new coefficient enters the polynomial
    coefficient it fixes linearly, so two evaluations of the tableau's polynomial (coefficient 0
    and 1) give it.  Returns (coupling row, coefficient row)."""
    if fam.order != 2:
        raise ValueError("stage patterns are built for second-order families")
    S = fam.S
    c, b = np.asarray(fam.c), np.asarray(fam.b)
    cp0 = None if fam.coupling is None else fam.coupling[r]
    A0 = member_matrix(c, fam.a_sub[r]) if cp0 is None else coupled_matrix(c, cp0, fam.a_sub[r])
    target = poly_of(A0, b)
    chain = [int(x) for x in chain]
    E = len(chain)
    if chain[0] != 0 or chain[-1] != S - 1 or any(q <= p for p, q in zip(chain, chain[1:])):
        raise ValueError("chain must rise strictly from stage 0 to stage S-1")
    coupling = -np.ones(S, dtype=np.int32)
    a = np.zeros(S)
    for m in range(E - 1, 1, -1):
        row, col = chain[m], chain[m - 1]
        coupling[row] = col
        k = E + 2 - m                       # polynomial degree this coefficient fixes
        vals = []
        for trial in (0.0, 1.0):
            a[row] = trial
            vals.append(poly_of(coupled_matrix(c, coupling, a), b)[k])
        a[row] = (target[k] - vals[0]) / (vals[1] - vals[0])
    if np.max(np.abs(poly_of(coupled_matrix(c, coupling, a), b) - target)) > 1e-12 * np.max(np.abs(target)):
        raise RuntimeError("rechain: polynomial not reproduced")
    return coupling, a


def with_chains(fam, chains):
    """The family with member r moved onto chains[r] (None: keep its stages)."""
    R, S = len(fam.E), fam.S
    cp = np.array([[i - 1 if i >= S - fam.E[r] + 2 else -1 for i in range(S)] for r in range(R)], np.int32) \
        if fam.coupling is None else np.array(fam.coupling, np.int32)
    a = np.array(fam.a_sub, float)
    for r, ch in enumerate(chains):
        if ch is None:
            continue
        if len(ch) != fam.E[r]:
            raise ValueError(f"member {r}: chain of {len(ch)} stages for E = {fam.E[r]}")
        cp[r], a[r] = rechain(fam, r, ch)
    return Family(fam.order, S, list(fam.E), np.asarray(fam.c), np.asarray(fam.b), a, fam.dt_opt, fam.h_ref, cp)


def hull_points(lam):
    """Boundary of the spectrum in the closed upper half plane (Sec. 4.1, step 2): convex hull
    of the eigenvalues with non-negative imaginary part plus the origin, with extra points on
    every hull edge so that consecutive points are no farther apart than the mean edge length.
    |P| <= 1 on this polygon implies |P| <= 1 inside it (maximum modulus principle)."""
    from scipy.spatial import ConvexHull
    pts = np.asarray(lam, complex)
    pts = pts[pts.imag >= 0]
    xy = np.unique(np.round(np.stack([np.append(pts.real, 0.0), np.append(pts.imag, 0.0)], axis=1), 14), axis=0)
    if len(xy) < 3:
        return pts
    hull = ConvexHull(xy)
    v = xy[hull.vertices]
    ring = np.concatenate([v, v[:1]])
    seg = np.linalg.norm(np.diff(ring, axis=0), axis=1)
    delta = seg.mean()
    out = []
    for k in range(len(v)):
        a, b = ring[k], ring[k + 1]
        m = max(1, int(np.ceil(seg[k] / delta)))
        for t in np.arange(m) / m:
            p = a + t * (b - a)
            out.append(p[0] + 1j * p[1])
    out = np.array(out)
    return out[out.imag >= -1e-14]


def build_family(order, E_list, lam, h_ref=None):
    """Optimise every member on the spectrum lam and build the family."""
    E_list = sorted(int(e) for e in E_list)
    S = E_list[-1]
    rows, dts = [], []
    for E in E_list:
        dt, alpha = optimise(lam, order, E)
        rows.append(perk2_row(alpha, E, S) if order == 2 else perk3_row(alpha, E, S))
        dts.append(dt)
    return Family(order, S, E_list, abscissae(order, S), weights(order, S), np.array(rows), dts, h_ref)


def check_family(fam, tol=1e-12):
    """Order conditions (eq. PRKOrderCondsSimplified) and internal consistency."""
    c, b = fam.c, fam.b
    ok = abs(b.sum() - 1) < tol and abs(b @ c - 0.5) < tol
    if fam.order == 3:
        ok &= abs(b @ c ** 2 - 1 / 3) < tol
        for r in range(len(fam.E)):
            ok &= abs(b @ member_matrix(c, fam.a_sub[r]) @ c - 1 / 6) < tol
    return bool(ok)


# ------------------------------------------------------------------ spectrum on the GPU
def fd_spectrum(solver, u_leaf, eps=1e-7):
    """Eigenvalues of dF/dU at u_leaf, Jacobian columns by central differences of the HIP
    right-hand side (slot layout)."""
    import torch
    solver.set_state(u_leaf)
    u0 = solver.u.clone()
    n = u0.numel()
    J = np.zeros((n, n))
    for k in range(n):
        h = eps * max(1.0, abs(float(u0[k])))
        up = u0.clone(); up[k] += h
        um = u0.clone(); um[k] -= h
        J[:, k] = ((solver.rhs_slot(up) - solver.rhs_slot(um)) / (2 * h)).cpu().numpy()
    torch.cuda.synchronize()
    lam = np.linalg.eigvals(J)
    lam = lam[lam.imag >= 0]                  # spectrum is symmetric about the real axis
    lam.real = np.minimum(lam.real, 0.0)      # round-off positive real parts
    return lam


def arnoldi(solver, u_slot, m, op="fd", eps=1e-7, seed=0):
    """m steps of the Arnoldi iteration on J = F'(u) at the solver's mesh (Sec. 4.1 step 4):
    products with J by central differences (op "fd", any equations), exact products with J
    (op "jvp", forward mode, Euler) or with J^T (op "vjp", Euler; same eigenvalues), orthogonalisation by two passes of classical
    Gram-Schmidt, all in libperk kernels on device vectors.  Returns the (j+1) x j Hessenberg
    matrix of the j <= m steps taken (fewer if the Krylov space closes)."""
    import torch
    from . import _lib as L
    n = u_slot.numel()
    V = torch.zeros((m + 1, n), dtype=torch.float64, device=u_slot.device)
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    v0 = torch.randn(n, generator=g, dtype=torch.float64)
    # element slots only (the reserved capacity's padding stays zero)
    v0 = v0.view(solver.nv, -1, solver.Nd)
    v0[:, solver.n_elements:, :] = 0.0
    V[0].copy_(v0.reshape(-1))
    nd = ctypes.c_int64()
    if solver.lib.pe_orthogonalize_scratch(m + 1, ctypes.byref(nd)) != 0:
        raise RuntimeError("pe_orthogonalize_scratch failed")
    scratch = torch.empty(nd.value, dtype=torch.float64, device=u_slot.device)
    solver.orthogonalize(V, 0, V[0], scratch)
    H = np.zeros((m + 1, m))
    steps = 0
    for j in range(m):
        if op == "fd":
            solver.jvp_fd_slot(u_slot, V[j], V[j + 1], eps)
        elif op == "jvp":
            solver.jvp_into(u_slot, V[j], V[j + 1])
        else:
            solver.vjp_into(u_slot, V[j], V[j + 1])
        h = solver.orthogonalize(V, j + 1, V[j + 1], scratch)
        H[: j + 2, j] = h
        steps = j + 1
        if h[j + 1] <= 1e-13 * max(1.0, np.abs(H[: j + 2, : j + 1]).max()):
            break
    torch.cuda.synchronize()
    return H[: steps + 1, :steps]


def harmonic_ritz(H, sigma):
    """Harmonic Ritz values of an Arnoldi factorisation with respect to the target sigma: the
    eigenvalue estimates from the Krylov space closest to sigma (the role the shifted Arnoldi runs
    around hull points play in Sec. 4.1)."""
    m = H.shape[1]
    Hm = H[:m, :m].astype(complex)
    A = Hm - sigma * np.eye(m)
    beta = H[m, m - 1] if H.shape[0] > m else 0.0
    em = np.zeros(m)
    em[-1] = 1.0
    f = np.linalg.solve(A.conj().T, em)
    return sigma + np.linalg.eigvals(A + (abs(beta) ** 2) * np.outer(f, em))


def full_mesh_spectrum(solver, u_slot, reduced_lam, h_reduced, h, m=240, per_shift=None, op="fd", eps=1e-7):
    """Outer eigenvalues of the real mesh's Jacobian (Sec. 4.1 steps 2-4): the hull points of the
    reduced spectrum scaled by h_reduced / h serve as targets; from one Arnoldi factorisation of m
    steps, the Ritz values and, per target, the harmonic Ritz values nearest to it (per_shift of
    them, 1000 / K by default) form the estimate."""
    H = arnoldi(solver, u_slot, m, op=op, eps=eps)
    shifts = hull_points(np.asarray(reduced_lam)) * (h_reduced / h)
    K = len(shifts)
    per = per_shift or max(1, 1000 // max(1, K))
    ritz = np.linalg.eigvals(H[: H.shape[1], : H.shape[1]])
    est = [ritz]
    for sg in shifts:
        th = harmonic_ritz(H, sg)
        est.append(th[np.argsort(np.abs(th - sg))[:per]])
    lam = np.concatenate(est)
    lam = lam[np.isfinite(lam)]
    lam = lam[lam.imag >= 0]
    lam.real = np.minimum(lam.real, 0.0)
    return lam, H


def family_from_solver_spectrum(solver, u_leaf, order, E_list, h_ref):
    """Sec. 4.1 steps 1-2 on the GPU right-hand side, then Sec. 4.2-4.3."""
    lam = fd_spectrum(solver, u_leaf)
    fam = build_family(order, E_list, hull_points(lam), h_ref=h_ref)
    if not check_family(fam):
        raise RuntimeError("constructed family violates the order conditions")
    return fam, lam
