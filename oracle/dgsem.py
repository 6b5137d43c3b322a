"""Oracle: Python front end of dgsem.cpp (serial C++ DGSEM + dense partitioned RK).

Test infrastructure only (see oracle/__init__.py).  States are numpy arrays of shape
[n_elements, n_vars, nodes_per_element] in the order of the leaf list given to the solver.

Also here: the level -> member rule of Sec. 6.4.1 (the finest level gets the member with the
most stage evaluations, the next finer the next member, all remaining coarse levels the
member with the fewest evaluations), and the scalar RHS-evaluation count eq. (ActualRHSEvals).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .perk_coeffs import PerkFamily, dense_A

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "dgsem.cpp")


def build(force=False):
    """Compile dgsem.cpp with g++ (serial, -O2, no floating-point contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ip, dp, dp, ctypes.c_int, ip]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_sizes.argtypes = [ctypes.c_void_p, ip]
        L.orc_rhs.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_node_coords.argtypes = [ctypes.c_void_p, dp]
        L.orc_lgl.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_mortar_ops.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        for name in ("orc_ec_flux", "orc_hll_flux"):
            getattr(L, name).argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_int, dp]
        L.orc_euler_flux.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, dp]
        L.orc_log_mean.restype = ctypes.c_double
        L.orc_log_mean.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_faces.argtypes = [ctypes.c_void_p, ip, ip]
        L.orc_prk_step.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   dp, dp, ip]
        L.orc_rk_step.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_int, dp, dp]
        L.orc_rhs_jvp.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.orc_rhs_vjp.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_prk_step_jvp.argtypes = [ctypes.c_void_p, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       dp, dp, ip, dp, dp]
        L.orc_prk_step_vjp.argtypes = [ctypes.c_void_p, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       dp, dp, ip, dp]
        L.orc_hll_branch_counts.argtypes = [ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]
        L.orc_set_shock_capturing.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double]
        L.orc_sc_indicator.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.orc_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def lgl(N):
    x, w, D = np.zeros(N), np.zeros(N), np.zeros(N * N)
    lib().orc_lgl(N, _dp(x), _dp(w), _dp(D))
    return x, w, D.reshape(N, N)


def ec_flux(dim, gamma, uL, uR, d):
    uL = np.ascontiguousarray(uL, float); uR = np.ascontiguousarray(uR, float)
    f = np.zeros(dim + 2)
    lib().orc_ec_flux(dim, gamma, _dp(uL), _dp(uR), d, _dp(f))
    return f


def hll_flux(dim, gamma, uL, uR, d):
    uL = np.ascontiguousarray(uL, float); uR = np.ascontiguousarray(uR, float)
    f = np.zeros(dim + 2)
    lib().orc_hll_flux(dim, gamma, _dp(uL), _dp(uR), d, _dp(f))
    return f


def euler_flux(dim, gamma, u, d):
    u = np.ascontiguousarray(u, float)
    f = np.zeros(dim + 2)
    lib().orc_euler_flux(dim, gamma, _dp(u), d, _dp(f))
    return f


def log_mean(a, b):
    return lib().orc_log_mean(float(a), float(b))


def _member_A(fam, r):
    """Full Butcher matrix of member r: families with alternative stage patterns (Sec. 3.2.4)
    carry it themselves, the classic ones by their a_{i,i-1} rows."""
    if hasattr(fam, "dense"):
        return fam.dense(r)
    return dense_A(fam.c, fam.a_sub[r])


class Oracle:
    """Serial DGSEM solver on one forest mesh."""

    def __init__(self, mesh, N, gamma=1.4, viscous=False, mu=0.0, prandtl=0.72, surface="hll"):
        self.mesh = mesh
        self.dim = mesh.dim
        self.N = N
        self.gamma = gamma
        leaves = np.ascontiguousarray(mesh.leaves, dtype=np.int32)
        nr = np.array(list(mesh.n_root) + [1] * (3 - mesh.dim), dtype=np.int32)
        lo = np.array(list(mesh.lo) + [0.0] * (3 - mesh.dim), dtype=float)
        hi = np.array(list(mesh.hi) + [1.0] * (3 - mesh.dim), dtype=float)
        h = lib().orc_create(mesh.dim, N, int(viscous), int(surface == "ec"), gamma, mu, prandtl, _ip(nr), _dp(lo), _dp(hi),
                             leaves.shape[0], _ip(leaves))
        if not h:
            raise ValueError(lib().orc_last_error().decode())
        self._h = h
        sz = np.zeros(3, np.int32)
        lib().orc_sizes(h, _ip(sz))
        self.n_elements, self.nv, self.Nd = (int(s) for s in sz)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    @property
    def shape(self):
        return (self.n_elements, self.nv, self.Nd)

    def node_coords(self):
        x = np.zeros((self.n_elements, self.dim, self.Nd))
        lib().orc_node_coords(self._h, _dp(x))
        return x

    def element_sizes(self):
        lev = self.mesh.leaves[:, 0]
        return np.array([[(self.mesh.hi[d] - self.mesh.lo[d]) / (self.mesh.n_root[d] << int(l))
                          for d in range(self.dim)] for l in lev])

    def set_shock_capturing(self, on=True, alpha_max=0.5, alpha_min=0.001, alpha_fixed=None):
        """Subcell shock capturing (Hennemann et al., used by the paper for its inviscid runs) with
        the blending factor of the density indicator, or alpha_fixed on every element."""
        if lib().orc_set_shock_capturing(self._h, int(bool(on)), float(alpha_max), float(alpha_min),
                                         -1.0 if alpha_fixed is None else float(alpha_fixed)) != 0:
            raise ValueError(lib().orc_last_error().decode())

    def sc_indicator(self, u):
        """(E, alpha) per element for state u, and the modal transform Vinv [N, N]."""
        u = np.ascontiguousarray(u, float).reshape(self.shape)
        E, a, V = np.zeros(self.n_elements), np.zeros(self.n_elements), np.zeros(self.N * self.N)
        lib().orc_sc_indicator(self._h, _dp(u), _dp(E), _dp(a), _dp(V))
        return E, a, V.reshape(self.N, self.N)

    def rhs(self, u):
        u = np.ascontiguousarray(u, float).reshape(self.shape)
        du = np.zeros(self.shape)
        lib().orc_rhs(self._h, _dp(u), _dp(du))
        return du

    def faces(self):
        nf = 2 * self.dim
        kinds = np.zeros((self.n_elements, nf), np.int32)
        nbrs = np.zeros((self.n_elements, nf, 4), np.int32)
        lib().orc_faces(self._h, _ip(kinds), _ip(nbrs))
        return kinds, nbrs

    def mortar_ops(self):
        N = self.N
        P0, P1, R0, R1 = (np.zeros(N * N) for _ in range(4))
        lib().orc_mortar_ops(self._h, _dp(P0), _dp(P1), _dp(R0), _dp(R1))
        return [P0.reshape(N, N), P1.reshape(N, N)], [R0.reshape(N, N), R1.reshape(N, N)]

    def prk_step(self, u, dt, fam: PerkFamily, member):
        """One step of the partitioned RK method (dense, masked)."""
        u = np.array(u, dtype=float, copy=True).reshape(self.shape)
        A = np.ascontiguousarray(np.stack([_member_A(fam, r) for r in range(len(fam.E))]))
        b = np.ascontiguousarray(fam.b, float)
        mem = np.ascontiguousarray(member, np.int32)
        rc = lib().orc_prk_step(self._h, _dp(u), float(dt), len(fam.E), fam.S, _dp(A), _dp(b), _ip(mem))
        if rc != 0:
            raise ValueError(lib().orc_last_error().decode())
        return u

    # ---- tangent and adjoint of the Euler operator and of the step (dual numbers, dense)
    def _arr(self, x):
        return np.ascontiguousarray(np.asarray(x, dtype=float).reshape(self.shape))

    def rhs_jvp(self, u, du):
        """(F(u), F'(u) du) for the Euler operator."""
        u, du = self._arr(u), self._arr(du)
        f, t = np.zeros(self.shape), np.zeros(self.shape)
        if lib().orc_rhs_jvp(self._h, _dp(u), _dp(du), _dp(f), _dp(t)) != 0:
            raise ValueError(lib().orc_last_error().decode())
        return f, t

    def rhs_vjp(self, u, w):
        """F'(u)^T w, assembled column by column (small meshes only)."""
        u, w = self._arr(u), self._arr(w)
        out = np.zeros(self.shape)
        if lib().orc_rhs_vjp(self._h, _dp(u), _dp(w), _dp(out)) != 0:
            raise ValueError(lib().orc_last_error().decode())
        return out

    def _step_args(self, fam, member):
        A = np.ascontiguousarray(np.stack([_member_A(fam, r) for r in range(len(fam.E))]))
        return A, np.ascontiguousarray(fam.b, float), np.ascontiguousarray(member, np.int32)

    def prk_step_jvp(self, u, du, dt, fam: PerkFamily, member):
        """(Phi(u), Phi'(u) du) for one partitioned step (Euler)."""
        u, du = self._arr(u), self._arr(du)
        A, b, mem = self._step_args(fam, member)
        u1, t = np.zeros(self.shape), np.zeros(self.shape)
        if lib().orc_prk_step_jvp(self._h, _dp(u), _dp(du), float(dt), len(fam.E), fam.S, _dp(A), _dp(b), _ip(mem),
                                  _dp(u1), _dp(t)) != 0:
            raise ValueError(lib().orc_last_error().decode())
        return u1, t

    def prk_step_vjp(self, u, lam, dt, fam: PerkFamily, member):
        """Phi'(u)^T lam for one partitioned step (Euler), column by column (small meshes)."""
        u, lam = self._arr(u), self._arr(lam)
        A, b, mem = self._step_args(fam, member)
        out = np.zeros(self.shape)
        if lib().orc_prk_step_vjp(self._h, _dp(u), _dp(lam), float(dt), len(fam.E), fam.S, _dp(A), _dp(b), _ip(mem),
                                  _dp(out)) != 0:
            raise ValueError(lib().orc_last_error().decode())
        return out

    def rk_step(self, u, dt, A, b):
        u = np.array(u, dtype=float, copy=True).reshape(self.shape)
        A = np.ascontiguousarray(A, float)
        b = np.ascontiguousarray(b, float)
        lib().orc_rk_step(self._h, _dp(u), float(dt), len(b), _dp(A), _dp(b))
        return u

    def integral(self, u):
        """sum_e prod_d (h_d/2) sum_nodes w_node u: the discrete integral of each variable."""
        x, w, _ = lgl(self.N)
        if self.dim == 2:
            W = np.einsum("i,j->ji", w, w).reshape(-1)
        else:
            W = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
        jac = np.prod(self.element_sizes() / 2.0, axis=1)
        return np.einsum("e,evn,n->v", jac, u, W)


def hll_branch_counts(reset=False):
    """Branches the oracle's HLL flux took since the last reset: [sL >= 0, sR <= 0, subsonic]."""
    out = (ctypes.c_longlong * 3)()
    lib().orc_hll_branch_counts(out, int(bool(reset)))
    return list(out)


def max_dt(o: Oracle, u, cfl=1.0, gamma=1.4):
    """Step-size bound of eq. (CFL_DG) and eq. (TimestepConstraint): for every element,
    beta_e = min over its nodes and the directions d of h_d / ((k+1) (|v_d| + c)), with k + 1 =
    o.N nodes per direction and c the speed of sound; beta per refinement level is the minimum
    over the level's elements, and dt = cfl * min over levels.  Returns (dt, {level: beta})."""
    h = o.element_sizes()
    lev = np.asarray(o.mesh.leaves)[:, 0]
    betas = {}
    for e in range(o.n_elements):
        rho = u[e, 0]
        vel = [u[e, 1 + d] / rho for d in range(o.dim)]
        p = (gamma - 1.0) * (u[e, o.dim + 1] - 0.5 * rho * sum(v * v for v in vel))
        c = np.sqrt(gamma * p / rho)
        b = min(float(np.min(h[e, d] / (o.N * (np.abs(vel[d]) + c)))) for d in range(o.dim))
        betas[int(lev[e])] = min(betas.get(int(lev[e]), np.inf), b)
    return cfl * min(betas.values()), betas


def member_of_levels_paper_rule(levels, n_members):
    """Sec. 6.4.1: finest level -> member R-1 (most evaluations), next finer -> R-2, ...,
    every level beyond the R-th finest -> member 0."""
    levels = np.asarray(levels)
    Lmax = int(levels.max())
    return np.maximum(0, (n_members - 1) - (Lmax - levels)).astype(np.int32)


def n_rhs_actual(levels_per_interval, member_of_level, E, n_vars, nodes_per_element, n_amr):
    """Scalar RHS evaluations, eq. (ActualRHSEvals): sum over AMR intervals of
    N_AMR * N * (k+1)^{N_D} * sum_elements E^(member)."""
    total = 0
    for levels in levels_per_interval:
        mem = member_of_level(levels)
        total += n_amr * n_vars * nodes_per_element * int(np.sum(np.asarray(E)[mem]))
    return total
