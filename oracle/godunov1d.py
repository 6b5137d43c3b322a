"""Oracle: first-order Godunov finite volumes for u_t + u_x = 0 with a partitioned RK step.

Test infrastructure only (see oracle/__init__.py).

Paper passages followed (Sec. 3.2)
  * Upwind semidiscretisation dU/dt = L U on a possibly non-uniform periodic grid,
    eq. (UpwindFullSystem): row i has -1/dx_i on the diagonal and +1/dx_i on column i-1
    (periodic, so row 1 couples to column N).
  * One step of a partitioned RK method with mask matrices I^(r) (Sec. 2.2):
    K_i^(r) = I^(r) F(U_n + dt sum_j sum_k a_ij^(k) K_j^(k)),
    U_{n+1} = U_n + dt sum_i sum_r b_i^(r) K_i^(r)  (eq. PartitionedRKSystem).
    For the linear F = L U this gives U_{n+1} = D U_n (eq. PartitionedSystem).
  * Monotonicity D_ij >= 0 (eq. MonotonicityRequirement); row sums 1 (conservation).
  * Relative total-variation increase after one step, Sec. 3.2.5, with TV(U) = sum |U_{i+1}-U_i|
    taken periodically, and cell averages of u_0 = 1 + sin(pi x)/2 on (-1, 1).
"""
from __future__ import annotations

import numpy as np

from .perk_coeffs import PerkFamily, dense_A


def upwind_matrix(dx: np.ndarray) -> np.ndarray:
    N = len(dx)
    L = np.zeros((N, N))
    for i in range(N):
        L[i, i] = -1.0 / dx[i]
        L[i, (i - 1) % N] = 1.0 / dx[i]
    return L


def prk_step_matrix(L: np.ndarray, dt: float, fam: PerkFamily, member_of_cell: np.ndarray):
    """D such that U_{n+1} = D U_n for the partitioned RK step with masks built from
    member_of_cell (index into fam.E per cell).  Plain dense evaluation of every stage of every
    member; stages a member does not use are multiplied by zero Butcher entries."""
    N = L.shape[0]
    R = len(fam.E)
    S = fam.S
    A = [dense_A(fam.c, fam.a_sub[r]) for r in range(R)]
    masks = [np.diag((member_of_cell == r).astype(float)) for r in range(R)]
    # K[j][k] is the N x N matrix mapping U_n to K_j^(k)
    K = [[None] * R for _ in range(S)]
    I = np.eye(N)
    for i in range(S):
        stage = I.copy()
        for j in range(i):
            for k in range(R):
                if A[k][i, j] != 0.0:
                    stage = stage + dt * A[k][i, j] * K[j][k]
        F = L @ stage
        for r in range(R):
            K[i][r] = masks[r] @ F
    D = I.copy()
    for i in range(S):
        for r in range(R):
            if fam.b[i] != 0.0:
                D = D + dt * fam.b[i] * K[i][r]
    return D


def prk_step_apply(L, dt: float, fam: PerkFamily, member_of_cell: np.ndarray, U: np.ndarray):
    """The same partitioned RK step applied to one vector U_n (L may be a sparse matrix)."""
    R = len(fam.E)
    A = [dense_A(fam.c, fam.a_sub[r]) for r in range(R)]
    masks = [(member_of_cell == r).astype(float) for r in range(R)]
    K = [[None] * R for _ in range(fam.S)]
    for i in range(fam.S):
        stage = U.copy()
        for j in range(i):
            for k in range(R):
                if A[k][i, j] != 0.0:
                    stage = stage + dt * A[k][i, j] * K[j][k]
        F = L @ stage
        for r in range(R):
            K[i][r] = masks[r] * F
    out = U.copy()
    for i in range(fam.S):
        for r in range(R):
            if fam.b[i] != 0.0:
                out = out + dt * fam.b[i] * K[i][r]
    return out


def _sparse_upwind(dx):
    import scipy.sparse as sp
    N = len(dx)
    rows = np.concatenate([np.arange(N), np.arange(N)])
    cols = np.concatenate([np.arange(N), (np.arange(N) - 1) % N])
    vals = np.concatenate([-1.0 / dx, 1.0 / dx])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def cell_averages(edges: np.ndarray) -> np.ndarray:
    """Exact averages of 1 + sin(pi x)/2 over [edges[i], edges[i+1]]."""
    xl, xr = edges[:-1], edges[1:]
    return 1.0 + 0.5 * (np.cos(np.pi * xl) - np.cos(np.pi * xr)) / (np.pi * (xr - xl))


def total_variation(U: np.ndarray) -> float:
    return float(np.sum(np.abs(np.roll(U, -1) - U)))


def refined_grid(n_coarse_total: int, alpha: float):
    """Grid on (-1,1): cells of size 2/n_coarse_total in (-1,-0.5] and [0.5,1), cells of size
    (2/n_coarse_total)/alpha in [-0.5,0.5].  Returns (edges, is_fine)."""
    dx1 = 2.0 / n_coarse_total
    n_side = int(round(0.5 / dx1))
    n_fine = int(round(1.0 / (dx1 / alpha)))
    left = -1.0 + dx1 * np.arange(n_side + 1)
    mid = -0.5 + (1.0 / n_fine) * np.arange(1, n_fine + 1)
    right = 0.5 + dx1 * np.arange(1, n_side + 1)
    edges = np.concatenate([left, mid, right])
    edges[-1] = 1.0
    is_fine = np.zeros(len(edges) - 1, dtype=bool)
    is_fine[n_side:n_side + n_fine] = True
    return edges, is_fine


def tv_increase(fam: PerkFamily, n_coarse_total: int, alpha: float, dt: float) -> float:
    edges, is_fine = refined_grid(n_coarse_total, alpha)
    dx = np.diff(edges)
    L = _sparse_upwind(dx)
    member = np.where(is_fine, 1, 0)
    U0 = cell_averages(edges)
    U1 = prk_step_apply(L, dt, fam, member, U0)
    tv0 = total_variation(U0)
    return (total_variation(U1) - tv0) / tv0
