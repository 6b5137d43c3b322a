"""GPU spectrum estimation (Sec. 4.1 steps 3-4): the directional derivative of the right-hand
side by central differences against the oracle's dual-number tangent (Euler) and against central
differences of the oracle's right-hand side (Navier-Stokes), the two-pass Gram-Schmidt step
against numpy, and a full-dimension Arnoldi factorisation of the Jacobian of a 2:1 mesh (products
by central differences, exact forward or exact transposed products) whose eigenvalues match the oracle's dense Jacobian spectrum (tangent columns, numpy eigenvalues)."""
import numpy as np
import pytest
import torch

import perk_inputs as pin
from oracle import dgsem as od
from oracle import perk_coeffs as pc

pytestmark = pytest.mark.gpu


def _mesh_2level_small():
    m = pin.uniform_mesh(2, (4, 4), (0, 0), (1, 1), 0)
    sel = [r for r, (l, i, j, k) in enumerate(m.leaves.tolist()) if 1 <= i < 3 and 1 <= j < 3]
    m.leaves = pin.refine_leaves(m.leaves, 2, sel)
    return m


def _state(o, seed):
    # discontinuous across faces (nodal perturbation), so that no HLL wave-speed minimum or
    # maximum sits at a tie, where the flux is not differentiable and differences see both sides
    x = o.node_coords().transpose(1, 0, 2)
    u = pin.smooth_random_state(x, o.dim, seed).transpose(1, 0, 2).copy()
    rng = np.random.default_rng(seed)
    return u * (1 + 0.01 * rng.standard_normal(u.shape))


def _solver(mesh, N, **kw):
    from paper_2403_05144_amd import PerkSolver
    lmax = int(np.asarray(mesh.leaves)[:, 0].max())
    return PerkSolver(mesh, N - 1, pc.perk2_family([4, 8]), [0] * lmax + [1], **kw)


@pytest.mark.parametrize("N", [3, 4])
def test_fd_directional_derivative_euler(N):
    mesh = _mesh_2level_small()
    o = od.Oracle(mesh, N)
    u = _state(o, 3)
    rng = np.random.default_rng(5)
    du = rng.standard_normal(u.shape)
    _, t_ora = o.rhs_jvp(u, du)
    s = _solver(mesh, N, capacity=2 * mesh.leaves.shape[0])      # padding slots present
    us, vs = s.to_slot(u), s.to_slot(du)
    out = torch.zeros_like(us)
    s.jvp_fd_slot(us, vs, out, 1e-6)
    t_gpu = s.to_leaf(out).cpu().numpy()
    err = np.max(np.abs(t_gpu - t_ora)) / np.max(np.abs(t_ora))
    print(f"FD directional derivative N={N}: rel err {err:.2e}", flush=True)
    assert err <= 1e-7
    # padding slots read zero
    pad = out.view(s.nv, -1, s.Nd)[:, s.n_elements:, :]
    assert torch.count_nonzero(pad).item() == 0


def test_fd_directional_derivative_navier_stokes():
    # the oracle has no tangent of the viscous operator: central differences of its right-hand
    # side with the same step (both O(h^2) from the same derivative)
    mesh = _mesh_2level_small()
    mu = 1e-2
    o = od.Oracle(mesh, 4, viscous=True, mu=mu)
    u = _state(o, 4)
    rng = np.random.default_rng(6)
    du = rng.standard_normal(u.shape)
    eps = 1e-6
    h = eps * np.linalg.norm(u) / np.linalg.norm(du)
    t_ora = (o.rhs(u + h * du) - o.rhs(u - h * du)) / (2 * h)
    s = _solver(mesh, 4, equations=1, mu=mu)
    us, vs = s.to_slot(u), s.to_slot(du)
    out = torch.zeros_like(us)
    s.jvp_fd_slot(us, vs, out, eps)
    t_gpu = s.to_leaf(out).cpu().numpy()
    err = np.max(np.abs(t_gpu - t_ora)) / np.max(np.abs(t_ora))
    print(f"FD directional derivative NS: rel err {err:.2e}", flush=True)
    assert err <= 1e-6


def test_gram_schmidt_step_against_numpy():
    s = _solver(_mesh_2level_small(), 4)
    n, k = 5000, 37
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    w = rng.standard_normal(n)
    V = torch.tensor(np.ascontiguousarray(Q.T), dtype=torch.float64, device="cuda")
    wd = torch.tensor(w, dtype=torch.float64, device="cuda")
    from paper_2403_05144_amd import _lib as L
    import ctypes
    nd = ctypes.c_int64()
    assert s.lib.pe_orthogonalize_scratch(k, ctypes.byref(nd)) == 0
    scratch = torch.empty(nd.value, dtype=torch.float64, device="cuda")
    h = s.orthogonalize(V, k, wd, scratch)
    proj = Q.T @ w
    r = w - Q @ proj
    np.testing.assert_allclose(h[:k], proj, rtol=1e-12, atol=1e-12 * np.abs(proj).max())
    assert abs(h[k] - np.linalg.norm(r)) <= 1e-12 * np.linalg.norm(r)
    got = wd.cpu().numpy()
    np.testing.assert_allclose(got, r / np.linalg.norm(r), atol=1e-12)
    assert np.max(np.abs(Q.T @ got)) <= 1e-13


@pytest.mark.parametrize("op", ["jvp", "vjp", "fd"])
def test_full_arnoldi_reproduces_the_dense_spectrum(op):
    from paper_2403_05144_amd import coeffs
    mesh = _mesh_2level_small()
    N = 3
    o = od.Oracle(mesh, N)
    u = _state(o, 8)
    n = u.size
    J = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        J[:, c] = o.rhs_jvp(u, e.reshape(u.shape))[1].ravel()
    lam = np.linalg.eigvals(J)
    s = _solver(mesh, N)
    us = s.to_slot(u)
    H = coeffs.arnoldi(s, us, n, op=op, eps=1e-7)
    ritz = np.linalg.eigvals(H[: H.shape[1], : H.shape[1]])
    rho = np.abs(lam).max()
    print(f"arnoldi {op}: {H.shape[1]} steps for n = {n}, spectral radius {rho:.3f}", flush=True)
    # the Krylov space closes a few steps early: the zero eigenvalue of the conserved
    # quantities is repeated (one per variable), so no start vector reaches every direction
    assert n - 8 <= H.shape[1] <= n
    tol = (1e-4 if op == "fd" else 1e-6) * rho
    d1 = max(np.min(np.abs(ritz - l)) for l in lam)
    d2 = max(np.min(np.abs(lam - r)) for r in ritz)
    assert d1 <= tol and d2 <= tol, (d1, d2, tol)
