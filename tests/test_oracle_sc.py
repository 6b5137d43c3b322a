"""Pins of the oracle's subcell shock capturing (Hennemann et al., used by the paper for its
inviscid runs, Sec. 4.1 and Sec. 7.2.1): the modal transform against numpy's Legendre
polynomials; the energy indicator on states whose modal content is known in closed form; the
blending factor's sigmoid at its midpoint, its cap and its cut-off; alpha = 0 giving the plain
DGSEM bitwise; alpha = 1 giving the first-order finite-volume scheme on the LGL subcells,
assembled here node by node; conservation and freestream on a 2:1 forest with the indicator's
own alpha."""
import math

import numpy as np
import pytest

import perk_inputs as pin
from oracle import dgsem as od

GAMMA = 1.4


def _T(N, a=0.5, c=1.8):
    return a * 10.0 ** (-c * N ** 0.25)


def _phi(k, x):
    """L2-orthonormal Legendre polynomial of degree k on [-1, 1] (numpy's Legendre series)."""
    coef = np.zeros(k + 1)
    coef[k] = 1.0
    return math.sqrt(k + 0.5) * np.polynomial.legendre.legval(x, coef)


def _state_from_rho(o, rho_fn):
    x = o.node_coords()                       # [e, d, node]
    u = np.zeros(o.shape)
    rho = rho_fn(*[x[:, d] for d in range(o.dim)])
    u[:, 0] = rho
    u[:, 1] = 0.1 * rho
    u[:, -1] = 2.5 + 0.5 * 0.01 * rho
    return u


@pytest.mark.parametrize("N", [3, 4])
def test_modal_transform_is_the_orthonormal_legendre_one(N):
    mesh = pin.uniform_mesh(2, (1, 1), (-1, -1), (1, 1), 0)
    o = od.Oracle(mesh, N)
    x, _, _ = od.lgl(N)
    _, _, Vinv = o.sc_indicator(np.ones(o.shape))
    for k in range(N):
        np.testing.assert_allclose(Vinv @ _phi(k, x), np.eye(N)[k], atol=1e-13)


@pytest.mark.parametrize("N", [3, 4])
def test_energy_indicator_closed_forms(N):
    # one element on [-1, 1]^2, so physical and reference coordinates coincide
    mesh = pin.uniform_mesh(2, (1, 1), (-1, -1), (1, 1), 0)
    o = od.Oracle(mesh, N)
    p = N - 1
    # degree <= p - 2 in each direction (p = 3: bilinear, p = 2: constant) -> no energy in the top
    # two layers
    lin = 1.0 if p >= 3 else 0.0
    E, _, _ = o.sc_indicator(_state_from_rho(o, lambda x, y: 1.0 + lin * (0.2 * x + 0.1 * y + 0.05 * x * y)))
    assert abs(E[0]) < 1e-14
    eps = 0.3
    # 1 = 2 phi_0(x) phi_0(y); eps phi_p(x) = sqrt(2) eps phi_p(x) phi_0(y): total 4 + 2 eps^2,
    # of which 2 eps^2 in the highest layer -> E = eps^2 / (2 + eps^2)
    E, _, _ = o.sc_indicator(_state_from_rho(o, lambda x, y: 1.0 + eps * _phi(p, x)))
    assert abs(E[0] - eps ** 2 / (2 + eps ** 2)) < 1e-14
    # the same in the second-highest layer (along y): the second ratio, same value
    E, _, _ = o.sc_indicator(_state_from_rho(o, lambda x, y: 1.0 + eps * _phi(p - 1, y)))
    assert abs(E[0] - eps ** 2 / (2 + eps ** 2)) < 1e-14
    # both layers: E = max(E_1, E_2) with E_1 = 2 e1^2 / (4 + 2 e1^2 + 2 e2^2), E_2 = 2 e2^2 / (4 + 2 e2^2)
    e1, e2 = 0.1, 0.4
    E, _, _ = o.sc_indicator(_state_from_rho(o, lambda x, y: 1.0 + e1 * _phi(p, y) + e2 * _phi(p - 1, x)))
    ref = max(2 * e1 ** 2 / (4 + 2 * e1 ** 2 + 2 * e2 ** 2), 2 * e2 ** 2 / (4 + 2 * e2 ** 2))
    assert abs(E[0] - ref) < 1e-14


@pytest.mark.parametrize("N", [3, 4])
def test_blending_factor_sigmoid(N):
    mesh = pin.uniform_mesh(2, (1, 1), (-1, -1), (1, 1), 0)
    o = od.Oracle(mesh, N)
    p = N - 1
    T = _T(N)
    # E = T exactly: the sigmoid's midpoint, alpha = 1/2
    eps = math.sqrt(2 * T / (1 - T))
    u = _state_from_rho(o, lambda x, y: 1.0 + eps * _phi(p, x))
    o.set_shock_capturing(True, alpha_max=1.0, alpha_min=0.001)
    E, a, _ = o.sc_indicator(u)
    assert abs(E[0] - T) < 1e-15
    assert abs(a[0] - 0.5) < 1e-9
    # capped at alpha_max
    o.set_shock_capturing(True, alpha_max=0.3, alpha_min=0.001)
    assert o.sc_indicator(u)[1][0] == 0.3
    # far above the threshold: alpha_max; far below: cut to 0
    o.set_shock_capturing(True, alpha_max=0.5, alpha_min=0.001)
    assert o.sc_indicator(_state_from_rho(o, lambda x, y: 1.0 + 0.5 * _phi(p, x)))[1][0] == 0.5
    assert o.sc_indicator(_state_from_rho(o, lambda x, y: 1.0 + 1e-3 * _phi(p, x)))[1][0] == 0.0
    # the cut-off: alpha below alpha_min is 0, just above it is kept
    s = math.log((1 - 1e-4) / 1e-4)
    E_min = T - T / s * math.log(1 / 0.001 - 1)              # alpha(E_min) = alpha_min
    for f, expect_zero in ((0.99, True), (1.01, False)):
        Et = E_min * f
        e = math.sqrt(2 * Et / (1 - Et))
        a = o.sc_indicator(_state_from_rho(o, lambda x, y: 1.0 + e * _phi(p, x)))[1][0]
        assert (a == 0.0) == expect_zero
        if not expect_zero:
            assert abs(a - 1 / (1 + math.exp(-s / T * (Et - T)))) < 1e-12


def _forest_state(o, seed, amp=0.03, rough_share=1.0):
    """Smooth seeded state with a nodal perturbation of relative size amp on a share of the
    elements (the others stay smooth)."""
    x = o.node_coords().transpose(1, 0, 2)
    u = pin.smooth_random_state(x, o.dim, seed).transpose(1, 0, 2).copy()
    rng = np.random.default_rng(seed)
    rough = rng.random(u.shape[0]) < rough_share
    return u * (1 + amp * rough[:, None, None] * rng.standard_normal(u.shape))


def test_alpha_zero_is_the_plain_dgsem():
    mesh = pin.random_forest_2d(5, n_root=3, max_level=2)
    o = od.Oracle(mesh, 4)
    u = _forest_state(o, 11)
    plain = o.rhs(u)
    o.set_shock_capturing(True, alpha_fixed=0.0)
    assert np.array_equal(o.rhs(u), plain)


@pytest.mark.parametrize("N", [3, 4])
def test_alpha_one_is_finite_volumes_on_the_lgl_subcells(N):
    # uniform periodic mesh: with alpha = 1 every node is a finite-volume cell of width
    # (h/2) w_i per direction, and every interface flux -- inside an element between
    # neighbouring nodes, and at element faces between the two coinciding end nodes -- is the
    # HLL flux of the two adjacent node values; assembled here node by node
    mesh = pin.uniform_mesh(2, (3, 2), (0.0, 0.0), (1.5, 1.0), 0)
    o = od.Oracle(mesh, N)
    u = _forest_state(o, 7)
    o.set_shock_capturing(True, alpha_fixed=1.0)
    got = o.rhs(u)
    _, w, _ = od.lgl(N)
    leaves = mesh.leaves
    index = {(int(l[1]), int(l[2])): e for e, l in enumerate(leaves)}
    nx, ny = mesh.n_root
    h = [(mesh.hi[d] - mesh.lo[d]) / mesh.n_root[d] for d in range(2)]
    ref = np.zeros(o.shape)
    for e, l in enumerate(leaves):
        ci, cj = int(l[1]), int(l[2])
        for j in range(N):
            for i in range(N):
                nd = i + N * j
                for d in range(2):
                    a = (i, j)[d]
                    # neighbour nodes along d (across the element face at the ends)
                    def node(ee, ii, jj):
                        return u[ee, :, ii + N * jj]
                    if a < N - 1:
                        nxt = node(e, i + (d == 0), j + (d == 1))
                    else:
                        c = [ci, cj]; c[d] = (c[d] + 1) % (nx, ny)[d]
                        ii, jj = (0, j) if d == 0 else (i, 0)
                        nxt = node(index[tuple(c)], ii, jj)
                    if a > 0:
                        prv = node(e, i - (d == 0), j - (d == 1))
                    else:
                        c = [ci, cj]; c[d] = (c[d] - 1) % (nx, ny)[d]
                        ii, jj = (N - 1, j) if d == 0 else (i, N - 1)
                        prv = node(index[tuple(c)], ii, jj)
                    me = u[e, :, nd]
                    Fp = od.hll_flux(2, GAMMA, me, nxt, d)
                    Fm = od.hll_flux(2, GAMMA, prv, me, d)
                    ref[e, :, nd] -= (Fp - Fm) / (0.5 * h[d] * w[a])
    scale = np.max(np.abs(ref), axis=(0, 2))
    for v in range(o.nv):
        assert np.max(np.abs(got[:, v] - ref[:, v])) <= 1e-12 * scale[v]


@pytest.mark.parametrize("fixed", [None, 0.37])
def test_blended_operator_conserves_and_keeps_freestream(fixed):
    mesh = pin.random_forest_2d(9, n_root=3, max_level=2)
    o = od.Oracle(mesh, 4)
    u = _forest_state(o, 13, amp=0.05, rough_share=0.5)
    o.set_shock_capturing(True, alpha_max=0.5, alpha_min=0.001, alpha_fixed=fixed)
    if fixed is None:
        _, a, _ = o.sc_indicator(u)
        assert np.count_nonzero(a) > 0 and np.count_nonzero(a == 0) > 0, a   # both kinds of element
    du = o.rhs(u)
    _, w, _ = od.lgl(4)
    W = np.outer(w, w).ravel()
    vol = np.prod(o.element_sizes(), axis=1) / 4.0
    tot = np.einsum("e,evn,n->v", vol, du, W)
    mag = np.einsum("e,evn,n->v", vol, np.abs(du), W)
    assert np.all(np.abs(tot) <= 1e-13 * mag), tot / mag
    # freestream: a constant state stays constant whatever alpha
    c = np.zeros(o.shape)
    c[:, 0], c[:, 1], c[:, 2], c[:, 3] = 1.2, 0.3, -0.2, 3.0
    assert np.max(np.abs(o.rhs(c))) < 1e-12
