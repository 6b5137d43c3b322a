"""Pins of the oracle's adaptation and projection (CPU): balance, honoured flags, complete
families only, conservation, exact interpolation of polynomials."""
import numpy as np
import pytest

import perk_inputs as pin
from oracle import amr
from oracle import dgsem as od


def _poly_state(o, deg):
    x = o.node_coords()
    u = np.zeros(o.shape)
    u[:, 0] = 1.0 + 0.1 * x[:, 0] ** deg + 0.05 * x[:, 1]
    u[:, 1] = 0.2 * x[:, 1] ** deg
    u[:, 2] = -0.1 * x[:, 0] * x[:, 1] ** (deg - 1)
    u[:, 3] = 3.0 + 0.3 * x[:, 0]
    return u


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_adapt_rules_and_conservation(seed):
    mesh = pin.random_forest_2d(seed, n_root=4, max_level=2)
    o = od.Oracle(mesh, 4)
    rng = np.random.default_rng(seed)
    flags = rng.choice([-1, 0, 1], size=o.n_elements, p=[0.5, 0.3, 0.2]).astype(np.int8)
    new, plan = amr.adapt(mesh.leaves, flags, 0, 3, 2, mesh.n_root)
    m2 = pin.MeshDesc(2, mesh.n_root, mesh.lo, mesh.hi, new)
    o2 = od.Oracle(m2, 4)          # raises unless the result is a 2:1-balanced cover
    lev = mesh.leaves[:, 0]
    newset = {tuple(r[:3]) for r in new.tolist()}
    for e, r in enumerate(mesh.leaves.tolist()):
        l, i, j = r[:3]
        if flags[e] > 0 and l < 3:
            # refined: its children exist
            assert all((l + 1, 2 * i + (m & 1), 2 * j + (m >> 1)) in newset for m in range(4))
        if (l - 1, i >> 1, j >> 1) in newset:
            # coarsened: every sibling was a leaf flagged -1
            sib = [(l, 2 * (i >> 1) + (m & 1), 2 * (j >> 1) + (m >> 1)) for m in range(4)]
            idx = {tuple(rr[:3]): k for k, rr in enumerate(mesh.leaves.tolist())}
            assert all(s in idx and flags[idx[s]] < 0 for s in sib)
    u = _poly_state(o, 3)
    u2 = amr.project(o, u, plan, 4)
    np.testing.assert_allclose(o2.integral(u2), o.integral(u), rtol=1e-13, atol=1e-13)


def test_refinement_interpolates_polynomials_exactly():
    mesh = pin.uniform_mesh(2, (3, 3), (0, 0), (1, 1), 0)
    o = od.Oracle(mesh, 4)
    u = _poly_state(o, 3)
    new, plan = amr.adapt(mesh.leaves, np.ones(o.n_elements, np.int8), 0, 1, 2, mesh.n_root)
    o2 = od.Oracle(pin.MeshDesc(2, mesh.n_root, mesh.lo, mesh.hi, new), 4)
    u2 = amr.project(o, u, plan, 4)
    np.testing.assert_allclose(u2, _poly_state(o2, 3), atol=1e-13)


def test_coarsening_keeps_constants_and_linears():
    mesh = pin.uniform_mesh(2, (2, 2), (0, 0), (1, 1), 1)
    o = od.Oracle(mesh, 4)
    u = _poly_state(o, 1)
    new, plan = amr.adapt(mesh.leaves, -np.ones(o.n_elements, np.int8), 0, 1, 2, mesh.n_root)
    assert len(new) == 4 and np.all(new[:, 0] == 0)
    o2 = od.Oracle(pin.MeshDesc(2, mesh.n_root, mesh.lo, mesh.hi, new), 4)
    np.testing.assert_allclose(amr.project(o, u, plan, 4), _poly_state(o2, 1), atol=1e-13)


def test_ripple_refinement_keeps_balance():
    # refining a leaf next to a coarser one forces the coarser one to refine (2:1 balance)
    mesh = pin.uniform_mesh(2, (4, 4), (0, 0), (1, 1), 0)
    mesh.leaves = pin.refine_leaves(mesh.leaves, 2, [5])
    o = od.Oracle(mesh, 3)
    flags = np.zeros(o.n_elements, np.int8)
    fine = [k for k, r in enumerate(mesh.leaves.tolist()) if r[0] == 1]
    flags[fine[0]] = 1
    new, plan = amr.adapt(mesh.leaves, flags, 0, 2, 2, mesh.n_root)
    od.Oracle(pin.MeshDesc(2, mesh.n_root, mesh.lo, mesh.hi, new), 3)
    assert (new[:, 0] == 2).sum() == 4 and len(new) > len(mesh.leaves) + 3


def test_indicator_of_linear_density():
    # rho = 1 + a x: |grad rho| = a everywhere, eta = h a / max rho
    mesh = pin.uniform_mesh(2, (4, 4), (0, 0), (1, 1), 0)
    o = od.Oracle(mesh, 4)
    x = o.node_coords()
    u = np.zeros(o.shape)
    u[:, 0] = 1 + 0.5 * x[:, 0]
    u[:, 3] = 2.5
    eta = amr.indicator(o, u)
    expect = 0.25 * 0.5 / np.max(u[:, 0], axis=1)
    np.testing.assert_allclose(eta, expect, rtol=1e-13)


# ------------------------------------------------------------------ Loehner indicator (Sec. 7.1.1)
def test_lohner_estimate_closed_forms():
    from oracle.amr import lohner_estimate
    # a peak (0, 1, 0): second difference 2 over 1 + 1 + f (0 + 2 + 0)
    assert lohner_estimate(0.0, 1.0, 0.0, 0.2) == 2.0 / 2.4
    # equal spacing of values (linear data) and constants give 0
    assert lohner_estimate(1.0, 2.0, 3.0, 0.2) == 0.0
    assert lohner_estimate(5.0, 5.0, 5.0, 0.2) == 0.0
    assert lohner_estimate(0.0, 0.0, 0.0, 0.2) == 0.0           # vanishing denominator
    rng = np.random.default_rng(0)
    for _ in range(200):
        um, u0, up = rng.standard_normal(3)
        e = lohner_estimate(um, u0, up, 0.2)
        assert 0.0 <= e <= 1.0                                   # |a - 2b + c| <= |a - b| + |b - c|
        assert abs(lohner_estimate(up, u0, um, 0.2) - e) <= 1e-15                     # stencil reflection
        assert abs(lohner_estimate(3.7 * um, 3.7 * u0, 3.7 * up, 0.2) - e) <= 1e-15   # degree-0 homogeneous
        assert lohner_estimate(um, u0, up, 0.0) >= e             # f_wave only damps


def test_lohner_indicator_on_the_shear_layer():
    # element indicator = max over interior nodes of every coordinate line; elements far from the
    # shear layers see a smooth v_x (small values), the layers (width 1/80) saturate it
    import perk_inputs as pin
    from oracle.amr import lohner_indicator, lohner_estimate, primitive_variable
    mesh = pin.uniform_mesh(2, (8, 8), (0, 0), (1, 1), 0)
    o = od.Oracle(mesh, 4)
    x = o.node_coords().transpose(1, 0, 2)
    u = pin.shear_layer(x[0], x[1]).transpose(1, 0, 2).copy()
    eta = lohner_indicator(o, u, var=1, f_wave=0.2)
    yc = np.array([(j + 0.5) / 8 for (_, i, j, _) in mesh.leaves.tolist()])
    near = np.abs(np.abs(yc - 0.5) - 0.25) < 0.07
    assert eta[near].min() > 3 * eta[~near].max()
    # brute force on one element: every interior node of every line, both directions
    e = int(np.argmax(eta))
    v = primitive_variable(u, 1, 2)[e].reshape(4, 4)         # [j, i]
    best = max(max(lohner_estimate(v[j, i - 1], v[j, i], v[j, i + 1], 0.2) for j in range(4) for i in (1, 2)),
               max(lohner_estimate(v[j - 1, i], v[j, i], v[j + 1, i], 0.2) for j in (1, 2) for i in range(4)))
    assert eta[e] == best
    # primitive variables: velocity and pressure of the initial state
    np.testing.assert_allclose(primitive_variable(u, 3, 2), 100.0 / 1.4, rtol=1e-14)
