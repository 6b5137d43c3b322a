"""Pins of the oracle's tangent-linear and adjoint Euler operator and partitioned step
(forward-mode dual numbers, adjoint assembled column by column):
  * the value part of the dual evaluation equals the plain evaluation bitwise;
  * tangents agree with central finite differences of the plain evaluation to 2e-9 relative
    at the best of three steps (states discontinuous across faces, so the HLL wave-speed
    minimum and maximum are away from ties);
  * discrete conservation on a periodic mesh (the quadrature-weighted sum of F(u) vanishes for
    every u) makes F'(u)^T M 1_v vanish for each conserved variable v;
  * at a constant state every constant perturbation is a steady state (free-stream
    preservation), so its tangent vanishes;
  * the adjoint of the step satisfies <lam, Phi'(u) du> = <Phi'(u)^T lam, du> and matches
    finite differences of <lam, Phi(u)>."""
import numpy as np

import perk_inputs as pin
from oracle import dgsem as od
from oracle import perk_coeffs as pc


def _setup(dim=2, N=3, seed=3):
    if dim == 2:
        mesh = pin.random_forest_2d(5, n_root=3, max_level=2)
    else:
        mesh = pin.uniform_mesh(3, (2, 2, 2), (0.0,) * 3, (1.0,) * 3, 0)
        mesh.leaves = pin.refine_leaves(mesh.leaves, 3, [0])
    o = od.Oracle(mesh, N)
    x = o.node_coords().transpose(1, 0, 2)
    if dim == 2:
        u = pin.smooth_random_state(x, 2, 11).transpose(1, 0, 2).copy()
    else:
        u = pin.taylor_green(2 * np.pi * x[0], 2 * np.pi * x[1], 2 * np.pi * x[2], mach=0.3).transpose(1, 0, 2).copy()
    rng = np.random.default_rng(seed)
    u = u * (1 + 0.01 * rng.standard_normal(u.shape))     # discontinuous across faces
    return mesh, o, u, rng


def _weights(o):
    _, w, _ = od.lgl(o.N)
    W = w
    for _ in range(o.dim - 1):
        W = np.multiply.outer(w, W).reshape(-1)
    jac = np.prod(o.element_sizes() / 2.0, axis=1)
    return jac[:, None] * W[None, :]


def test_dual_values_equal_plain_evaluation():
    mesh, o, u, rng = _setup()
    f, _ = o.rhs_jvp(u, rng.standard_normal(o.shape))
    assert np.array_equal(f, o.rhs(u))
    import json, os
    with open(os.path.join(os.path.dirname(__file__), "golden", "perk3_4_8_16_disk.json")) as fh:
        fam = pc.PerkFamily.from_json(json.load(fh))
    member = np.asarray(od.member_of_levels_paper_rule(np.arange(3), 3))[mesh.leaves[:, 0]]
    u1, _ = o.prk_step_jvp(u, rng.standard_normal(o.shape), 1e-3, fam, member)
    assert np.array_equal(u1, o.prk_step(u, 1e-3, fam, member))


def test_rhs_tangent_matches_central_differences_2d_and_3d():
    for dim, N in ((2, 3), (2, 4), (3, 3)):
        mesh, o, u, rng = _setup(dim, N)
        du = rng.standard_normal(o.shape) * np.abs(u)
        _, t = o.rhs_jvp(u, du)
        errs = []
        for eps in (1e-5, 1e-6, 1e-7):
            fd = (o.rhs(u + eps * du) - o.rhs(u - eps * du)) / (2 * eps)
            errs.append(np.max(np.abs(fd - t)) / np.max(np.abs(t)))
        # the best step is limited by truncation above and round-off below; a step that
        # straddles a wave-speed switch of some face node only spoils that step
        assert min(errs) < 2e-9, (dim, N, errs)


def test_adjoint_annihilates_conserved_weights():
    mesh, o, u, rng = _setup()
    W = _weights(o)
    scale = np.max(np.abs(o.rhs_vjp(u, rng.standard_normal(o.shape))))
    for v in range(o.nv):
        m = np.zeros(o.shape)
        m[:, v] = W
        g = o.rhs_vjp(u, m)
        assert np.max(np.abs(g)) <= 1e-12 * scale * np.max(W), (v, np.max(np.abs(g)))


def test_tangent_of_freestream_vanishes():
    mesh, o, u, rng = _setup()
    c = np.zeros(o.shape)
    c[:, 0], c[:, 1], c[:, 2], c[:, 3] = 1.1, 0.3, -0.2, 2.5
    dc = np.zeros(o.shape)
    dc[:, 0], dc[:, 1], dc[:, 2], dc[:, 3] = 0.7, -0.4, 0.9, 0.1
    _, t = o.rhs_jvp(c, dc)
    _, tu = o.rhs_jvp(u, dc)
    assert np.max(np.abs(t)) <= 1e-12 * np.max(np.abs(tu))


def test_step_adjoint_transpose_and_finite_differences():
    mesh, o, u, rng = _setup()
    fam = pc.perk2_family([4, 8])
    member = np.asarray(od.member_of_levels_paper_rule(np.arange(3), 2))[mesh.leaves[:, 0]]
    dt = 2e-3
    lam = rng.standard_normal(o.shape)
    du = rng.standard_normal(o.shape) * np.abs(u)
    g = o.prk_step_vjp(u, lam, dt, fam, member)
    _, t = o.prk_step_jvp(u, du, dt, fam, member)
    assert abs(np.sum(lam * t) - np.sum(g * du)) <= 1e-12 * np.sum(np.abs(lam * t))
    errs = []
    for eps in (1e-5, 1e-6, 1e-7):
        fd = (np.sum(lam * o.prk_step(u + eps * du, dt, fam, member)) -
              np.sum(lam * o.prk_step(u - eps * du, dt, fam, member))) / (2 * eps)
        errs.append(abs(fd - np.sum(g * du)) / np.sum(np.abs(lam * t)))
    assert min(errs) <= 1e-9, errs
