"""Subcell shock capturing on the GPU (pe_set_shock_capturing, 2D Euler; Hennemann et al., used by
the paper for its inviscid runs, Sec. 4.1 and 7.2.1) against the oracle: the indicator's sigmoid
per element (refinement indicator kind), the blended right-hand side on 2:1 forests at p = 2 and 3
(both 2D p=3 launch shapes), partitioned P-ERK3 steps; alpha capped at 0 equal to the plain
operator; graph replay equal to eager launches; the tangent and adjoint refused.  States: the
paper's Kelvin-Helmholtz initial condition (its shear layers are under-resolved on these meshes,
so elements with alpha = 0, alpha in between and alpha at the cap all occur).  Bar: 1e-12 of the
flux scale per conserved variable, as the other parity tests; indicator values 1e-11 absolute
(the sigmoid's slope, up to 1600 at p = 3, scales the rounding of the modal energies)."""
import numpy as np
import pytest
import torch

import perk_inputs as pin
from oracle import dgsem as od
from oracle import perk_coeffs as pc

pytestmark = pytest.mark.gpu
TOL = 1e-12
AMAX, AMIN = 0.5, 0.001


def _kh_state(o, k=1):
    """The paper's Kelvin-Helmholtz state, compressed k times in both directions (k layers of
    each sign per unit length: sharper layers for finer meshes; periodic on [-1, 1]^2)."""
    x = o.node_coords().transpose(1, 0, 2)
    return pin.kelvin_helmholtz_paper(k * x[0], k * x[1]).transpose(1, 0, 2).copy()


def _flux_scale(o, u):
    gam = 1.4
    rho = u[:, 0]
    vel = u[:, 1:3] / rho[:, None]
    p = (gam - 1) * (u[:, 3] - 0.5 * rho * np.sum(vel * vel, axis=1))
    jmax = np.max(2.0 / o.element_sizes(), axis=1)[:, None]
    out = []
    for d in range(2):
        f = [u[:, 1 + d], u[:, 1] * vel[:, d] + (p if d == 0 else 0), u[:, 2] * vel[:, d] + (p if d == 1 else 0),
             (u[:, 3] + p) * vel[:, d]]
        out.append([np.max(jmax * np.abs(fv)) for fv in f])
    return np.max(np.array(out), axis=0)


def _close(g, r, scale, tol=TOL):
    return all(np.max(np.abs(g[:, v] - r[:, v])) <= tol * max(np.max(np.abs(r[:, v])), scale[v])
               for v in range(r.shape[1]))


def _worst(g, r, scale):
    return max(np.max(np.abs(g[:, v] - r[:, v])) / max(np.max(np.abs(r[:, v])), scale[v]) for v in range(r.shape[1]))


def _alpha_checked(o, u):
    """The oracle's alpha with the test's parameters, after checking that no element sits within
    1e-9 (relative) of the cut-off or the cap, where two roundings could decide differently."""
    o.set_shock_capturing(True, alpha_max=1.0, alpha_min=0.0)
    _, raw, _ = o.sc_indicator(u)
    for edge in (AMIN, AMAX):
        assert np.all(np.abs(raw - edge) > 1e-9 * edge), "an element sits on a decision edge"
    o.set_shock_capturing(True, alpha_max=AMAX, alpha_min=AMIN)
    _, a, _ = o.sc_indicator(u)
    return a


def _solver(mesh, N, fam=None, mol=None):
    from paper_2403_05144_amd import PerkSolver
    lmax = int(mesh.leaves[:, 0].max())
    fam = fam or pc.perk2_family([4, 8])
    return PerkSolver(mesh, N - 1, fam, mol if mol is not None else [0] * (lmax + 1))


CASES = {
    "kh_16x16_p3": (lambda: pin.uniform_mesh(2, (16, 16), (-1, -1), (1, 1), 0), 4, 1),
    "kh_forest_p3": (lambda: pin.random_forest_2d(4, n_root=8, max_level=2), 4, 1),
    "kh_forest_p2": (lambda: pin.random_forest_2d(6, n_root=8, max_level=2), 3, 1),
    # above 2048 elements: the one-wave 2D p=3 body, four elements per block (layers compressed
    # 8 times to stay sharp); 3511 elements leave the last block ragged
    "kh_mid_forest_p3": (lambda: pin.random_forest_2d(3, n_root=28, max_level=2, p_refine=0.3), 4, 8),
    "kh_large_forest_p3": (lambda: pin.random_forest_2d(3, n_root=48, max_level=2, p_refine=0.35), 4, 8),
}


@pytest.mark.parametrize("N", [3, 4])
def test_indicator_matches_oracle(N):
    mesh = pin.random_forest_2d(4, n_root=8, max_level=2)
    o = od.Oracle(mesh, N)
    u = _kh_state(o)
    o.set_shock_capturing(True, alpha_max=1.0, alpha_min=0.0)      # the plain sigmoid
    _, ref, _ = o.sc_indicator(u)
    s = _solver(mesh, N)
    s.set_indicator("hennemann_gassner", variable=0)
    s.set_state(u)
    eta = s.indicator()
    print(f"N={N}: sigmoid range {ref.min():.3e} .. {ref.max():.3e}, max |diff| {np.max(np.abs(eta - ref)):.2e}",
          flush=True)
    assert np.max(np.abs(eta - ref)) <= 1e-11


@pytest.mark.parametrize("case", list(CASES))
def test_blended_rhs_matches_oracle(case):
    mk, N, k = CASES[case]
    mesh = mk()
    o = od.Oracle(mesh, N)
    u = _kh_state(o, k)
    a = _alpha_checked(o, u)
    print(f"{case}: {len(a)} elements, alpha = 0: {np.sum(a == 0)}, capped: {np.sum(a == AMAX)}, "
          f"between: {np.sum((a > 0) & (a < AMAX))}", flush=True)
    assert np.sum(a == 0) > 0 and np.sum((a > 0) & (a < AMAX)) > 0
    ref = o.rhs(u)
    s = _solver(mesh, N)
    s.set_shock_capturing(True, alpha_max=AMAX, alpha_min=AMIN)
    g = s.rhs_leaf(u).cpu().numpy()
    sc = _flux_scale(o, u)
    assert _close(g, ref, sc), _worst(g, ref, sc)
    # the blend matters: the plain operator is far from it
    o.set_shock_capturing(False)
    assert not _close(g, o.rhs(u), sc, tol=1e-6)


def _perk3_family(E_list):
    th = np.linspace(0, 2 * np.pi, 200, endpoint=False)
    eigs = -1.0 + np.exp(1j * th)
    return pc.perk3_family(E_list, {E: pc.optimize_alpha(eigs, 3, E)[1] for E in E_list})


@pytest.mark.parametrize("N", [3, 4])
def test_perk3_steps_match_oracle(N):
    mesh = pin.random_forest_2d(4, n_root=8, max_level=2)
    o = od.Oracle(mesh, N)
    u0 = _kh_state(o)
    _alpha_checked(o, u0)
    fam = _perk3_family([3, 6])
    mol = od.member_of_levels_paper_rule(np.arange(3), 2)
    member = np.asarray(mol)[mesh.leaves[:, 0]]
    s = _solver(mesh, N, fam, mol)
    s.set_shock_capturing(True, alpha_max=AMAX, alpha_min=AMIN)
    s.set_state(u0)
    dt, n = 2e-4, 3
    u_ora = u0.copy()
    for _ in range(n):
        u_ora = o.prk_step(u_ora, dt, fam, member)
    s.step(dt, n)
    g = s.get_state().cpu().numpy()
    worst = max(np.max(np.abs(g[:, v] - u_ora[:, v])) / np.max(np.abs(u_ora[:, v])) for v in range(4))
    print(f"N={N}: {n} P-ERK3 steps, worst relative error {worst:.2e}", flush=True)
    assert worst <= TOL


def test_alpha_capped_at_zero_is_the_plain_operator():
    mesh = pin.random_forest_2d(4, n_root=8, max_level=2)
    o = od.Oracle(mesh, 4)
    u0 = _kh_state(o)
    outs = []
    for on in (False, True):
        s = _solver(mesh, 4, pc.perk2_family([4, 8]), [0, 0, 1])
        if on:
            s.set_shock_capturing(True, alpha_max=0.0, alpha_min=0.0)
        s.set_state(u0)
        s.step(2e-4, 3)
        outs.append(s.get_state().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_graph_replay_equals_eager():
    mesh = pin.random_forest_2d(4, n_root=8, max_level=2)
    o = od.Oracle(mesh, 4)
    u0 = _kh_state(o)
    outs = []
    for graph in (True, False):
        s = _solver(mesh, 4, pc.perk2_family([4, 8]), [0, 0, 1])
        s.set_shock_capturing(True, alpha_max=AMAX, alpha_min=AMIN)
        s.set_graph_replay(graph)
        s.set_state(u0)
        for _ in range(3):
            s.step(2e-4, 2)
            torch.cuda.synchronize()
        outs.append(s.get_state().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_tangent_and_adjoint_refused():
    from paper_2403_05144_amd import PerkError
    mesh = pin.random_forest_2d(4, n_root=8, max_level=2)
    o = od.Oracle(mesh, 4)
    u = _kh_state(o)
    s = _solver(mesh, 4)
    s.set_shock_capturing(True)
    us = s.to_slot(u)
    with pytest.raises(PerkError):
        s.jvp_into(us, us, torch.zeros_like(us))
    with pytest.raises(PerkError):
        s.vjp_into(us, us, torch.zeros_like(us))
    s.set_shock_capturing(False)
    s.jvp_into(us, us, torch.zeros_like(us))


def test_kh_adaptation_on_the_indicator_and_blended_steps():
    # the paper's KH run (Sec. 7.2.1, its layers compressed twice): the shock-capturing indicator
    # of the density drives the
    # adaptation; flags from the oracle's sigmoid (the GPU's checked against it), replayed on both
    # sides, leaf lists bit-exact; then P-ERK3 steps with shock capturing on the adapted forest
    from oracle import amr
    from paper_2403_05144_amd import PerkSolver
    mesh = pin.uniform_mesh(2, (16, 16), (-1, -1), (1, 1), 0)
    lmax = 2
    fam = _perk3_family([3, 6])
    mol = [0, 0, 1]
    s = PerkSolver(mesh, 3, fam, mol, capacity=8192)
    s.set_indicator("hennemann_gassner", variable=0)
    s.set_shock_capturing(True, alpha_max=AMAX, alpha_min=AMIN)
    leaves = mesh.leaves
    for cyc in range(3):
        o = od.Oracle(pin.MeshDesc(2, (16, 16), (-1, -1), (1, 1), leaves), 4)
        u = _kh_state(o, 2)
        s.set_state(u)
        o.set_shock_capturing(True, alpha_max=1.0, alpha_min=0.0)
        _, eta_o, _ = o.sc_indicator(u)
        eta_g = s.indicator()
        assert np.max(np.abs(eta_g - eta_o)) <= 1e-11
        for edge in (0.003, 0.0003):
            assert np.all(np.abs(eta_o - edge) > 1e-9 * edge)
        flags = amr.flags_from_indicator(eta_o, 0.003, 0.0003)
        print(f"KH cycle {cyc}: {len(leaves)} leaves, refine {np.sum(flags > 0)}, coarsen {np.sum(flags < 0)}",
              flush=True)
        leaves, _ = amr.adapt(leaves, flags, 0, lmax, 2, (16, 16))
        s.adapt(flags, 0, lmax, mol)
        np.testing.assert_array_equal(s.leaves(), leaves)
    lv = np.asarray(leaves)[:, 0]
    assert lv.max() == lmax, np.bincount(lv)
    o = od.Oracle(pin.MeshDesc(2, (16, 16), (-1, -1), (1, 1), leaves), 4)
    u0 = _kh_state(o, 2)
    assert np.count_nonzero(_alpha_checked(o, u0)) > 0
    s.set_state(u0)
    member = np.asarray(mol)[lv]
    dt, n = 2e-4, 2
    u_ora = u0.copy()
    for _ in range(n):
        u_ora = o.prk_step(u_ora, dt, fam, member)
    s.step(dt, n)
    g = s.get_state().cpu().numpy()
    worst = max(np.max(np.abs(g[:, v] - u_ora[:, v])) / np.max(np.abs(u_ora[:, v])) for v in range(4))
    assert worst <= TOL, worst
