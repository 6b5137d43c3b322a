"""Discrete adjoint on the GPU against the oracle's (dense, column by column from dual
numbers): the right-hand-side adjoint F'(u)^T w on 2D and 3D meshes with 2:1 mortars,
p = 2 and 3, and the adjoint of partitioned P-ERK2 / P-ERK3 steps with inactive stages.
States are discontinuous across faces (no HLL wave-speed ties).  Bar: 1e-12 relative to the
largest entry of the oracle's result per conserved variable (floor: its overall largest)."""
import json
import os

import numpy as np
import pytest

import perk_inputs as pin
from oracle import dgsem as od
from oracle import perk_coeffs as pc

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _mesh3d():
    m = pin.uniform_mesh(3, (2, 2, 2), (0.0,) * 3, (1.0,) * 3, 0)
    m.leaves = pin.refine_leaves(m.leaves, 3, [0])
    return m


def _state(o, seed):
    x = o.node_coords().transpose(1, 0, 2)
    if o.dim == 2:
        u = pin.smooth_random_state(x, 2, seed).transpose(1, 0, 2).copy()
    else:
        u = pin.taylor_green(2 * np.pi * x[0], 2 * np.pi * x[1], 2 * np.pi * x[2], mach=0.3).transpose(1, 0, 2).copy()
    rng = np.random.default_rng(seed)
    return u * (1 + 0.01 * rng.standard_normal(u.shape)), rng


def _close(g, ref, tol=1e-12):
    floor = np.max(np.abs(ref))
    for v in range(ref.shape[1]):
        scale = max(np.max(np.abs(ref[:, v])), 1e-3 * floor)
        if np.max(np.abs(g[:, v] - ref[:, v])) > tol * scale:
            return False
    return True


def _err(g, ref):
    return [float(np.max(np.abs(g[:, v] - ref[:, v])) / np.max(np.abs(ref[:, v]))) for v in range(ref.shape[1])]


CASES = {
    "forest2d_p3": (lambda: pin.random_forest_2d(11, n_root=3, max_level=2), 4),
    "forest2d_p2": (lambda: pin.random_forest_2d(5, n_root=3, max_level=2), 3),
    "mesh3d_p2": (_mesh3d, 3),
    "mesh3d_p3": (_mesh3d, 4),
}


@pytest.mark.parametrize("case", list(CASES))
def test_rhs_vjp_matches_oracle(case):
    from paper_2403_05144_amd import PerkSolver
    mk, N = CASES[case]
    mesh = mk()
    o = od.Oracle(mesh, N)
    u, rng = _state(o, 21)
    w = rng.standard_normal(o.shape)
    lmax = int(mesh.leaves[:, 0].max())
    s = PerkSolver(mesh, N - 1, pc.perk2_family([4, 8]), [0] * (lmax + 1))
    g = s.rhs_vjp_leaf(u, w).cpu().numpy()
    ref = o.rhs_vjp(u, w)
    assert _close(g, ref), _err(g, ref)


@pytest.mark.parametrize("order", [2, 3])
def test_step_adjoint_matches_oracle(order):
    from paper_2403_05144_amd import PerkSolver
    mesh = pin.random_forest_2d(5, n_root=3, max_level=2)
    N = 3
    o = od.Oracle(mesh, N)
    u, rng = _state(o, 31 + order)
    lam = rng.standard_normal(o.shape)
    if order == 2:
        fam = pc.perk2_family([4, 8])
    else:
        with open(os.path.join(GOLD, "perk3_4_8_16_disk.json")) as f:
            fam = pc.PerkFamily.from_json(json.load(f))
    R = len(fam.E)
    mol = od.member_of_levels_paper_rule(np.arange(3), R)
    member = np.asarray(mol)[mesh.leaves[:, 0]]
    dt = 2e-3
    s = PerkSolver(mesh, N - 1, fam, mol)
    g = s.to_leaf(s.step_adjoint(s.to_slot(u), s.to_slot(lam), dt)).cpu().numpy()
    ref = o.prk_step_vjp(u, lam, dt, fam, member)
    assert _close(g, ref), _err(g, ref)
    # the state held by the solver is untouched by the adjoint
    s.set_state(u)
    s.step_adjoint(s.to_slot(u), s.to_slot(lam), dt)
    assert np.array_equal(s.get_state().cpu().numpy(), u)


def test_adjoint_rejects_navier_stokes():
    from paper_2403_05144_amd import PerkError, PerkSolver
    mesh = pin.random_forest_2d(5, n_root=3, max_level=2)
    s = PerkSolver(mesh, 2, pc.perk2_family([4, 8]), [0, 0, 0], equations=1, mu=1e-3)
    o = od.Oracle(mesh, 3)
    u, rng = _state(o, 3)
    with pytest.raises(PerkError):
        s.rhs_vjp_leaf(u, u)


@pytest.mark.parametrize("order", [2, 3])
def test_recorded_step_adjoint_equals_recomputing(order):
    # pe_step_record + pe_step_adjoint_recorded against pe_step_adjoint (which recomputes the
    # step) and pe_step: bitwise the same next state and cotangent; the bound state untouched
    import torch
    from paper_2403_05144_amd import PerkSolver
    mesh = pin.random_forest_2d(7, n_root=3, max_level=2)
    N = 4
    o = od.Oracle(mesh, N)
    u, rng = _state(o, 41 + order)
    lam = rng.standard_normal(o.shape)
    if order == 2:
        fam = pc.perk2_family([4, 8])
    else:
        with open(os.path.join(GOLD, "perk3_4_8_16_disk.json")) as f:
            fam = pc.PerkFamily.from_json(json.load(f))
    mol = od.member_of_levels_paper_rule(np.arange(3), len(fam.E))
    dt = 2e-3
    s = PerkSolver(mesh, N - 1, fam, mol)
    s.set_state(u)
    u_slot, lam_slot = s.to_slot(u), s.to_slot(lam)
    bound = s.u.clone()
    u_next, rec = s.step_record(u_slot, dt)
    g_rec = s.step_adjoint_recorded(u_slot, rec, lam_slot, dt)
    g_ref = s.step_adjoint(u_slot, lam_slot, dt)
    torch.cuda.synchronize()
    assert torch.equal(s.u, bound)
    assert torch.equal(g_rec, g_ref)
    s.step(dt, 1)
    stepped = s.get_state().cpu().numpy()
    np.testing.assert_array_equal(s.to_leaf(u_next).cpu().numpy(), stepped)
