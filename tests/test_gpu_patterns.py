"""GPU parity of alternative stage-evaluation patterns (Sec. 3.2.4, eq.
PERK_ButcherTableauAlternating and eq. PERK_ButcherTableauEarlyShared) against the oracle's dense
partitioned step (eq. PartitionedRKSystem with each member's full Butcher matrix), bar 1e-12 as
in tests/parity_util.py.

Cases: the printed S = 6, E = 4 patterns (classic chain given as a table, alternating, early
shared) next to a full E = 6 member; an S = 8 family whose members evaluate non-nested stage sets
(E = 4 alternating, E = 6 early shared, E = 8), so that the active elements of some stages are
two separate member ranges; p = 2 blocks of two elements; a forest above the size where 2D p = 3
launches change body; 3D; graph replay against eager launches; evaluation counters (eq.
ActualRHSEvals)."""
import numpy as np
import pytest

import perk_inputs as pin
from oracle import dgsem as od
from oracle import perk_coeffs as pc
from parity_util import TOL, flux_scale, state_close, worst

pytestmark = pytest.mark.gpu

NONNESTED = [[0, 3, 5, 7], [0, 1, 2, 3, 4, 7], list(range(8))]


def _three_level_vortex():
    mesh = pin.mesh_vortex_2level()
    sel = [r for r, (l, i, j, k) in enumerate(mesh.leaves.tolist()) if l == 1 and 14 <= i < 18 and 14 <= j < 18]
    mesh.leaves = pin.refine_leaves(mesh.leaves, 2, sel)
    return mesh


def _vortex(o):
    x = o.node_coords().transpose(1, 0, 2)
    return pin.isentropic_vortex(x[0], x[1]).transpose(1, 0, 2).copy()


def _random2d(seed):
    def f(o):
        x = o.node_coords().transpose(1, 0, 2)
        return pin.smooth_random_state(x, 2, seed).transpose(1, 0, 2).copy()
    return f


def _tgv(o):
    x = o.node_coords().transpose(1, 0, 2)
    return pin.taylor_green(x[0], x[1], x[2]).transpose(1, 0, 2).copy()


def _mesh3d():
    m = pin.uniform_mesh(3, (4, 4, 4), (-np.pi,) * 3, (np.pi,) * 3, 0)
    sel = [r for r, (l, i, j, k) in enumerate(m.leaves.tolist()) if (i, j, k) in ((1, 1, 1), (2, 1, 1), (1, 2, 1))]
    m.leaves = pin.refine_leaves(m.leaves, 3, sel)
    return m


def _run(mesh, N, fam, mol, u0_fn, dt, n_steps, graphs=True):
    from paper_2403_05144_amd import PerkSolver
    o = od.Oracle(mesh, N)
    u0 = u0_fn(o)
    s = PerkSolver(mesh, N - 1, fam, mol)
    s.set_graph_replay(graphs)
    s.set_state(u0)
    member = np.asarray(mol)[np.asarray(mesh.leaves)[:, 0]]
    u_ora = u0.copy()
    for _ in range(n_steps):
        u_ora = o.prk_step(u_ora, dt, fam, member)
    s.step(dt, n_steps)
    u_gpu = s.get_state().cpu().numpy()
    sig = flux_scale(o, u0)
    return u_gpu, u_ora, sig, s, member


@pytest.mark.parametrize("kind", list(pc.PAPER_CHAINS_S6_E4))
def test_paper_patterns_step_parity(kind):
    fam = pc.pattern_family([pc.PAPER_CHAINS_S6_E4[kind], list(range(6))], 6)
    mesh = pin.mesh_vortex_2level()
    for n in (1, 5):
        print(f"pattern {kind}: {n} steps", flush=True)
        u_gpu, u_ora, sig, _, _ = _run(mesh, 4, fam, [0, 1], _vortex, 0.02, n)
        assert state_close(u_gpu, u_ora, sig, n, 0.02), worst(u_gpu, u_ora, sig, n, 0.02)


def test_classic_chain_as_a_table_equals_the_classic_family():
    # the classic family given with an explicit coupling table runs the same scheme as the
    # classic family itself (the two paths form some stage values in another order: 1e-12)
    from paper_2403_05144_amd import PerkSolver
    mesh = pin.mesh_vortex_2level()
    classic = pc.perk2_family([4, 8])
    table = pc.pattern_family([[0, 5, 6, 7], list(range(8))], 8)
    np.testing.assert_array_equal(np.asarray(table.a_sub), np.asarray(classic.a_sub))
    o = od.Oracle(mesh, 4)
    u0 = _vortex(o)
    outs = []
    for fam in (classic, table):
        s = PerkSolver(mesh, 3, fam, [0, 1])
        s.set_state(u0)
        s.step(0.02, 4)
        outs.append(s.get_state().cpu().numpy())
    sig = flux_scale(o, u0)
    assert state_close(outs[1], outs[0], sig, 4, 0.02)


def test_nonnested_family_step_parity_and_counters():
    fam = pc.pattern_family(NONNESTED, 8)
    mesh = _three_level_vortex()
    levels = np.asarray(mesh.leaves)[:, 0]
    assert sorted(set(levels.tolist())) == [0, 1, 2]
    for n in (1, 4):
        print(f"non-nested S=8 family: {n} steps", flush=True)
        u_gpu, u_ora, sig, s, member = _run(mesh, 4, fam, [0, 1, 2], _vortex, 0.01, n)
        assert state_close(u_gpu, u_ora, sig, n, 0.01), worst(u_gpu, u_ora, sig, n, 0.01)
        tot, per = s.counters()
        E = np.asarray(fam.E)
        assert tot == n * int(np.sum(E[member]))
        assert per == [n * E[r] * int(np.sum(member == r)) for r in range(3)]


def test_nonnested_family_p2_blocks_of_two_elements():
    fam = pc.pattern_family(NONNESTED, 8)
    mesh = pin.random_forest_2d(5, n_root=3, max_level=3)
    nl = int(np.asarray(mesh.leaves)[:, 0].max()) + 1
    mol = [0] * max(0, nl - 3) + [0, 1, 2][-min(3, nl):]
    print(f"p=2 forest, {len(mesh.leaves)} elements, levels {nl}", flush=True)
    u_gpu, u_ora, sig, _, _ = _run(mesh, 3, fam, mol, _random2d(3), 0.002, 3)
    assert state_close(u_gpu, u_ora, sig, 3, 0.002), worst(u_gpu, u_ora, sig, 3, 0.002)


def test_nonnested_family_large_forest_both_launch_shapes():
    fam = pc.pattern_family(NONNESTED, 8)
    # 3511 elements, levels of 187, 2076 and 1248: stages above 2048 active elements on the
    # one-wave body, the others on the two-wave one
    mesh = pin.random_forest_2d(3, n_root=28, max_level=2, p_refine=0.3)
    assert len(mesh.leaves) > 2048 and np.bincount(mesh.leaves[:, 0]).min() < 2048
    print(f"large forest, {len(mesh.leaves)} elements", flush=True)
    u_gpu, u_ora, sig, _, _ = _run(mesh, 4, fam, [0, 1, 2], _random2d(11), 0.002, 2)
    assert state_close(u_gpu, u_ora, sig, 2, 0.002), worst(u_gpu, u_ora, sig, 2, 0.002)


@pytest.mark.parametrize("N", [3, 4])
def test_pattern_step_parity_3d(N):
    fam = pc.pattern_family([pc.PAPER_CHAINS_S6_E4["alternating"], list(range(6))], 6)
    print(f"3D N={N}", flush=True)
    u_gpu, u_ora, sig, _, _ = _run(_mesh3d(), N, fam, [0, 1], _tgv, 0.004, 2)
    assert state_close(u_gpu, u_ora, sig, 2, 0.004), worst(u_gpu, u_ora, sig, 2, 0.004)


def test_pattern_graph_replay_equals_eager():
    fam = pc.pattern_family(NONNESTED, 8)
    mesh = _three_level_vortex()
    a, *_ = _run(mesh, 4, fam, [0, 1, 2], _vortex, 0.01, 3, graphs=True)
    b, *_ = _run(mesh, 4, fam, [0, 1, 2], _vortex, 0.01, 3, graphs=False)
    np.testing.assert_array_equal(a, b)
