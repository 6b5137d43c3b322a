"""GPU vs oracle on the adaptive Kelvin-Helmholtz setup: indicator, adaptation (bit-exact leaf
lists), projection, re-partition and third-order P-ERK steps across adaptation cycles.

Adaptation decisions are replayed from the oracle's indicator (floating point decides an
integer flag; both sides must take the same decision), and the GPU indicator is compared
separately.  Bar: 1e-12 relative per conserved variable."""
import json
import os

import numpy as np
import pytest

import perk_inputs as pin
from oracle import amr
from oracle import dgsem as od
from oracle import perk_coeffs as pc

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-12


def rel_err(a, b):
    return max(np.max(np.abs(a[:, v] - b[:, v])) / max(np.max(np.abs(b[:, v])), 1e-300) for v in range(b.shape[1]))


def golden_family(name):
    with open(os.path.join(GOLD, name)) as f:
        return pc.PerkFamily.from_json(json.load(f))


def kh_ic(o):
    x = o.node_coords().transpose(1, 0, 2)
    return pin.kelvin_helmholtz(x[0], x[1]).transpose(1, 0, 2).copy()


def test_indicator_adapt_project_replay():
    from paper_2403_05144_amd import PerkSolver
    mesh = pin.uniform_mesh(2, (8, 8), (-1, -1), (1, 1), 0)
    fam = golden_family("perk3_4_6_8_12_16_disk.json")
    lmax = 3
    mol = [max(0, 4 - (lmax - l)) for l in range(lmax + 1)]
    s = PerkSolver(mesh, 3, fam, mol, capacity=4096)
    o = od.Oracle(mesh, 4)
    u = kh_ic(o)
    s.set_state(u)
    for _ in range(3):
        eta_o = amr.indicator(o, u)
        eta_g = s.indicator()
        assert np.max(np.abs(eta_g - eta_o)) <= TOL * np.max(np.abs(eta_o))
        flags = amr.flags_from_indicator(eta_o, 0.05, 0.01)
        new, plan = amr.adapt(o.mesh.leaves, flags, 0, lmax, 2, (8, 8))
        s.adapt(flags, 0, lmax, mol)
        np.testing.assert_array_equal(s.leaves(), new)
        u_new = amr.project(o, u, plan, 4)
        assert rel_err(s.get_state().cpu().numpy(), u_new) <= TOL
        o = od.Oracle(pin.MeshDesc(2, (8, 8), (-1, -1), (1, 1), new), 4)
        u = kh_ic(o)
        s.set_state(u)
    assert s.n_elements > 64 and np.max(new[:, 0]) == lmax
    # partition follows the levels: finest members first
    leaf_of_slot, mem = s.element_info()
    member = np.asarray(mol)[new[:, 0]]
    np.testing.assert_array_equal(leaf_of_slot, np.argsort(-member, kind="stable"))

    # third-order P-ERK steps with an adaptation every 4 steps (replayed)
    dt = 2e-4
    member = np.asarray(mol)[o.mesh.leaves[:, 0]]
    for cycle in range(3):
        for _ in range(4):
            u = o.prk_step(u, dt, fam, member)
        s.step(dt, 4)
        assert rel_err(s.get_state().cpu().numpy(), u) <= TOL
        eta_o = amr.indicator(o, u)
        # move the thresholds so that both refinement and coarsening happen
        flags = amr.flags_from_indicator(eta_o, 0.03, 0.02)
        new, plan = amr.adapt(o.mesh.leaves, flags, 0, lmax, 2, (8, 8))
        s.adapt(flags, 0, lmax, mol)
        np.testing.assert_array_equal(s.leaves(), new)
        u = amr.project(o, u, plan, 4)
        o = od.Oracle(pin.MeshDesc(2, (8, 8), (-1, -1), (1, 1), new), 4)
        member = np.asarray(mol)[new[:, 0]]
        assert rel_err(s.get_state().cpu().numpy(), u) <= TOL


def test_adapt_rejects_over_capacity():
    from paper_2403_05144_amd import PerkSolver, PerkError
    mesh = pin.uniform_mesh(2, (4, 4), (-1, -1), (1, 1), 0)
    fam = golden_family("perk3_4_8_16_disk.json")
    s = PerkSolver(mesh, 3, fam, [2, 2], capacity=40)
    o = od.Oracle(mesh, 4)
    s.set_state(kh_ic(o))
    with pytest.raises(PerkError):
        s.adapt(np.ones(16, np.int8), 0, 1, [1, 2])
    # the mesh is unchanged and still steps
    assert s.n_elements == 16
    s.step(1e-4, 1)


def test_graph_replay_across_adaptations_equals_eager():
    # after every re-partition the captured step is updated in place (same launches, new sizes)
    # or re-instantiated; stepping by graph replay and by eager launches must give bitwise the
    # same leaves and states through several adaptation cycles
    from paper_2403_05144_amd import PerkSolver
    from paper_2403_05144_amd.amr import AmrDriver
    fam = golden_family("perk3_4_6_8_12_16_disk.json")
    lmax = 3
    mol = [max(0, 4 - (lmax - l)) for l in range(lmax + 1)]

    def ic_leaf(x):
        return pin.kelvin_helmholtz(x[:, 0], x[:, 1]).transpose(1, 0, 2).copy()

    runs = []
    for graphs in (True, False):
        s = PerkSolver(pin.uniform_mesh(2, (8, 8), (-1, -1), (1, 1), 0), 3, fam, mol, capacity=4096)
        s.set_graph_replay(graphs)
        drv = AmrDriver(s, 0, lmax, mol, 0.05, 0.01, 3)
        drv.initial_mesh(ic_leaf, passes=2)
        states = []
        for _ in range(4):
            s.step(2e-4, 3)
            states.append(s.get_state().cpu().numpy())
            drv.adapt_once()
            states.append(s.get_state().cpu().numpy())
        states.append(s.leaves().copy())
        runs.append(states)
    assert runs[0][-1].shape == runs[1][-1].shape
    for a, b in zip(runs[0], runs[1]):
        np.testing.assert_array_equal(a, b)


def test_amr_cycle_equals_separate_calls():
    # one library call (indicator, threshold flags, adaptation, re-partition) against the
    # indicator download, the flags formed in Python and the adapt + partition calls: the same
    # flags, leaves and states, bitwise, through several cycles with steps in between
    from paper_2403_05144_amd import PerkSolver
    from paper_2403_05144_amd.amr import flags_from_indicator
    fam = golden_family("perk3_4_6_8_12_16_disk.json")
    lmax = 3
    mol = [max(0, 4 - (lmax - l)) for l in range(lmax + 1)]

    def ic_leaf(x):
        return pin.kelvin_helmholtz(x[:, 0], x[:, 1]).transpose(1, 0, 2).copy()

    runs = []
    for fused in (True, False):
        s = PerkSolver(pin.uniform_mesh(2, (8, 8), (-1, -1), (1, 1), 0), 3, fam, mol, capacity=4096)
        s.set_state(ic_leaf(s.node_coords().cpu().numpy()))
        rec = []
        for cycle in range(5):
            if fused:
                flags = s.amr_cycle(0.05, 0.01, 0, lmax, mol)
            else:
                flags = flags_from_indicator(s.indicator(), 0.05, 0.01)
                s.adapt(flags, 0, lmax, mol)
            rec += [flags, s.leaves().copy(), s.get_state().cpu().numpy()]
            if cycle < 2:
                s.set_state(ic_leaf(s.node_coords().cpu().numpy()))
            s.step(2e-4, 3)
            rec.append(s.get_state().cpu().numpy())
        runs.append(rec)
    assert len(runs[0]) == len(runs[1])
    assert any(np.any(r != 0) for r in runs[0][0::4])   # the cycles did change the mesh
    for a, b in zip(runs[0], runs[1]):
        assert a.shape == b.shape
        np.testing.assert_array_equal(a, b)


def test_lohner_indicator_and_ns_steps_on_the_shear_layer():
    # Sec. 7.1.1: Loehner's indicator on v_x drives the adaptation of the doubly periodic shear
    # layer; P-ERK3{3,4,7} Navier-Stokes steps (BR1, mu = 1/Re, Re = 2.5e4) on the adapted forest.
    # The GPU indicator against the oracle's (1e-14: one division per estimate, contraction may
    # differ), flags replayed from the oracle, leaf lists bit-exact, states 1e-12.
    from paper_2403_05144_amd import PerkSolver
    from parity_util import flux_scale, state_close, worst
    th = np.linspace(0, 2 * np.pi, 200, endpoint=False)
    eigs = -1.0 + np.exp(1j * th)
    fam = pc.perk3_family([3, 4, 7], {E: pc.optimize_alpha(eigs, 3, E)[1] for E in (4, 7)})
    mu = 1.0 / 2.5e4
    mesh = pin.uniform_mesh(2, (8, 8), (0, 0), (1, 1), 0)
    lmax = 3
    s = PerkSolver(mesh, 3, fam, [0, 0, 1, 2], capacity=8192, equations=1, mu=mu)
    s.set_indicator("lohner", 1, 0.2)
    leaves = mesh.leaves
    for cyc in range(3):
        o = od.Oracle(pin.MeshDesc(2, (8, 8), (0, 0), (1, 1), leaves), 4, viscous=True, mu=mu)
        x = o.node_coords().transpose(1, 0, 2)
        u = pin.shear_layer(x[0], x[1]).transpose(1, 0, 2).copy()
        s.set_state(u)
        eta_o = amr.lohner_indicator(o, u, var=1, f_wave=0.2)
        eta_g = s.indicator()
        print(f"shear layer cycle {cyc}: {len(leaves)} leaves, max eta {eta_o.max():.3f}", flush=True)
        assert np.max(np.abs(eta_g - eta_o)) <= 1e-14
        flags = amr.flags_from_indicator(eta_o, 0.2, 0.05)
        leaves, _ = amr.adapt(leaves, flags, 0, lmax, 2, (8, 8))
        s.adapt(flags, 0, lmax, [0, 0, 1, 2])
        np.testing.assert_array_equal(s.leaves(), leaves)
    lv = np.asarray(leaves)[:, 0]
    assert lv.max() == lmax and lv.min() == 0, np.bincount(lv)
    o = od.Oracle(pin.MeshDesc(2, (8, 8), (0, 0), (1, 1), leaves), 4, viscous=True, mu=mu)
    x = o.node_coords().transpose(1, 0, 2)
    u0 = pin.shear_layer(x[0], x[1]).transpose(1, 0, 2).copy()
    s.set_state(u0)
    member = np.asarray([0, 0, 1, 2])[lv]
    dt = 2e-5
    u_ora = u0.copy()
    for _ in range(2):
        u_ora = o.prk_step(u_ora, dt, fam, member)
    s.step(dt, 2)
    u_gpu = s.get_state().cpu().numpy()
    sig = flux_scale(o, u0)
    assert state_close(u_gpu, u_ora, sig, 2, dt), worst(u_gpu, u_ora, sig, 2, dt)
