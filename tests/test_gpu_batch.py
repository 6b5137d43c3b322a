"""Batched independent runs (one launch per stage tick): every run's state after the batch is
bitwise equal to the same run stepped alone with pe_step, for every tile shape, with runs of
degree 2 and 3, two- and three-member families and different step counts; one run is also
checked against the oracle.  Unsupported runs are rejected."""
import numpy as np
import pytest

import perk_inputs as pin
from oracle import dgsem as od
from oracle import perk_coeffs as pc

pytestmark = pytest.mark.gpu

SPECS = [  # (roots per side, disk levels, degree, family, steps, vortex strength)
    (8, 1, 3, (4, 8), 5, 5.0),
    (10, 2, 2, (4, 8, 16), 3, 2.0),
    (12, 3, 3, (4, 8, 16), 2, 3.5),
    (9, 1, 2, (4, 8), 7, 1.0),
    (14, 2, 3, (4, 8), 4, 4.2),
    (8, 3, 2, (4, 8, 16), 1, 2.7),
]


def _runs():
    from paper_2403_05144_amd import PerkSolver
    out = []
    for n, L, p, E, steps, eps in SPECS:
        mesh = pin.mesh_vortex_disks(n, L)
        fam = pc.perk2_family(list(E))
        lmax = int(mesh.leaves[:, 0].max())
        mol = od.member_of_levels_paper_rule(np.arange(lmax + 1), len(E))
        s = PerkSolver(mesh, p, fam, mol)
        x = s.node_coords().cpu().numpy().transpose(1, 0, 2)
        u0 = pin.isentropic_vortex(x[0], x[1], eps=eps).transpose(1, 0, 2).copy()
        s.set_state(u0)
        h_min = 10.0 / n / 2 ** lmax
        dt = 0.5 * h_min / ((p + 1) * 3.0)           # half the convective bound; well inside stability
        out.append(dict(s=s, u0=u0, dt=dt, steps=steps, mesh=mesh, fam=fam, mol=mol, p=p))
    return out


def _reference(runs):
    refs = []
    for r in runs:
        r["s"].set_state(r["u0"])
        r["s"].step(r["dt"], r["steps"])
        refs.append(r["s"].get_state().cpu().numpy())
        r["s"].set_state(r["u0"])
    return refs


@pytest.mark.parametrize("tiling", [(1, 0), (2, 0), (4, 0), (1, 64), (2, 7), (4, 256)])
def test_batch_bitwise_equals_single_runs(tiling):
    from paper_2403_05144_amd import PerkBatch
    runs = _runs()
    refs = _reference(runs)
    b = PerkBatch([r["s"] for r in runs])
    b.set_steps([r["dt"] for r in runs], [r["steps"] for r in runs])
    b.set_tiling(*tiling)
    n_ticks, es = b.info()
    assert n_ticks == max(r["steps"] * r["fam"].S for r in runs)
    for r in runs:
        r["s"].counters(reset=True)
    b.run()
    for r, ref in zip(runs, refs):
        got = r["s"].get_state().cpu().numpy()
        assert np.array_equal(got, ref), np.max(np.abs(got - ref))
    # per-run evaluation counters: the element-stages of the tick table, run by run
    assert sum(r["s"].counters()[0] for r in runs) == es


def test_batch_autotune_restores_state_and_ticks_split():
    from paper_2403_05144_amd import PerkBatch
    runs = _runs()
    refs = _reference(runs)
    b = PerkBatch([r["s"] for r in runs])
    b.set_steps([r["dt"] for r in runs], [r["steps"] for r in runs])
    res = b.autotune(candidates=[(1, 0), (2, 128), (4, 0)], ticks=20, reps=1)
    assert tuple(res["tiling"]) in {(1, 0), (2, 128), (4, 0)}
    n = b.n_ticks
    b.run(0, 13)          # ticks may be launched in pieces
    b.run(13, n)
    for r, ref in zip(runs, refs):
        assert np.array_equal(r["s"].get_state().cpu().numpy(), ref)


def test_batch_run_matches_oracle():
    from paper_2403_05144_amd import PerkBatch
    runs = _runs()[:2]
    b = PerkBatch([r["s"] for r in runs])
    b.set_steps([r["dt"] for r in runs], [r["steps"] for r in runs])
    b.run()
    r = runs[1]                                    # degree 2, three members, 3 steps
    o = od.Oracle(r["mesh"], r["p"] + 1)
    member = np.asarray(r["mol"])[r["mesh"].leaves[:, 0]]
    u = r["u0"].copy()
    for _ in range(r["steps"]):
        u = o.prk_step(u, r["dt"], r["fam"], member)
    g = r["s"].get_state().cpu().numpy()
    for v in range(4):
        assert np.max(np.abs(g[:, v] - u[:, v])) <= 1e-12 * np.max(np.abs(u[:, v]))


def test_batch_rejects_unsupported_runs():
    from paper_2403_05144_amd import PerkBatch, PerkError, PerkSolver
    runs = _runs()[:2]
    with pytest.raises(PerkError):
        PerkBatch([runs[0]["s"], runs[0]["s"]])
    m3 = pin.uniform_mesh(3, (2, 2, 2), (-1,) * 3, (1,) * 3, 0)
    s3 = PerkSolver(m3, 3, pc.perk2_family([4, 8]), [0])
    x = s3.node_coords().cpu().numpy().transpose(1, 0, 2)
    s3.set_state(pin.taylor_green(x[0], x[1], x[2]).transpose(1, 0, 2).copy())
    with pytest.raises(PerkError):
        PerkBatch([runs[0]["s"], s3])
    b = PerkBatch([runs[0]["s"]])
    with pytest.raises(PerkError):
        b.run()                                      # no steps set
    with pytest.raises(PerkError):
        b.set_tiling(3, 0)
