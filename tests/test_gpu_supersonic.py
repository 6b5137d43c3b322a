"""GPU vs oracle where the HLL surface flux takes its supersonic branches (sL >= 0: the left
state's flux; sR <= 0: the right state's flux), on 2:1 forests in 2D and 3D, Euler and
Navier-Stokes: right-hand side and partitioned P-ERK steps (eq. PartitionedRKSystem).  The state
is a seeded smooth stream faster than sound along every axis (towards +x, -y, +z), so the faces
normal to x take the first branch and those normal to y the second; the oracle counts the
branches it took, so the test proves that both were reached.  Bars as in tests/parity_util.py
(1e-12 of the flux scale per conserved variable)."""
import numpy as np
import pytest

import perk_inputs as pin
from oracle import dgsem as od
from oracle import perk_coeffs as pc
from parity_util import flux_scale, rel_err, rhs_close, state_close, worst

pytestmark = pytest.mark.gpu


def _mesh(dim):
    if dim == 2:
        return pin.random_forest_2d(11, n_root=4, max_level=2)
    m = pin.uniform_mesh(3, (4, 4, 4), (-5.0,) * 3, (5.0,) * 3, 0)
    sel = [r for r, (l, i, j, k) in enumerate(m.leaves.tolist()) if (i, j, k) in ((1, 1, 1), (2, 1, 1), (1, 2, 1))]
    m.leaves = pin.refine_leaves(m.leaves, 3, sel)
    return m


CASES = [(2, 4, False), (2, 3, False), (3, 4, False), (2, 4, True), (3, 3, True)]


@pytest.mark.parametrize("dim,N,visc", CASES)
def test_supersonic_rhs_and_steps(dim, N, visc):
    from paper_2403_05144_amd import PerkSolver
    mesh = _mesh(dim)
    mu = 1e-3 if visc else 0.0
    o = od.Oracle(mesh, N, viscous=visc, mu=mu, prandtl=0.72)
    x = o.node_coords().transpose(1, 0, 2)
    u0 = pin.supersonic_state(x, dim, 30 + dim + N).transpose(1, 0, 2).copy()
    od.hll_branch_counts(reset=True)
    du_ora = o.rhs(u0)
    left, right, sub = od.hll_branch_counts()
    assert left > 0 and right > 0, (left, right, sub)
    fam = pc.perk2_family([4, 8])
    lv = mesh.leaves[:, 0]
    mol = od.member_of_levels_paper_rule(np.arange(lv.max() + 1), 2)
    s = PerkSolver(mesh, N - 1, fam, mol, equations=1 if visc else 0, mu=mu, prandtl=0.72)
    du_gpu = s.rhs_leaf(u0).cpu().numpy()
    sig = flux_scale(o, u0)
    assert rhs_close(du_gpu, du_ora, sig), rel_err(du_gpu, du_ora)
    dt, n = od.max_dt(o, u0, 0.3)[0], 3
    s.set_state(u0)
    s.step(dt, n)
    u = u0.copy()
    member = np.asarray(mol)[lv]
    for _ in range(n):
        u = o.prk_step(u, dt, fam, member)
    g = s.get_state().cpu().numpy()
    assert state_close(g, u, sig, n, dt), worst(g, u, sig, n, dt)
