"""Oracle pins of the alternative stage-evaluation patterns (Sec. 3.2.4, eq.
PERK_ButcherTableauAlternating and eq. PERK_ButcherTableauEarlyShared): the printed S = 6, E = 4
tableau structures and stage sets, one stability polynomial for all patterns, identical results
on a linear problem, the classic chain equal to the classic construction, and for a partitioned
DG step with members on different chains: conservation, second order in time, and results that
depend on the pattern (nonlinear problem, non-uniform mesh)."""
import math

import numpy as np
import pytest

import perk_inputs as pin
from oracle import dgsem as od
from oracle import perk_coeffs as pc

S6 = 6


def _paper_member(kind):
    al = pc.disk_optimal_alpha_p2(4)
    j, a = pc.chain_member(al, pc.PAPER_CHAINS_S6_E4[kind], S6)
    return pc.dense_A_coupled(pc.perk2_abscissae(S6), j, a)


@pytest.mark.parametrize("kind,nonzero,stages", [
    # 1-based (row, column) of the coefficients beyond the first column, and the evaluated
    # stages, as printed in Sec. 3.1 (classic) and Sec. 3.2.4
    ("classic", {(5, 4), (6, 5)}, [1, 4, 5, 6]),
    ("alternating", {(4, 3), (6, 4)}, [1, 3, 4, 6]),
    ("early_shared", {(3, 2), (6, 3)}, [1, 2, 3, 6]),
])
def test_printed_structures(kind, nonzero, stages):
    A = _paper_member(kind)
    c = pc.perk2_abscissae(S6)
    np.testing.assert_allclose(c, [0, 0.1, 0.2, 0.3, 0.4, 0.5], atol=1e-16)
    got = {(i + 1, j + 1) for i in range(S6) for j in range(1, S6) if A[i, j] != 0.0}
    assert got == nonzero
    assert np.all(A[1:, 0] != 0.0) and np.all(np.triu(A) == 0.0)
    np.testing.assert_allclose(A.sum(axis=1), c, atol=1e-15)          # eq. (InternalConsistency)
    assert pc.stage_evaluations(A, pc.perk2_weights(S6)) == stages


def test_one_polynomial_for_every_pattern():
    # the free coefficients of every pattern come from the same P_{2;4} (Sec. 3.2.4)
    al = pc.disk_optimal_alpha_p2(4)
    target = np.array([1.0, 1.0, 0.5, al[3], al[4], 0.0, 0.0])
    for kind in pc.PAPER_CHAINS_S6_E4:
        P = pc.stability_poly(_paper_member(kind), pc.perk2_weights(S6))
        np.testing.assert_allclose(P, target, rtol=1e-14, atol=1e-17)
    # a longer member on an arbitrary chain, with an optimised polynomial
    th = np.linspace(0, 2 * np.pi, 100, endpoint=False)
    _, alpha = pc.optimize_alpha(-2.0 + 2.0 * np.exp(1j * th), 2, 6)
    chain = [0, 2, 3, 7, 9, 11]
    j, a = pc.chain_member(alpha, chain, 12)
    P = pc.stability_poly(pc.dense_A_coupled(pc.perk2_abscissae(12), j, a), pc.perk2_weights(12))
    np.testing.assert_allclose(P[:7], [1, 1, 0.5] + [alpha[k] for k in range(3, 7)], rtol=1e-13)
    assert np.all(P[7:] == 0.0)


def test_classic_chain_is_the_classic_construction():
    for E, S in ((4, 8), (8, 16), (3, 6)):
        al = pc.disk_optimal_alpha_p2(E)
        j, a = pc.chain_member(al, [0] + list(range(S - E + 1, S)), S)
        np.testing.assert_array_equal(a, pc.perk2_a_from_alpha(al, E, S))
        assert [int(x) for x in j] == [i - 1 if i >= S - E + 2 else -1 for i in range(S)]


def test_patterns_agree_on_a_linear_problem():
    # for y' = J y every pattern is the same polynomial in dt J (Sec. 3.2.4)
    rng = np.random.default_rng(3)
    n = 12
    J = rng.standard_normal((n, n)) - 3 * np.eye(n)
    y0 = rng.standard_normal(n)
    dt = 0.1
    outs = []
    for kind in pc.PAPER_CHAINS_S6_E4:
        A, b = _paper_member(kind), pc.perk2_weights(S6)
        K = np.zeros((S6, n))
        for i in range(S6):
            K[i] = J @ (y0 + dt * (A[i, :i] @ K[:i]))
        outs.append(y0 + dt * (b @ K))
    for o in outs[1:]:
        np.testing.assert_allclose(o, outs[0], rtol=1e-13, atol=1e-14)


def _family_nonnested():
    # S = 8: E = 4 on an alternating chain, E = 6 on an early chain, E = 8 on every stage; the
    # members evaluating stage 6 (1-based) are E = 4 and E = 8 but not E = 6
    return pc.pattern_family([[0, 3, 5, 7], [0, 1, 2, 3, 4, 7], list(range(8))], 8)


def _three_level_setup():
    mesh = pin.mesh_vortex_2level()
    sel = [r for r, (l, i, j, k) in enumerate(mesh.leaves.tolist()) if l == 1 and 14 <= i < 18 and 14 <= j < 18]
    mesh.leaves = pin.refine_leaves(mesh.leaves, 2, sel)
    o = od.Oracle(mesh, 4)
    x = o.node_coords().transpose(1, 0, 2)
    u0 = pin.isentropic_vortex(x[0], x[1]).transpose(1, 0, 2).copy()
    member = np.asarray(mesh.leaves)[:, 0].astype(np.int32)      # level l -> member l
    return o, u0, member


def test_stage_sets_of_the_nonnested_family():
    fam = _family_nonnested()
    sets = [pc.stage_evaluations(fam.dense(r), fam.b) for r in range(3)]
    assert sets == [[1, 4, 6, 8], [1, 2, 3, 4, 5, 8], list(range(1, 9))]
    for r in range(3):
        P = pc.stability_poly(fam.dense(r), fam.b)
        al = pc.disk_optimal_alpha_p2(fam.E[r])
        np.testing.assert_allclose(P[3:fam.E[r] + 1], [al[k] for k in range(3, fam.E[r] + 1)], rtol=1e-13)


def test_partitioned_pattern_step_conserves_and_is_second_order():
    o, u0, member = _three_level_setup()
    assert sorted(set(member.tolist())) == [0, 1, 2]
    fam = _family_nonnested()
    I0 = o.integral(u0)
    u = u0.copy()
    for _ in range(10):
        u = o.prk_step(u, 0.02, fam, member)
    assert np.all(np.abs(o.integral(u) - I0) < 1e-12 * np.maximum(1.0, np.abs(I0)))   # eq. (Conservation)
    T = 0.2

    def run(dt):
        v = u0.copy()
        for _ in range(int(round(T / dt))):
            v = o.prk_step(v, dt, fam, member)
        return v

    ref = run(T / 160)
    errs = [np.max(np.abs(run(T / n) - ref)) for n in (20, 40)]
    slope = math.log2(errs[0] / errs[1])
    assert 1.8 < slope < 2.3, (errs, slope)


def test_patterns_differ_on_a_partitioned_nonlinear_step():
    # on a non-uniform mesh the stage pattern matters (Sec. 3.2.4): the same polynomials on other
    # chains give another partitioned result, though each is consistent
    mesh = pin.mesh_vortex_2level()
    o2 = od.Oracle(mesh, 4)
    x = o2.node_coords().transpose(1, 0, 2)
    u2 = pin.isentropic_vortex(x[0], x[1]).transpose(1, 0, 2).copy()
    mem2 = np.asarray(mesh.leaves)[:, 0].astype(np.int32)
    res = {}
    for kind, ch in pc.PAPER_CHAINS_S6_E4.items():
        fam = pc.pattern_family([ch, list(range(6))], 6)
        res[kind] = o2.prk_step(u2, 0.05, fam, mem2)
    scale = np.max(np.abs(u2))
    for k1 in res:
        for k2 in res:
            if k1 < k2:
                assert np.max(np.abs(res[k1] - res[k2])) > 1e-9 * scale, (k1, k2)
