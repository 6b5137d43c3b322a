"""The product's coefficient tool (paper_2403_05144_amd.coeffs), checked on the CPU against the
paper's printed table and against the oracle's independent tableau code."""
import math
import os

import numpy as np
import pytest

from paper_2403_05144_amd import coeffs as pt
from oracle import perk_coeffs as pc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_perk2_rows_match_paper_table():
    rows = [l.split() for l in open(os.path.join(GOLD, "perk2_8_16_table.txt")) if l.strip() and l[0] != "#"]
    T = np.array([[float(x) for x in r] for r in rows])
    for col, E in ((2, 8), (3, 16)):
        alpha = {k: (E - 1) / E * math.comb(E, k) / (E - 1) ** k for k in range(3, E + 1)}
        np.testing.assert_allclose(pt.perk2_row(alpha, E, 16), T[:, col], atol=1e-15, rtol=0)


@pytest.mark.parametrize("order,E_list", [(2, [4, 8]), (3, [4, 8]), (3, [3, 6])])
def test_family_on_disk_spectrum(order, E_list):
    th = np.linspace(0, np.pi, 120)
    lam = -1.0 + np.exp(1j * th)
    fam = pt.build_family(order, E_list, lam, h_ref=1.0)
    assert pt.check_family(fam)
    ofam = pc.PerkFamily(fam.order, fam.S, fam.E, fam.c, fam.b, fam.a_sub)
    assert np.max(np.abs(pc.order_condition_residuals(ofam))) < 1e-12
    assert np.max(np.abs(pc.internal_consistency_residuals(ofam))) < 1e-15
    for r, E in enumerate(fam.E):
        coef = pc.stability_poly(pc.dense_A(fam.c, fam.a_sub[r]), fam.b)
        P = np.polynomial.Polynomial(coef)
        # the optimised step keeps the whole disk inside the (polygon-approximated) unit disk
        assert np.max(np.abs(P(fam.dt_opt[r] * lam))) <= 1.0 / math.cos(math.pi / 128) + 1e-9
        assert np.all(np.abs(coef[E + 1:]) < 1e-15)
    # steps grow with the number of stage evaluations (Sec. 3: dt_opt roughly linear in E)
    assert all(fam.dt_opt[i] < fam.dt_opt[i + 1] for i in range(len(fam.E) - 1))


def test_rechained_members_match_the_oracle_patterns():
    # the library's pattern construction (a linear solve per coefficient through the tableau's
    # polynomial) against the oracle's closed-form chain recursion (Sec. 3.2.4)
    import numpy as np
    from oracle import perk_coeffs as pc
    from paper_2403_05144_amd import coeffs
    f = pc.perk2_family([4, 6])
    fam = coeffs.Family(2, 6, [4, 6], f.c, f.b, f.a_sub)
    for kind, chain in pc.PAPER_CHAINS_S6_E4.items():
        got = coeffs.with_chains(fam, [chain, None])
        ref = pc.pattern_family([chain, list(range(6))], 6)
        np.testing.assert_array_equal(got.coupling, ref.coupling)
        np.testing.assert_allclose(got.a_sub, ref.a_val, rtol=1e-13, atol=1e-16)
    f8 = pc.perk2_family([4, 6, 8])
    fam8 = coeffs.Family(2, 8, [4, 6, 8], f8.c, f8.b, f8.a_sub)
    got = coeffs.with_chains(fam8, [[0, 3, 5, 7], [0, 1, 2, 3, 4, 7], None])
    ref = pc.pattern_family([[0, 3, 5, 7], [0, 1, 2, 3, 4, 7], list(range(8))], 8)
    np.testing.assert_array_equal(got.coupling, ref.coupling)
    np.testing.assert_allclose(got.a_sub, ref.a_val, rtol=1e-13, atol=1e-16)
