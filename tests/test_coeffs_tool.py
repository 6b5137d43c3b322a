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


# ---- the product's optimiser against closed forms (no oracle code involved)
@pytest.mark.parametrize("E", [4, 8, 16])
def test_optimiser_second_order_disk_closed_form(E):
    # the largest disk {|z + r| <= r} inside the stability region of an E-stage second-order
    # method has r = E - 1 (the shifted polynomial 1 - (E - 1) + ... of the circle), so on the
    # unit disk centred at -1 the optimal step is E - 1
    th = np.linspace(0, np.pi, 200)
    lam = -1.0 + np.exp(1j * th)
    dt, _ = pt.optimise(lam, 2, E)
    assert abs(dt - (E - 1)) <= 2e-4 * (E - 1), dt   # polygon and bisection tolerances


def test_optimiser_fixed_polynomials_on_the_real_axis():
    # E = p leaves no free coefficient: the step is the real stability limit of the truncated
    # exponential; on the spectrum [-1, 0] that is 2 for 1 + z + z^2/2 and the real root x of
    # 1 - x + x^2/2 - x^3/6 = -1 (2.5127...) for the third-order one
    lam = -np.linspace(1e-3, 1.0, 400).astype(complex)
    dt2, _ = pt.optimise(lam, 2, 2)
    assert abs(dt2 - 2.0) < 1e-6
    x = [r.real for r in np.roots([-1 / 6, 1 / 2, -1, 2]) if abs(r.imag) < 1e-12 and r.real > 0][0]
    dt3, _ = pt.optimise(lam, 3, 3)
    assert abs(dt3 - x) < 1e-6 and abs(x - 2.5127453266183) < 1e-9
