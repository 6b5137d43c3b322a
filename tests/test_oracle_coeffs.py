"""Pins of the oracle's P-ERK tableau code against the paper and closed forms (CPU only)."""
import math
import os

import numpy as np
import pytest

from oracle import perk_coeffs as pc
from oracle.godunov1d import upwind_matrix

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_table():
    rows = [l.split() for l in open(os.path.join(GOLD, "perk2_8_16_table.txt")) if l.strip() and l[0] != "#"]
    return np.array([[float(x) for x in r] for r in rows])


def test_perk2_8_16_table_matches_paper():
    # eq. (PERK_8_16_CompactForm): closed-form disk-optimal polynomials + eq. (PERKCoeffsConstruction)
    T = load_table()
    fam = pc.perk2_family([8, 16])
    assert fam.S == 16
    np.testing.assert_allclose(fam.c * 30, T[:, 1], atol=1e-13)
    np.testing.assert_allclose(fam.a_sub[0], T[:, 2], atol=1e-15, rtol=0)
    np.testing.assert_allclose(fam.a_sub[1], T[:, 3], atol=1e-15, rtol=0)


def test_perk2_6_stage_structure():
    # eq. (PERK_ButcherTableauClassic): S = 6, c_i = (i-1)/10, E=4 member evaluates K1,K4,K5,K6
    fam = pc.perk2_family([4, 6])
    np.testing.assert_allclose(fam.c, np.arange(6) / 10.0, atol=1e-16)
    assert pc.member_stage_evaluations(fam.a_sub[0], fam.c, fam.b) == [1, 4, 5, 6]
    assert pc.member_stage_evaluations(fam.a_sub[1], fam.c, fam.b) == [1, 2, 3, 4, 5, 6]
    # zero pattern of a_{i,i-1}: nonzero exactly for i >= S - E + 3
    for r, E in enumerate(fam.E):
        nz = [i + 1 for i in range(fam.S) if fam.a_sub[r][i] != 0.0]
        assert nz == list(range(fam.S - E + 3, fam.S + 1))


def test_dt_0_21875_from_disk_polynomial():
    # Sec. 3.2.2: N = 64, dx = 2/64, the E=8 method's maximum stable step is 0.21875
    N = 64
    L = upwind_matrix(np.full(N, 2.0 / N))
    eigs = np.linalg.eigvals(L)
    fam = pc.perk2_family([8])
    coef = pc.stability_poly(pc.dense_A(fam.c, fam.a_sub[0]), fam.b)
    h = pc.max_stable_step(coef, eigs)
    assert abs(h - 0.21875) < 1e-6 * 0.21875


@pytest.mark.parametrize("p,E", [(2, 4), (2, 8), (1, 6)])
def test_lp_optimiser_disk_closed_form(p, E):
    # Optimal step for a disk spectrum of radius 1 (centre -1): E-1 for p=2, E for p=1
    # (closed forms of the cited optimal-polynomial literature).  The circumscribed polygon
    # lets |P| reach 1/cos(pi/M), so the LP result may exceed the optimum by a hair.
    th = np.linspace(0, 2 * np.pi, 400, endpoint=False)
    eigs = -1.0 + np.exp(1j * th)
    h, alpha = pc.optimize_alpha(eigs, p, E, M=128)
    exact = (E - 1) if p == 2 else E
    assert exact * 0.98 < h <= exact * 1.02
    coef = np.zeros(E + 1)
    for j in range(p + 1):
        coef[j] = 1.0 / math.factorial(j)
    for j, v in alpha.items():
        coef[j] = v
    P = np.polynomial.Polynomial(coef)
    assert np.max(np.abs(P(h * eigs))) <= 1.0 / np.cos(np.pi / 128) + 1e-9


@pytest.mark.parametrize("E_list", [[4, 8], [8, 16], [3, 6, 12], [4, 8, 16]])
def test_perk2_order_consistency_and_polynomial(E_list):
    fam = pc.perk2_family(E_list)
    assert np.max(np.abs(pc.order_condition_residuals(fam))) < 1e-14
    assert np.max(np.abs(pc.internal_consistency_residuals(fam))) < 1e-15
    for r, E in enumerate(fam.E):
        coef = pc.stability_poly(pc.dense_A(fam.c, fam.a_sub[r]), fam.b)
        alpha = pc.disk_optimal_alpha_p2(E)
        assert coef[0] == 1.0 and abs(coef[1] - 1) < 1e-15 and abs(coef[2] - 0.5) < 1e-15
        for k in range(3, E + 1):
            assert abs(coef[k] - alpha[k]) <= 1e-12 * abs(alpha[k])
        assert np.all(np.abs(coef[E + 1:]) < 1e-18)


def test_perk3_shu_osher_special_case():
    # E = S = 3 reproduces the Shu-Osher base, eq. (PERK_ThirdOrderShuOsher)
    a = pc.perk3_member({}, 3, 3)
    A = pc.dense_A(pc.perk3_abscissae(3), a)
    np.testing.assert_allclose(A, [[0, 0, 0], [1, 0, 0], [0.25, 0.25, 0]], atol=1e-16)
    np.testing.assert_allclose(pc.perk3_weights(3), [1 / 6, 1 / 6, 2 / 3], atol=1e-16)


def test_perk3_family_from_optimised_polynomials():
    # Sec. 4.3.2: optimise on a disk spectrum, solve for positive a_i, verify order 3
    th = np.linspace(0, 2 * np.pi, 200, endpoint=False)
    eigs = -1.0 + np.exp(1j * th)
    alphas = {}
    for E in (4, 8):
        h, al = pc.optimize_alpha(eigs, 3, E, M=128)
        alphas[E] = al
    fam = pc.perk3_family([4, 8], alphas)
    assert np.max(np.abs(pc.order_condition_residuals(fam))) < 1e-12
    assert np.max(np.abs(pc.internal_consistency_residuals(fam))) < 1e-15
    for r, E in enumerate(fam.E):
        a = fam.a_sub[r]
        rows = np.arange(fam.S - E + 2, fam.S)     # 0-based rows with a free a_{i,i-1}
        assert np.all(a[rows] > 0) and np.all(a[rows] < fam.c[rows])
        coef = pc.stability_poly(pc.dense_A(fam.c, a), fam.b)
        for k in range(4, E + 1):
            assert abs(coef[k] - alphas[E][k]) <= 1e-10 * max(1e-6, abs(alphas[E][k]))
        assert abs(coef[3] - 1 / 6) < 1e-13
    # shared b and c across members (eq. Conservation)
    assert fam.b.shape == (fam.S,) and fam.c.shape == (fam.S,)


def test_perk3_abscissae():
    # eq. (Free_Timesteps)
    c = pc.perk3_abscissae(8)
    np.testing.assert_allclose(c[:6], np.arange(6) / 5.0, atol=1e-16)
    assert c[6] == 1.0 and c[7] == 0.5
