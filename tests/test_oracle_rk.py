"""Pins of the oracle's RK / stage-conversion arithmetic against facts fixed by the
mathematics (eq. rk_schemes, eq. rk_crrection, eqs. fc_1 / fc_2)."""
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import rk

TABS = [rk.RK4, rk.SSPRK3]


def _rk_stages_direct(tab, Lmat, y, dt):
    """Stages of one RK step for y' = L y computed straight from eq. rk_schemes."""
    a = np.array([[float(x) for x in r] for r in tab.a])
    ks = []
    for s in range(tab.p):
        arg = y.copy()
        for q in range(s):
            arg = arg + dt * a[s, q] * ks[q]
        ks.append(Lmat @ arg)
    return np.array(ks)


@pytest.mark.parametrize("tab", TABS, ids=lambda t: t.name)
def test_stage_relation_linear_ode(tab):
    """K = C P D with D_j = L^j y for a linear ODE (eq. rk_crrection, reading K = C P D)."""
    rng = np.random.default_rng(1)
    Lm = rng.standard_normal((3, 3))
    y = rng.standard_normal(3)
    dt = 0.37
    K = _rk_stages_direct(tab, Lm, y, dt)
    C = np.array([[float(x) for x in r] for r in rk.c_matrix(tab)])
    D = np.array([np.linalg.matrix_power(Lm, j) @ y for j in range(1, tab.p + 1)])
    P = np.diag([dt ** j for j in range(tab.p)])
    assert np.abs(C @ P @ D - K).max() <= 1e-14 * np.abs(K).max()
    # the printed order P C does not reproduce the stages
    assert np.abs(P @ C @ D - K).max() > 1e-2


@pytest.mark.parametrize("tab", TABS, ids=lambda t: t.name)
def test_same_level_case_is_tableau(tab):
    W = rk.conversion_weights(tab, 0, 1)
    for s in range(tab.p):
        assert W[s] == list(tab.a[s])


@pytest.mark.parametrize("tab", TABS, ids=lambda t: t.name)
@pytest.mark.parametrize("case", rk.CASES)
def test_row_sums(tab, case):
    """With all stages equal (u' = const) Y_s = U0 + (Delta + c_s dt_r) k."""
    d, r = case
    W = rk.conversion_weights(tab, d, r)
    for s in range(tab.p):
        assert sum(W[s]) == d + tab.c[s]


@pytest.mark.parametrize("tab", TABS, ids=lambda t: t.name)
def test_taylor_at_source_end_is_rk_update(tab):
    """At Delta = dt_n the Taylor part equals the RK update: b^T C = (1/j!) for
    methods of order p on linear problems."""
    W = rk.conversion_weights(tab, 2, 2)
    assert W[0] == [2 * x for x in tab.b]


@pytest.mark.parametrize("tab", TABS, ids=lambda t: t.name)
def test_conversion_round_trip(tab):
    """M_{rho -> 1} M_{1 -> rho} = I (fig. oct_2_1_nuts: M and its inverse)."""
    for rho in (Fr(2), Fr(1, 2)):
        T1 = rk.converted_stages(tab, 0, rho)
        T2 = rk.converted_stages(tab, 0, 1 / rho)
        p = tab.p
        prod = [[sum(T1[i][k] * T2[k][j] for k in range(p)) for j in range(p)] for i in range(p)]
        assert prod == [[Fr(int(i == j)) for j in range(p)] for i in range(p)]


def test_hand_derived_rk4_entries():
    """Entries derived by hand from the definitions (RK4):
    (delta, rho) = (0, 1/2), stage 3: Y_3 = U0 + dt_r a_32 k~_2, and
    k~_2 = sum_j C_2j rho^{1-j} (C^{-1})_j. = row1(C^{-1}) + row2(C^{-1})
         = (1,0,0,0) + (-2,2,0,0), so w^_3 = (-1/2, 1, 0, 0).
    (0, 2), stage 2: k~_1 = C_11 D_1 = (C^{-1})_1. = (1,0,0,0), w^_2 = (1/2, 0, 0, 0)."""
    W = rk.conversion_weights(rk.RK4, 0, Fr(1, 2))
    assert W[2] == [Fr(-1, 2), Fr(1), Fr(0), Fr(0)]
    W = rk.conversion_weights(rk.RK4, 0, 2)
    assert W[1] == [Fr(1, 2), Fr(0), Fr(0), Fr(0)]


@pytest.mark.parametrize("tab", TABS, ids=lambda t: t.name)
@pytest.mark.parametrize("case", rk.CASES)
def test_conversion_order_on_linear_ode(tab, case):
    """For y' = L y the source stages determine D_j = L^j y0 exactly, so with a
    common start (delta = 0) the converted stage states equal the receiver's own
    RK stage states to rounding.  With delta = 1 the Taylor shift is truncated at
    order p and the difference to the receiver's stages started from the exact
    solution is O(dt^(p+1)): halving every step divides it by ~2^(p+1)."""
    d, r = float(case[0]), float(case[1])
    rng = np.random.default_rng(7)
    Lm = rng.standard_normal((4, 4))
    Lm = Lm - Lm.T - 0.3 * np.eye(4)
    y0 = rng.standard_normal(4)
    W = np.array([[float(x) for x in row] for row in rk.conversion_weights(tab, case[0], case[1])])
    a = np.array([[float(x) for x in row] for row in tab.a])
    errs = []
    for dtr in (0.04, 0.02, 0.01):
        dtn = r * dtr
        K = _rk_stages_direct(tab, Lm, y0, dtn)              # source record
        yr = expm(d * dtr * Lm) @ y0                           # exact state at receiver start
        krec = _rk_stages_direct(tab, Lm, yr, dtr)
        worst = 0.0
        for s in range(tab.p):
            y_conv = y0 + dtr * (W[s] @ K)
            y_true = yr + dtr * sum(a[s, q] * krec[q] for q in range(s))
            worst = max(worst, np.abs(y_conv - y_true).max())
        errs.append(worst)
    if d == 0.0:
        assert max(errs) <= 1e-13 * np.abs(y0).max(), errs
    else:
        rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert min(rates) > tab.p + 1 - 0.35, (errs, rates)


def test_float_weights_correctly_rounded():
    W = rk.weight_table(rk.RK4)
    Wf = rk.weight_table_f64(rk.RK4)
    for c in range(4):
        for s in range(4):
            for i in range(4):
                x = W[c][s][i]
                assert Fr(Wf[c, s, i]) == Fr(x) or abs(Fr(Wf[c, s, i]) - x) <= abs(x) * Fr(1, 2 ** 53)
