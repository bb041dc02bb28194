"""A tunable force-gradient family and its shadow Hamiltonian to dt^4 (CPU).

The family P(lam) Q(1/2) G(1 - 2 lam, xi) Q(1/2) P(lam), with the exact G
stage, contains Table 1's FG integrator at (1/6, 1/72) and PQPQP(alpha) at
(alpha, 0).  Its dt^2 and dt^4 shadow-Hamiltonian coefficients come from the
BCH series to fifth order (paper_0910_2950_amd/bch.py) and are kept in closed
form in tuning.py.  Pins:
  - the derivation reproduces what Table 1 prints: the dt^2 row of PQPQP(alpha)
    for every alpha, and the dt^4 rows of the FG and Campostrini integrators;
  - the closed forms equal the derivation as polynomials in (lam, xi);
  - on the lattice, for members away from the fourth-order point, the oracle's
    dH minus the predicted dt^2 + dt^4 terms (brackets measured at both ends of
    the trajectory) falls as dt^6, on 4^4 pure gauge and with Nf = 2 fermions;
  - the tuner returns the member whose predicted <dH^2> is smallest.
"""
import numpy as np
import pytest
import sympy as sp

from paper_0910_2950_amd import bch, synth, tuning

R = sp.Rational


def test_bch_reproduces_table1_rows():
    al = sp.Symbol("alpha")
    c2, c4 = bch.shadow_coefficients([("P", al, 0), ("Q", R(1, 2), 0), ("P", 1 - 2 * al, 0), ("Q", R(1, 2), 0),
                                      ("P", al, 0)])
    assert sp.simplify(c2["SST"] - (6 * al ** 2 - 6 * al + 1) / 12) == 0
    assert sp.simplify(c2["TST"] - (1 - 6 * al) / 24) == 0
    c2, c4 = bch.shadow_coefficients([("P", R(1, 6), 0), ("Q", R(1, 2), 0), ("G", R(2, 3), R(1, 72)),
                                      ("Q", R(1, 2), 0), ("P", R(1, 6), 0)])
    assert c2 == {"SST": 0, "TST": 0}
    # Table 1, FG: dH = + dt^4 Delta(36 STSST + 72 STTST + 126 TTSST + 54 TTTST) / 155520
    assert {k: c4[k] * 155520 for k in tuning.FG_KEYS4} == {"STSST": -36, "STTST": -72, "TTSST": -126,
                                                           "TTTST": -54}
    # Campostrini: the weights as functions of c, fourth order where c^3 = 2
    c = sp.Symbol("c")
    w1, w0 = 1 / (2 - c), -c / (2 - c)
    c2, c4 = bch.shadow_coefficients([("Q", w1 / 2, 0), ("P", w1, 0), ("Q", (w1 + w0) / 2, 0), ("P", w0, 0),
                                      ("Q", (w1 + w0) / 2, 0), ("P", w1, 0), ("Q", w1 / 2, 0)])
    cr = sp.root(2, 3)
    assert all(sp.simplify(c2[k].subs(c, cr)) == 0 for k in tuning.FG_KEYS2)
    c4 = {k: v.subs(c, cr) for k, v in c4.items()}
    c2n, c4n = 2 ** (1 / 3), 4 ** (1 / 3)
    row = {"STSST": 180 * c4n + 240 * c2n + 312, "STTST": 60 * c4n + 80 * c2n + 104, "TTSST": 20 * c2n + 32,
           "TTTST": 5 * c2n + 8}
    for k in tuning.FG_KEYS4:  # Table 1, Campostrini: the same row with the opposite sign, over 34560
        assert abs(float(c4[k]) * 34560 - row[k]) < 1e-9 * row[k], k


def test_closed_forms_equal_the_derivation():
    lam, xi = sp.symbols("lam xi")
    stages = [(k, sp.nsimplify(w), sp.nsimplify(x)) for k, w, x in tuning.fg_family_stages(lam, xi)]
    c2, c4 = bch.shadow_coefficients(stages)
    f2, f4 = tuning.fg_family_coeffs(lam, xi)
    for k in tuning.FG_KEYS2:
        assert sp.simplify(sp.nsimplify(f2[k]) - c2[k]) == 0, k
    for k in tuning.FG_KEYS4:
        assert sp.simplify(sp.nsimplify(f4[k]) - c4[k]) == 0, k


MEMBERS = [(0.19, 0.008), (0.15, 0.02)]
CASES = [("gauge", (4, 4, 4, 4), 6.0, 0.0), ("nf2", (4, 4, 2, 2), 5.6, 0.155)]


@pytest.mark.parametrize("case,dims,beta,kappa", CASES)
@pytest.mark.parametrize("lam,xi", MEMBERS)
def test_family_dH_follows_its_shadow_hamiltonian(orc, case, dims, beta, kappa, lam, xi):
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + (10 if case == "gauge" else 11), fermions=kappa != 0)
    kw = dict(kappa=kappa, phi=orc.pf_heatbath(dims, kappa, U0, eta)) if kappa else {}
    stages = tuning.fg_family_stages(lam, xi)
    b0 = orc.brackets4(dims, beta, U0, P0, h=1e-3, **kw)
    res, dhs = [], []
    for n in (8, 16, 32, 64):
        U1, P1, dH, _, status = orc.trajectory(dims, beta, stages, 1.0, n, U0, P0, fg_exact=True, **kw)
        assert status == 0
        b1 = orc.brackets4(dims, beta, U1, P1, h=1e-3, **kw)
        dB = {k: b1[k] - b0[k] for k in tuning.FG_KEYS2 + tuning.FG_KEYS4}
        pred = float(tuning.predicted_dh_fg_family(lam, xi, dB, 1.0 / n))
        res.append(dH - pred)
        dhs.append(dH)
    ratios = [abs(res[i] / res[i + 1]) for i in range(len(res) - 1)]
    assert all(48 < r < 80 for r in ratios), (ratios, res)
    assert abs(res[-1]) < 0.01 * abs(dhs[-1])
    # these members are second order: dH itself falls as dt^2
    r2 = [abs(dhs[i] / dhs[i + 1]) for i in range(3)]
    assert all(3 < r < 5 for r in r2), r2


def test_tuner_finds_the_best_member():
    rng = np.random.default_rng(5)
    true = (0.175, 0.011)
    # bracket changes for which the member `true` predicts dH = 0 on every trajectory
    # (dt^2 and dt^4 terms cancelling), plus the inert direction of the others
    dt = 1.0 / 24
    dB = {k: rng.normal(size=16) for k in tuning.FG_KEYS2 + tuning.FG_KEYS4}
    c2, c4 = tuning.fg_family_coeffs(*true)
    rest = -(dt ** 2) * sum(c2[k] * dB[k] for k in ("TST",)) - (dt ** 4) * sum(c4[k] * dB[k] for k in tuning.FG_KEYS4)
    dB["SST"] = rest / ((dt ** 2) * c2["SST"])
    assert np.allclose(tuning.predicted_dh_fg_family(*true, dB, dt), 0.0, atol=1e-12)
    lam, xi = tuning.tune_fg_family(dB, dt)
    assert abs(lam - true[0]) < 2e-3 and abs(xi - true[1]) < 2e-4, (lam, xi)
    # the fourth-order point when only the dt^2 brackets change
    dB2 = {k: (rng.normal(size=8) if k in tuning.FG_KEYS2 else np.zeros(8)) for k in dB}
    lam, xi = tuning.tune_fg_family(dB2, dt)
    assert abs(lam - 1 / 6) < 1e-3 and abs(xi - 1 / 72) < 1e-4, (lam, xi)
