"""Pins of the oracle's Hasenbusch (mass-preconditioned) pseudofermion terms
and its nested-time-scale integrator (no GPU).

S_F = S_1 + S_2, S_1 = phi1^+ (Mhat2^+ Mhat2)^-1 phi1 at kappa2 < kappa,
S_2 = chi^+ (Mhat^+ Mhat)^-1 chi with chi = Mhat2^+ phi2.
"""
import numpy as np
import pytest
import scipy.linalg

from paper_0910_2950_amd import synth
from oracle.oracle import table

T = 0.5j * synth.gell_mann()
K, K2 = 0.155, 0.140


def start(dims, seed):
    U, P, eta1, _ = synth.hot_start(dims, seed, fermions=True)
    eta2 = synth.gaussian_noise(synth.rng(seed + 1), dims)
    return U, P, eta1, eta2


def test_heatbath_identities(orc):
    dims = (4, 4, 2, 2)
    U, _, eta1, eta2 = start(dims, 1)
    phi1 = orc.pf_heatbath(dims, K2, U, eta1)
    s1, _ = orc.pf_action(dims, K2, U, phi1)
    assert abs(s1 - np.vdot(eta1, eta1).real) < 1e-12 * s1
    phi2 = orc.hasen_heatbath(dims, K, K2, U, eta2)
    s2, _ = orc.hasen_action(dims, K, K2, U, phi2)
    e2 = np.vdot(eta2, eta2).real
    assert abs(s2 - e2) < 1e-12 * e2


def test_ratio_term_vanishes_at_equal_kappa(orc):
    """kappa2 = kappa: S_2 = phi2^+ phi2 does not depend on U, so its force is zero."""
    dims = (2, 2, 2, 2)
    U, _, _, eta2 = start(dims, 2)
    phi2 = eta2
    s2, X2 = orc.hasen_action(dims, K, K, U, phi2)
    assert abs(s2 - np.vdot(phi2, phi2).real) < 1e-12 * s2
    F = orc.hasen_force(dims, K, K, U, phi2, X2)
    assert np.max(np.abs(F)) < 1e-11


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 2, 2)])
def test_ratio_force_finite_difference(orc, dims):
    U, _, _, eta2 = start(dims, 3)
    phi2 = orc.hasen_heatbath(dims, K, K2, U, eta2)
    _, X2 = orc.hasen_action(dims, K, K2, U, phi2)
    F = orc.hasen_force(dims, K, K2, U, phi2, X2)
    V = synth.volume(dims)
    h = 1e-5
    worst = 0.0
    for (mu, i) in [(0, 0), (3, V - 1), (3, 0), (1, V // 2 + 1)]:
        for a in range(8):
            Up, Um = U.copy(), U.copy()
            Up[mu, i] = scipy.linalg.expm(h * T[a]) @ U[mu, i]
            Um[mu, i] = scipy.linalg.expm(-h * T[a]) @ U[mu, i]
            fd = -(orc.hasen_action(dims, K, K2, Up, phi2)[0] - orc.hasen_action(dims, K, K2, Um, phi2)[0]) / (2 * h)
            worst = max(worst, abs(fd - F[mu, i, a]))
    assert worst < 1e-6 * max(1.0, np.max(np.abs(F)))


def test_nested_driver_reduces_to_single_level(orc):
    """One level with all terms and no Hasenbusch is the pinned single-level trajectory."""
    dims = (4, 4, 2, 2)
    U, P, eta1, _ = start(dims, 4)
    a = orc.trajectory(dims, 5.6, table("FG"), 1.0, 4, U, P, kappa=K, eta=eta1)
    b = orc.trajectory_nested(dims, 5.6, [(table("FG"), 7, 1)], 1.0, 4, U, P, kappa=K, eta1=eta1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # dH: the fermion part is summed globally here and per site there (rounding only)
    assert abs(a[2] - b[2]) < 1e-10 and a[3]["solves"] == b[3]["solves"]


def levels_fg3():
    """S_2 on the outer scale, S_1 on the middle one, S_G innermost (FG on each)."""
    return [(table("FG"), 4, 1), (table("FG"), 2, 2), (table("FG"), 1, 2)]


def test_nested_hasenbusch_energy_and_order(orc):
    dims = (4, 4, 2, 2)
    U, P, eta1, eta2 = start(dims, 5)
    dh = []
    for n in (4, 8):
        _, _, d, st, status = orc.trajectory_nested(dims, 5.6, levels_fg3(), 1.0, n, U, P, kappa=K, kappa2=K2,
                                                    eta1=eta1, eta2=eta2)
        assert status == 0
        dh.append(abs(d))
    assert dh[1] < 1e-3
    assert 10 < dh[0] / dh[1] < 24, dh   # fourth order in the outer step (inner scales refined with it)


def test_nested_solve_count(orc):
    """Outer FG on S_2: 3n+1 solves; middle FG (2 steps per outer Q, two Q per
    step) on S_1: (3*2+1) per Q; plus the phi2 heatbath and the two final actions."""
    dims = (2, 2, 2, 2)
    U, P, eta1, eta2 = start(dims, 6)
    n = 2
    _, _, _, st, _ = orc.trajectory_nested(dims, 5.6, levels_fg3(), 1.0, n, U, P, kappa=K, kappa2=K2,
                                           eta1=eta1, eta2=eta2, tol=1e-8)
    outer = 3 * n + 1
    middle = (2 * n) * (3 * 2 + 1)
    assert st["solves"] == outer + middle + 1 + 2


def test_nested_exact_form_reduces_to_single_level(orc):
    """One level, exact G stages: the pinned single-level exact trajectory."""
    dims = (4, 4, 2, 2)
    U, P, eta1, _ = start(dims, 6)
    a = orc.trajectory(dims, 5.6, table("FG"), 1.0, 3, U, P, kappa=K, eta=eta1, fg_exact=True)
    b = orc.trajectory_nested(dims, 5.6, [(table("FG"), 3, 1)], 1.0, 3, U, P, kappa=K, eta1=eta1, fg_exact=True)
    assert b[4] == 0 and a[3]["solves"] == b[3]["solves"]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and abs(a[2] - b[2]) < 1e-10


def test_nested_exact_form_order_and_reversibility(orc):
    """S_F on the outer scale, S_G on the inner one (two sub-steps), FG with
    exact G stages on both: dH falls as dt^4 and stays within a few percent of
    the displacement form's; the pure-gauge nested exact trajectory reverses."""
    dims = (4, 4, 2, 2)
    U, P, eta1, _ = start(dims, 7)
    levels = [(table("FG"), 2, 1), (table("FG"), 1, 2)]
    dh, dh_disp = [], []
    for n in (8, 16):
        _, _, d, _, status = orc.trajectory_nested(dims, 5.6, levels, 1.0, n, U, P, kappa=K, eta1=eta1,
                                                   fg_exact=True)
        assert status == 0
        dh.append(abs(d))
        dh_disp.append(abs(orc.trajectory_nested(dims, 5.6, levels, 1.0, n, U, P, kappa=K, eta1=eta1)[2]))
    assert abs(np.log2(dh[0] / dh[1]) - 4) < 0.3, dh
    assert abs(dh[1] / dh_disp[1] - 1) < 0.2, (dh, dh_disp)
    two = [(table("FG"), 1, 1), (table("FG"), 1, 2)]
    Ug1, Pg1, dg, _, _ = orc.trajectory_nested(dims, 5.6, two, 1.0, 3, U, P, fg_exact=True)
    Ug2, Pg2, dg2, _, _ = orc.trajectory_nested(dims, 5.6, two, 1.0, 3, Ug1, -Pg1, fg_exact=True)
    assert np.max(np.abs(Ug2 - U)) < 1e-12 and np.max(np.abs(-Pg2 - P)) < 1e-11 and abs(dg + dg2) < 1e-10


def test_nested_exact_hasenbusch_order_and_solves(orc):
    """Three nested FG scales (S_2, S_1, S_G) with exact G stages: dH falls as
    dt^4, close to the displacement form's; each G stage of a fermion level
    costs one solve more than its force (d_V X), like the displaced force."""
    dims = (4, 4, 2, 2)
    U, P, eta1, eta2 = start(dims, 8)
    args = dict(kappa=K, kappa2=K2, eta1=eta1, eta2=eta2)
    dh, dd = [], []
    for n in (4, 8):
        Ue, Pe, d, st, status = orc.trajectory_nested(dims, 5.6, levels_fg3(), 1.0, n, U, P, fg_exact=True, **args)
        assert status == 0
        Ud, Pd, d2, st2, _ = orc.trajectory_nested(dims, 5.6, levels_fg3(), 1.0, n, U, P, **args)
        dh.append(abs(d))
        dd.append(abs(d2))
        assert st["solves"] == st2["solves"]
    assert abs(np.log2(dh[0] / dh[1]) - 4) < 0.4, dh
    assert abs(dh[1] / dd[1] - 1) < 0.3, (dh, dd)


def test_nested_exact_form_refused_for_smearing(orc):
    dims = (4, 4, 2, 2)
    U, P, eta1, eta2 = start(dims, 8)
    r = orc.trajectory_nested(dims, 5.6, [(table("FG"), 3, 1)], 1.0, 2, U, P, kappa=K, eta1=eta1, fg_exact=True,
                              stout_rho=0.1, stout_n=1)
    assert r[4] == -2


def _alg(p):
    T = 0.5j * synth.gell_mann()
    return np.einsum("...a,aij->...ij", p, T)


def _comp(M):
    T = 0.5j * synth.gell_mann()
    return -2 * np.einsum("aij,...ji->...a", T, M).real


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 2, 2)])
def test_hasen_force_tangent_finite_difference(orc, dims):
    """The S_2 force gradient against Richardson-extrapolated central
    differences of the (separately pinned) S_2 force, its X2 re-solved at
    each displaced field."""
    U = synth.haar_su3(synth.rng(140), 4 * synth.volume(dims)).reshape(4, -1, 3, 3)
    phi2 = synth.gaussian_noise(synth.rng(141), dims)
    Vd = synth.rng(142).standard_normal((4, synth.volume(dims), 8))
    _, X2 = orc.hasen_action(dims, K, K2, U, phi2)
    J = orc.hasen_force_tangent(dims, K, K2, U, phi2, X2, Vd)

    def F2(W):
        _, Xw = orc.hasen_action(dims, K, K2, W, phi2, tol=1e-15)
        return orc.hasen_force(dims, K, K2, W, phi2, Xw)

    def central(h):
        return (F2(orc.link_update(dims, h, Vd, U)) - F2(orc.link_update(dims, -h, Vd, U))) / (2 * h)

    h = 2e-3
    fd = (4 * central(h / 2) - central(h)) / 3
    assert np.max(np.abs(fd - J)) < 1e-9 * np.max(np.abs(J))


def test_hasen_force_tangent_chart_commutator(orc):
    """<W, J_V F_2> - <V, J_W F_2> = <[W, V], F_2>: pins the explicit link
    terms of both force parts (the solve terms are symmetric)."""
    dims = (4, 4, 2, 2)
    U = synth.haar_su3(synth.rng(143), 4 * synth.volume(dims)).reshape(4, -1, 3, 3)
    phi2 = synth.gaussian_noise(synth.rng(144), dims)
    Vd, Wd = synth.rng(145).standard_normal((2, 4, synth.volume(dims), 8))
    _, X2 = orc.hasen_action(dims, K, K2, U, phi2)
    JV = orc.hasen_force_tangent(dims, K, K2, U, phi2, X2, Vd)
    JW = orc.hasen_force_tangent(dims, K, K2, U, phi2, X2, Wd)
    F = orc.hasen_force(dims, K, K2, U, phi2, X2)
    lhs = np.sum(Wd * JV) - np.sum(Vd * JW)
    rhs = np.sum(_comp(_alg(Wd) @ _alg(Vd) - _alg(Vd) @ _alg(Wd)) * F)
    assert abs(lhs - rhs) < 1e-11 * np.sum(np.abs(Wd * JV))
