"""Pins of the oracle's improved gauge action (no GPU).

S_G = beta sum_x [c0 sum_{mu<nu} (1 - ReTr P_{mu nu}(x)/3) + c1 sum_{mu!=nu} (1 - ReTr R_{mu nu}(x)/3)],
c0 = 1 - 8 c1, R the 2x1 rectangle (two links along mu, one along nu).  The
conclusions of the paper state that the force-gradient construction carries
over to any common action; this is the first one beyond Wilson's.  Checks:

  - the action against a brute-force numpy sum over shifted link arrays (a
    different enumeration from the oracle's path walker);
  - closed forms: a constant abelian flux through one plane (plaquettes see
    the flux f, rectangles 2f) and a single non-trivial link (18 rectangles
    hold it on a lattice with every extent >= 3; on 2^4 the six rectangles
    that run twice along a direction of extent 2 contain the link and its
    inverse and drop out, leaving 12); the single-link force in closed form;
  - gauge invariance of S and covariance of F;
  - the force as the finite-difference gradient of the action, and the force
    tangent as the finite-difference derivative of the force, at c1 = -1/12
    (tree-level Symanzik) and -0.331 (Iwasaki);
  - trajectories: reversibility and the dt^4 scaling of dH for the FG
    integrator (a force that was not the gradient of the action in H would
    stop dH from falling at the integrator's order).
"""
import numpy as np
import pytest
import scipy.linalg

from paper_0910_2950_amd import synth
from oracle.oracle import table

L2 = (2, 2, 2, 2)
L4 = (4, 4, 4, 4)
T = 0.5j * synth.gell_mann()
C1S = [-1.0 / 12.0, -0.331]


def rand_links(dims, seed):
    return synth.haar_su3(synth.rng(seed), 4 * synth.volume(dims)).reshape(4, -1, 3, 3)


def _grid(dims, U):
    """links as (4, Lt, Lz, Ly, Lx, 3, 3) so that direction mu is array axis 4 - mu"""
    Lx, Ly, Lz, Lt = dims
    return U.reshape(4, Lt, Lz, Ly, Lx, 3, 3)


def _at(A, mu, k):
    """field A (Lt, Lz, Ly, Lx, ...) read at x + k mu"""
    return np.roll(A, -k, axis=3 - mu)


def _dag(A):
    return np.conj(np.swapaxes(A, -1, -2))


def brute_force_sums(dims, U):
    """(sum over plaquettes of 1 - ReTr/3, sum over rectangles of 1 - ReTr/3)"""
    G = _grid(dims, U)
    sp = sr = 0.0
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            Um, Un = G[mu], G[nu]
            if mu < nu:
                P = Um @ _at(Un, mu, 1) @ _dag(_at(Um, nu, 1)) @ _dag(Un)
                sp += np.sum(1 - np.trace(P, axis1=-2, axis2=-1).real / 3)
            R = (Um @ _at(Um, mu, 1) @ _at(Un, mu, 2) @ _dag(_at(_at(Um, mu, 1), nu, 1))
                 @ _dag(_at(Um, nu, 1)) @ _dag(Un))
            sr += np.sum(1 - np.trace(R, axis1=-2, axis2=-1).real / 3)
    return sp, sr


@pytest.mark.parametrize("dims", [L2, (4, 2, 2, 4), (6, 4, 2, 4)])
def test_action_matches_brute_force(orc, dims):
    U = rand_links(dims, 301)
    sp, sr = brute_force_sums(dims, U)
    for c1 in [0.0] + C1S:
        S = orc.gauge_action(dims, 5.0, U, c1)
        ref = 5.0 * ((1 - 8 * c1) * sp + c1 * sr)
        assert abs(S - ref) < 1e-12 * abs(ref), c1


def _gauge_transform(dims, U, G):
    """U_mu(x) -> G(x) U_mu(x) G(x+mu)^+"""
    V = synth.volume(dims)
    c = np.stack(np.unravel_index(np.arange(V), dims[::-1])[::-1], axis=1)
    out = np.empty_like(U)
    for mu in range(4):
        cp = c.copy()
        cp[:, mu] = (cp[:, mu] + 1) % dims[mu]
        ip = cp[:, 0] + dims[0] * (cp[:, 1] + dims[1] * (cp[:, 2] + dims[2] * cp[:, 3]))
        out[mu] = G @ U[mu] @ _dag(G[ip])
    return out


@pytest.mark.parametrize("c1", C1S)
def test_constant_flux_closed_form(orc, c1):
    """U_y(x) = diag(e^{ifx}, e^{-ifx}, 1), f = 2 pi k / Lx, other links 1:
    every (x,y) plaquette is diag(e^{if}, e^{-if}, 1) and both orientations of
    the (x,y) rectangles carry 2f; every other loop is 1.  Gauge-rotated."""
    dims = (8, 4, 2, 4)
    V = synth.volume(dims)
    f = 2 * np.pi * 3 / dims[0]
    U = synth.unit_links(dims)
    x = np.arange(V) % dims[0]
    U[1, :, 0, 0] = np.exp(1j * f * x)
    U[1, :, 1, 1] = np.exp(-1j * f * x)
    beta, c0 = 5.3, 1 - 8 * c1
    ref = beta * V * (c0 * (1 - (2 * np.cos(f) + 1) / 3) + 2 * c1 * (1 - (2 * np.cos(2 * f) + 1) / 3))
    Ug = _gauge_transform(dims, U, synth.haar_su3(synth.rng(302), V))
    for W in (U, Ug):
        assert abs(orc.gauge_action(dims, beta, W, c1) - ref) < 1e-11 * abs(ref)


@pytest.mark.parametrize("dims,nrect", [(L4, 18), ((4, 4, 4, 6), 18), (L2, 12)])
@pytest.mark.parametrize("c1", C1S)
def test_one_link_closed_form(orc, dims, nrect, c1):
    beta, th = 5.6, 0.9
    U = synth.unit_links(dims)
    mu, site = 2, 3
    U[mu, site] = np.diag([np.exp(1j * th / 2), np.exp(-1j * th / 2), 1.0])
    c0 = 1 - 8 * c1
    S = orc.gauge_action(dims, beta, U, c1)
    assert abs(S - beta * (6 * c0 + nrect * c1) * (1 - (2 * np.cos(th / 2) + 1) / 3)) < 1e-12
    F = orc.gauge_force(dims, beta, U, c1)
    ref = np.zeros(8)
    ref[2] = -beta * (6 * c0 + nrect * c1) * np.sin(th / 2) / 3
    assert np.max(np.abs(F[mu, site] - ref)) < 1e-13


def test_gauge_invariance_and_covariance(orc):
    dims, beta, c1 = (4, 2, 2, 4), 5.6, -0.331
    U = rand_links(dims, 303)
    G = synth.haar_su3(synth.rng(304), synth.volume(dims))
    Ug = _gauge_transform(dims, U, G)
    S0, S1 = orc.gauge_action(dims, beta, U, c1), orc.gauge_action(dims, beta, Ug, c1)
    assert abs(S1 - S0) < 1e-13 * abs(S0)
    alg = lambda p: np.einsum("...a,aij->...ij", p, T)
    F0, F1 = alg(orc.gauge_force(dims, beta, U, c1)), alg(orc.gauge_force(dims, beta, Ug, c1))
    assert np.max(np.abs(F1 - G @ F0 @ _dag(G))) < 1e-12


@pytest.mark.parametrize("dims", [L2, (4, 4, 2, 2)])
@pytest.mark.parametrize("c1", C1S)
def test_force_is_gradient_of_action(orc, dims, c1):
    beta, h = 6.0, 1e-5
    U = rand_links(dims, 305)
    F = orc.gauge_force(dims, beta, U, c1)
    V = synth.volume(dims)
    for (mu, i) in [(0, 0), (1, 3), (3, V - 1), (2, V // 2 + 1)]:
        fd = []
        for a in range(8):
            Up, Um = U.copy(), U.copy()
            Up[mu, i] = scipy.linalg.expm(h * T[a]) @ U[mu, i]
            Um[mu, i] = scipy.linalg.expm(-h * T[a]) @ U[mu, i]
            fd.append(-(orc.gauge_action(dims, beta, Up, c1) - orc.gauge_action(dims, beta, Um, c1)) / (2 * h))
        assert np.max(np.abs(np.array(fd) - F[mu, i])) < 1e-7 * max(1.0, np.max(np.abs(F[mu, i])))


@pytest.mark.parametrize("dims", [L2, (4, 2, 2, 4)])
@pytest.mark.parametrize("c1", C1S)
def test_force_tangent_finite_difference(orc, dims, c1):
    beta, h = 6.0, 1e-5
    U = rand_links(dims, 306)
    Vd = synth.rng(307).standard_normal((4, synth.volume(dims), 8))
    J = orc.gauge_force_tangent(dims, beta, U, Vd, c1)
    Fp = orc.gauge_force(dims, beta, orc.link_update(dims, h, Vd, U), c1)
    Fm = orc.gauge_force(dims, beta, orc.link_update(dims, -h, Vd, U), c1)
    assert np.max(np.abs((Fp - Fm) / (2 * h) - J)) < 1e-7 * np.max(np.abs(J))


def test_rectangle_part_changes_force_and_tangent(orc):
    """c1 enters: the force and tangent move by an amount of the size of the terms"""
    dims = L2
    U = rand_links(dims, 308)
    Vd = synth.rng(309).standard_normal((4, synth.volume(dims), 8))
    F0, F1 = orc.gauge_force(dims, 6.0, U), orc.gauge_force(dims, 6.0, U, -1 / 12)
    J0, J1 = orc.gauge_force_tangent(dims, 6.0, U, Vd), orc.gauge_force_tangent(dims, 6.0, U, Vd, -1 / 12)
    assert np.max(np.abs(F1 - F0)) > 0.1 * np.max(np.abs(F0))
    assert np.max(np.abs(J1 - J0)) > 0.1 * np.max(np.abs(J0))


@pytest.mark.parametrize("name", ["PQPQP", "FG"])
def test_reversibility(orc, name):
    U0, P0, eta, _ = synth.hot_start((4, 4, 2, 2), synth.SEED_BASE + 310, fermions=True)
    dims, c1 = (4, 4, 2, 2), -1 / 12
    phi = orc.pf_heatbath(dims, 0.155, U0, eta)
    args = dict(kappa=0.155, phi=phi, tol=1e-14, c1=c1)
    U1, P1, dH, _, status = orc.trajectory(dims, 5.6, table(name), 1.0, 5, U0, P0, **args)
    assert status == 0
    U2, P2, dH2, _, _ = orc.trajectory(dims, 5.6, table(name), 1.0, 5, U1, -P1, **args)
    assert np.max(np.abs(U2 - U0)) < 1e-11
    assert np.max(np.abs(-P2 - P0)) < 1e-11 * np.max(np.abs(P0))
    assert abs(dH + dH2) < 1e-9


@pytest.mark.parametrize("fg_exact", [False, True])
def test_fg_fourth_order(orc, fg_exact):
    U0, P0, _, _ = synth.hot_start(L4, synth.SEED_BASE + 311, fermions=False)
    dh = []
    for n in (16, 32):
        _, _, d, _, _ = orc.trajectory(L4, 2.5, table("FG"), 1.0, n, U0, P0, c1=-0.331, fg_exact=fg_exact)
        dh.append(abs(d))
    assert abs(np.log2(dh[0] / dh[1]) - 4) < 0.3, dh
