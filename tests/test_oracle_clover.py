"""Pins of the oracle's clover (Sheikholeslami-Wohlert) fermion operator (no GPU).

The paper's conclusions state that the force-gradient construction applies to
the usual improved actions; the clover term is the standard O(a) improvement
of the Wilson operator, in the hopping normalisation

    M = A - kappa D,  A(x) = 1 + i kappa csw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),
    sigma_{mu nu} = (i/2)[g_mu, g_nu],  Fhat = (Q - Q^+)/8,  Q the four-leaf clover,

with the two-flavour action phi^+ (Mhat^+ Mhat)^-1 phi - 2 sum_{x odd} log det A(x)
and Mhat = A_ee - kappa^2 D_eo A_oo^-1 D_oe.  Checks:

  - sigma: Hermitian, i g_mu g_nu for mu != nu, squares to one, commutes with
    g5 = g1 g2 g3 g4 = diag(1, 1, -1, -1) (the basis in which A is
    block-diagonal and Mhat^+ = g5 Mhat g5);
  - A(x) against a numpy construction from shifted link arrays and Kronecker
    products (a different enumeration of the leaves), its inverse and log det
    against numpy's;
  - a closed form: a constant abelian flux through one plane (every leaf the
    same diagonal plaquette), det A(x) = (1 - kappa^2 csw^2 sin^2 f)^4, also
    after a random gauge rotation;
  - csw = 0 is the Wilson operator, bit for bit;
  - the even-odd algebra against dense linear algebra: Mhat equals the Schur
    complement M_ee - M_eo M_oo^-1 M_oe of the dense full-lattice M, and
    log|det M| = sum_{x odd} log det A(x) + log|det Mhat|;
  - gauge invariance of both action terms;
  - the forces (log det alone, pseudofermion alone, total with the gauge
    force) as finite-difference gradients of the actions;
  - trajectories: reversibility and the dt^4 scaling of dH for FG, and the
    exact G stage refused (it would need the clover force's tangent).
"""
import numpy as np
import pytest
import scipy.linalg

from paper_0910_2950_amd import synth
from oracle.oracle import table

T = 0.5j * synth.gell_mann()
K, CSW = 0.155, 1.0   # kappa csw < 1/6 keeps A(x) positive for any links


def rand_links(dims, seed):
    return synth.haar_su3(synth.rng(seed), 4 * synth.volume(dims)).reshape(4, -1, 3, 3)


def _grid(dims, U):
    Lx, Ly, Lz, Lt = dims
    return U.reshape(4, Lt, Lz, Ly, Lx, 3, 3)


def _at(A, mu, k):
    return np.roll(A, -k, axis=3 - mu)


def _dag(A):
    return np.conj(np.swapaxes(A, -1, -2))


def _gauge_transform(dims, U, G):
    V = synth.volume(dims)
    c = np.stack(np.unravel_index(np.arange(V), dims[::-1])[::-1], axis=1)
    out = np.empty_like(U)
    for mu in range(4):
        cp = c.copy()
        cp[:, mu] = (cp[:, mu] + 1) % dims[mu]
        ip = cp[:, 0] + dims[0] * (cp[:, 1] + dims[1] * (cp[:, 2] + dims[2] * cp[:, 3]))
        out[mu] = G @ U[mu] @ _dag(G[ip])
    return out


def parity(dims):
    V = synth.volume(dims)
    c = np.stack(np.unravel_index(np.arange(V), dims[::-1])[::-1], axis=1)
    return c.sum(axis=1) % 2


def gammas(orc):
    g = []
    for mu in range(4):
        out = np.zeros((4, 4), np.complex128)
        orc.lib().oracle_gamma(mu, out.ctypes.data)
        g.append(out)
    return g


def brute_clover(dims, U, kappa, csw, orc):
    """A(x) from np.roll-shifted link arrays and np.kron, [V, 12, 12]"""
    G = _grid(dims, U)
    g = gammas(orc)
    V = synth.volume(dims)
    A = np.tile(np.eye(12, dtype=np.complex128), (V, 1, 1))
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Um, Un = G[mu], G[nu]
            l1 = Um @ _at(Un, mu, 1) @ _dag(_at(Um, nu, 1)) @ _dag(Un)
            l2 = Un @ _dag(_at(_at(Um, mu, -1), nu, 1)) @ _dag(_at(Un, mu, -1)) @ _at(Um, mu, -1)
            l3 = (_dag(_at(Um, mu, -1)) @ _dag(_at(_at(Un, mu, -1), nu, -1)) @ _at(_at(Um, mu, -1), nu, -1)
                  @ _at(Un, nu, -1))
            l4 = _dag(_at(Un, nu, -1)) @ _at(Um, nu, -1) @ _at(_at(Un, nu, -1), mu, 1) @ _dag(Um)
            Q = (l1 + l2 + l3 + l4).reshape(V, 3, 3)
            Fh = (Q - _dag(Q)) / 8
            sig = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
            A += 1j * kappa * csw * np.einsum("st,xab->xsatb", sig, Fh).reshape(V, 12, 12)
    return A


def test_sigma(orc):
    g = gammas(orc)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=1e-15)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            s = orc.sigma(mu, nu)
            assert np.allclose(s, 1j * g[mu] @ g[nu], atol=1e-15)
            assert np.allclose(s, s.conj().T, atol=1e-15)
            assert np.allclose(s @ s, np.eye(4), atol=1e-15)
            assert np.allclose(s @ g5, g5 @ s, atol=1e-15)
            assert np.allclose(orc.sigma(nu, mu), -s, atol=1e-15)


@pytest.mark.parametrize("dims", [(4, 2, 2, 4), (2, 2, 2, 2), (4, 4, 2, 2)])
def test_clover_matches_brute_force(orc, dims):
    U = rand_links(dims, 601)
    A, Ai, ld, sdet = orc.clover(dims, K, CSW, U)
    Ab = brute_clover(dims, U, K, CSW, orc)
    assert np.max(np.abs(A - Ab)) < 1e-14
    assert np.max(np.abs(A - _dag(A))) < 1e-15
    g5 = np.kron(np.diag([1, 1, -1, -1]), np.eye(3))
    assert np.max(np.abs(A @ g5 - g5 @ A)) < 1e-15
    assert np.max(np.abs(A @ Ai - np.eye(12))) < 1e-13
    sign, ref = np.linalg.slogdet(Ab)
    assert np.all(np.abs(sign - 1) < 1e-12)
    assert np.max(np.abs(ld - ref)) < 1e-12
    assert abs(sdet - (-2.0 * ref[parity(dims) == 1].sum())) < 1e-11
    assert np.min(np.linalg.eigvalsh(Ab)) > 0


def test_constant_flux_closed_form(orc):
    dims = (8, 4, 2, 4)
    V = synth.volume(dims)
    f = 2 * np.pi * 3 / dims[0]
    U = synth.unit_links(dims)
    x = np.arange(V) % dims[0]
    U[1, :, 0, 0] = np.exp(1j * f * x)
    U[1, :, 1, 1] = np.exp(-1j * f * x)
    ref = 4 * np.log(1 - (K * CSW * np.sin(f)) ** 2)
    Ug = _gauge_transform(dims, U, synth.haar_su3(synth.rng(602), V))
    for W in (U, Ug):
        _, _, ld, sdet = orc.clover(dims, K, CSW, W)
        assert np.max(np.abs(ld - ref)) < 1e-13
        assert abs(sdet - (-2 * ref * V / 2)) < 1e-11


def test_zero_csw_is_wilson(orc):
    dims = (4, 4, 2, 2)
    U, P, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 603)
    A, Ai, ld, sdet = orc.clover(dims, K, 0.0, U)
    assert np.array_equal(A, np.tile(np.eye(12), (synth.volume(dims), 1, 1)))
    assert sdet == 0.0
    assert np.array_equal(orc.clover_mhat(dims, K, 0.0, U, eta), orc.mhat(dims, K, U, eta))
    phi = orc.pf_heatbath(dims, K, U, eta)
    F0, _ = orc.force(dims, 5.6, U, kappa=K, phi=phi)
    F1, _ = orc.force(dims, 5.6, U, kappa=K, phi=phi, csw=0.0)
    assert np.array_equal(F0, F1)


def _dense(fn, n):
    cols = []
    for j in range(n):
        e = np.zeros(n, np.complex128)
        e[j] = 1
        cols.append(fn(e))
    return np.stack(cols, axis=1)


def test_even_odd_schur_complement_dense(orc):
    dims = (2, 2, 2, 4)
    V = synth.volume(dims)
    U = rand_links(dims, 604)
    M = _dense(lambda e: orc.clover_wilson(dims, K, CSW, U, e.reshape(V, 12)).ravel(), 12 * V)
    par = np.repeat(parity(dims), 12)
    ev, od = np.where(par == 0)[0], np.where(par == 1)[0]
    Mee, Meo, Moe, Moo = M[np.ix_(ev, ev)], M[np.ix_(ev, od)], M[np.ix_(od, ev)], M[np.ix_(od, od)]
    schur = Mee - Meo @ np.linalg.solve(Moo, Moe)
    Vh = V // 2
    Mh = _dense(lambda e: orc.clover_mhat(dims, K, CSW, U, e.reshape(Vh, 12)).ravel(), 12 * Vh)
    assert np.max(np.abs(Mh - schur)) < 1e-13
    Mhd = _dense(lambda e: orc.clover_mhat(dims, K, CSW, U, e.reshape(Vh, 12), dagger=True).ravel(), 12 * Vh)
    assert np.max(np.abs(Mhd - Mh.conj().T)) < 1e-14
    _, _, ld, sdet = orc.clover(dims, K, CSW, U)
    s_full = np.linalg.slogdet(M)[1]
    s_hat = np.linalg.slogdet(Mh)[1]
    assert abs(s_full - (ld[parity(dims) == 1].sum() + s_hat)) < 1e-10


def test_gauge_invariance(orc):
    dims = (4, 2, 2, 4)
    V = synth.volume(dims)
    U, _, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 605)
    G = synth.haar_su3(synth.rng(606), V)
    Ug = _gauge_transform(dims, U, G)
    phi = orc.clover_mhat(dims, K, CSW, U, eta, dagger=True)
    Ge = G[parity(dims) == 0]
    phig = np.einsum("xab,xsb->xsa", Ge, phi.reshape(-1, 4, 3)).reshape(phi.shape)
    s0, s1 = orc.clover(dims, K, CSW, U)[3], orc.clover(dims, K, CSW, Ug)[3]
    assert abs(s1 - s0) < 1e-12 * abs(s0)
    f0, f1 = orc.clover_pf_action(dims, K, CSW, U, phi)[0], orc.clover_pf_action(dims, K, CSW, Ug, phig)[0]
    assert abs(f1 - f0) < 1e-11 * abs(f0)


def _fd(dims, U, fn, links, h=1e-5):
    out = []
    for (mu, i) in links:
        row = []
        for a in range(8):
            Up, Um = U.copy(), U.copy()
            Up[mu, i] = scipy.linalg.expm(h * T[a]) @ U[mu, i]
            Um[mu, i] = scipy.linalg.expm(-h * T[a]) @ U[mu, i]
            row.append(-(fn(Up) - fn(Um)) / (2 * h))
        out.append(row)
    return np.array(out)


@pytest.mark.parametrize("dims", [(4, 2, 2, 4), (2, 2, 2, 2)])
def test_log_det_force_is_gradient(orc, dims):
    U = rand_links(dims, 607)
    V = synth.volume(dims)
    links = [(0, 0), (1, 3), (3, V - 1), (2, V // 2 + 1)]
    F = orc.clover_force(dims, K, CSW, U, None, det_scale=1.0)
    fd = _fd(dims, U, lambda W: orc.clover(dims, K, CSW, W)[3], links)
    ref = np.array([F[mu, i] for (mu, i) in links])
    assert np.max(np.abs(fd - ref)) < 1e-8 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(ref)) > 1e-3


@pytest.mark.parametrize("dims", [(4, 2, 2, 4), (2, 2, 2, 2)])
def test_pf_force_is_gradient(orc, dims):
    U, _, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 608)
    V = synth.volume(dims)
    phi = orc.clover_mhat(dims, K, CSW, U, eta, dagger=True)
    X, it = orc.clover_cg(dims, K, CSW, U, phi)
    assert it > 0
    links = [(0, 1), (1, 2), (3, V - 2), (2, V // 2)]
    F = orc.clover_force(dims, K, CSW, U, X, pf_scale=1.0, det_scale=0.0)
    fd = _fd(dims, U, lambda W: orc.clover_pf_action(dims, K, CSW, W, phi)[0], links)
    ref = np.array([F[mu, i] for (mu, i) in links])
    assert np.max(np.abs(fd - ref)) < 1e-7 * np.max(np.abs(ref))
    # the clover part matters: the Wilson-form force at the same X is far off
    Fw = orc.clover_force(dims, K, 0.0, U, X, pf_scale=1.0, det_scale=0.0)
    assert np.max(np.abs(Fw - F)) > 1e-2 * np.max(np.abs(F))


def test_total_force_is_gradient(orc):
    dims = (4, 2, 2, 4)
    U, _, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 609)
    V = synth.volume(dims)
    phi = orc.clover_mhat(dims, K, CSW, U, eta, dagger=True)
    F, st = orc.force(dims, 5.6, U, kappa=K, phi=phi, csw=CSW)
    assert st["solves"] == 1
    links = [(0, 5), (2, 9), (3, V - 3)]
    S = lambda W: (orc.gauge_action(dims, 5.6, W) + orc.clover_pf_action(dims, K, CSW, W, phi)[0]
                   + orc.clover(dims, K, CSW, W)[3])
    fd = _fd(dims, U, S, links)
    ref = np.array([F[mu, i] for (mu, i) in links])
    assert np.max(np.abs(fd - ref)) < 1e-7 * np.max(np.abs(ref))


@pytest.mark.parametrize("name", ["PQPQP", "FG"])
def test_reversibility(orc, name):
    dims = (4, 4, 2, 2)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 610)
    phi = orc.clover_mhat(dims, K, CSW, U0, eta, dagger=True)
    args = dict(kappa=K, phi=phi, tol=1e-14, csw=CSW)
    U1, P1, dH, _, status = orc.trajectory(dims, 5.6, table(name), 1.0, 4, U0, P0, **args)
    assert status == 0
    U2, P2, dH2, _, _ = orc.trajectory(dims, 5.6, table(name), 1.0, 4, U1, -P1, **args)
    assert np.max(np.abs(U2 - U0)) < 1e-11
    assert np.max(np.abs(-P2 - P0)) < 1e-11 * np.max(np.abs(P0))
    assert abs(dH + dH2) < 1e-9


def test_fg_fourth_order_and_heatbath(orc):
    dims = (4, 4, 2, 2)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 611)
    dh = []
    for n in (8, 16):
        _, _, d, st, status = orc.trajectory(dims, 5.6, table("FG"), 1.0, n, U0, P0, kappa=K, eta=eta, csw=CSW)
        assert status == 0
        dh.append(d)
    assert abs(np.log2(abs(dh[0] / dh[1])) - 4) < 0.3, dh
    # with eta the start's S_F is eta^+ eta: the same trajectory from phi = Mhat^+ eta agrees
    phi = orc.clover_mhat(dims, K, CSW, U0, eta, dagger=True)
    _, _, d2, _, _ = orc.trajectory(dims, 5.6, table("FG"), 1.0, 16, U0, P0, kappa=K, phi=phi, csw=CSW)
    assert abs(d2 - dh[1]) < 1e-9


def test_exact_form_refused(orc):
    dims = (4, 4, 2, 2)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 612)
    *_, status = orc.trajectory(dims, 5.6, table("FG"), 1.0, 2, U0, P0, kappa=K, eta=eta, csw=CSW, fg_exact=True)
    assert status == -2


def test_nested_driver_with_clover(orc):
    """the nested driver with the clover term: one level with every term is
    the single-level trajectory; two scales (S_F + log det outside, S_G
    inside) are reversible and fourth order in FG"""
    dims = (4, 4, 2, 2)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 613)
    a = orc.trajectory(dims, 5.6, table("FG"), 1.0, 4, U0, P0, kappa=K, eta=eta, csw=CSW)
    b = orc.trajectory_nested(dims, 5.6, [(table("FG"), 3, 1)], 1.0, 4, U0, P0, kappa=K, eta1=eta, csw=CSW)
    assert b[4] == 0 and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert abs(a[2] - b[2]) < 1e-10 and a[3]["solves"] == b[3]["solves"]
    levels = [(table("FG"), 2, 1), (table("FG"), 1, 2)]
    dh = []
    for n in (12, 24):   # (at 6 and 12 the ratio is still pre-asymptotic: slope 5.2)
        U1, P1, d, _, status = orc.trajectory_nested(dims, 5.6, levels, 1.0, n, U0, P0, kappa=K, eta1=eta, csw=CSW)
        assert status == 0
        dh.append(d)
    assert abs(np.log2(abs(dh[0] / dh[1])) - 4) < 0.5, dh
    # refused: the exact form with the clover term
    assert orc.trajectory_nested(dims, 5.6, levels, 1.0, 2, U0, P0, kappa=K, eta1=eta, csw=CSW,
                                 fg_exact=True)[4] == -2


def test_brackets_with_clover(orc):
    """SST is the squared total force, with the clover and log det parts"""
    dims = (4, 2, 2, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 614)
    phi = orc.clover_mhat(dims, K, CSW, U0, eta, dagger=True)
    F, _ = orc.force(dims, 5.6, U0, kappa=K, phi=phi, csw=CSW)
    sst, tst = orc.brackets(dims, 5.6, U0, P0, kappa=K, phi=phi, csw=CSW)
    assert abs(sst - np.sum(F * F)) < 1e-10 * sst
    sst0, _ = orc.brackets(dims, 5.6, U0, P0, kappa=K, phi=phi)
    assert abs(sst - sst0) > 1e-3 * sst


def test_hasenbusch_with_clover(orc):
    """the Hasenbusch split of the clover determinant, det M = det A_oo(kappa)
    det Mhat2 det(Mhat2^-1 Mhat), on three scales (S_2 outside, S_1 and the log
    det in the middle, S_G inside): at tau = 0 the heatbath energies return
    exactly (S_1 = |eta1|^2, S_2 = |eta2|^2 to the solver tolerance), dH falls
    at fourth order in FG and the trajectory reverses"""
    dims = (4, 4, 2, 2)
    U0, P0, eta1, _ = synth.hot_start(dims, synth.SEED_BASE + 615)
    eta2 = synth.gaussian_noise(synth.rng(synth.SEED_BASE + 616), dims)
    K2 = 0.13
    levels = [(table("FG"), 4, 1), (table("FG"), 2, 2), (table("FG"), 1, 2)]
    args = dict(kappa=K, kappa2=K2, eta1=eta1, eta2=eta2, csw=CSW)
    _, _, d0, _, status = orc.trajectory_nested(dims, 5.6, levels, 0.0, 1, U0, P0, **args)
    assert status == 0 and abs(d0) < 1e-10
    dh = []
    for n in (8, 16):
        U1, P1, d, st, status = orc.trajectory_nested(dims, 5.6, levels, 1.0, n, U0, P0, **args)
        assert status == 0
        dh.append(d)
    assert abs(np.log2(abs(dh[0] / dh[1])) - 4) < 0.5, dh
    # without the split the same field and noise give another dH (the split changes the action terms' noise)
    _, _, dnh, _, _ = orc.trajectory_nested(dims, 5.6, [(table("FG"), 3, 1)], 1.0, 16, U0, P0, kappa=K, eta1=eta1,
                                            csw=CSW)
    assert abs(dnh - dh[1]) > 1e-6
