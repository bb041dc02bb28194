"""The fourth-order Poisson brackets of Table 1 on the lattice (oracle).

Table 1 gives the shadow Hamiltonians of the fourth-order integrators in
terms of {{S,T},{S,{S,T}}}, {{S,T},{T,{S,T}}}, {T,{T,{S,{S,T}}}} and
{T,{T,{T,{S,T}}}} (the two brackets starting {S,{S,..}} / {T,{S,{S,..}}}
vanish for T quadratic in p).  The oracle evaluates them from the exact force
gradient J_V[F] and central differences of it (oracle_brackets4).  Pins:

  - closed forms on the abelian torus: links exp(theta_3 T^3 + theta_8 T^8)
    with momenta along T^3, T^8 stay diagonal under both flows, the gauge
    action is a sum of (beta/3)(1 - cos(w.theta)) over plaquettes and colours,
    and the brackets are the flat-space expressions in its gradient, Hessian
    and third and fourth derivative tensors (2^4, where x + mu = x - mu, and
    4 x 2 x 2 x 4);
  - the same brackets from forces alone (no force gradient): second, third
    and nested central differences of |F|^2 and <p, F> along exp(tP) U and
    the S-hat flow, on a non-abelian 4^4 field;
  - Table 1 on the lattice: over one trajectory the exact force-gradient
    integrator's dH minus dt^4/155520 Delta(36 STSST + 72 STTST + 126 TTSST +
    54 TTTST), and Campostrini's dH plus its dt^4/34560 row, fall as dt^6
    (ratio 64 per halving of dt), on 4^4 pure gauge and on 4 x 4 x 2 x 2 with
    Nf = 2 Wilson fermions; the displacement form of the FG stage does not
    follow the exact form's row (its residual falls as dt^4).
"""
import numpy as np
import pytest

from paper_0910_2950_amd import synth

# diagonal phases of exp(theta_3 T^3 + theta_8 T^8), T^a = i lambda^a / 2
CART = np.array([[0.5, 0.5 / np.sqrt(3)], [-0.5, 0.5 / np.sqrt(3)], [0.0, -1.0 / np.sqrt(3)]])
KEYS = ("STSST", "STTST", "TTSST", "TTTST")


def torus_field(dims, seed):
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    th = rng.uniform(-np.pi, np.pi, (4, V, 2))
    pp = rng.normal(size=(4, V, 2))
    ph = np.einsum("kc,mvc->mvk", CART, th)
    U = np.zeros((4, V, 3, 3), complex)
    for k in range(3):
        U[:, :, k, k] = np.exp(1j * ph[:, :, k])
    P = np.zeros((4, V, 8))
    P[:, :, 2], P[:, :, 7] = pp[:, :, 0], pp[:, :, 1]
    return th, pp, U, P


def torus_brackets(dims, beta, th, pp):
    """Closed forms: S = sum (beta/3)(1 - cos(w.theta)), w the plaquette's
    signed link incidence times the colour's Cartan weights; g = grad S,
    H, K, L its derivative tensors (rank one per term)."""
    X, Y, Z, T = dims
    V = X * Y * Z * T
    rows = []
    for t in range(T):
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    s = [x, y, z, t]
                    i = x + X * (y + Y * (z + Z * t))
                    for mu in range(4):
                        for nu in range(mu + 1, 4):
                            a, b = list(s), list(s)
                            a[mu] = (a[mu] + 1) % dims[mu]
                            b[nu] = (b[nu] + 1) % dims[nu]
                            ia = a[0] + X * (a[1] + Y * (a[2] + Z * a[3]))
                            ib = b[0] + X * (b[1] + Y * (b[2] + Z * b[3]))
                            for k in range(3):
                                w = np.zeros((4, V, 2))
                                w[mu, i] += CART[k]
                                w[nu, ia] += CART[k]
                                w[mu, ib] -= CART[k]
                                w[nu, i] -= CART[k]
                                rows.append(w.ravel())
    W = np.array(rows)
    q, p = th.ravel(), pp.ravel()
    a, c = W @ q, beta / 3.0
    g = (c * np.sin(a)) @ W
    wp, wg = W @ p, W @ g
    Hp = (c * np.cos(a) * wp) @ W
    Kgpp = np.sum(-c * np.sin(a) * wg * wp ** 2)
    return dict(SST=g @ g, TST=-p @ Hp, STSST=-2 * np.sum(c * np.cos(a) * wg ** 2),
                STTST=-2 * Hp @ Hp + Kgpp, TTSST=2 * Kgpp + 2 * Hp @ Hp,
                TTTST=np.sum(c * np.cos(a) * wp ** 4))


@pytest.mark.parametrize("dims,beta,seed", [((2, 2, 2, 2), 6.0, 1), ((4, 2, 2, 4), 5.6, 2)])
def test_brackets4_abelian_closed_forms(orc, dims, beta, seed):
    th, pp, U, P = torus_field(dims, seed)
    ref = torus_brackets(dims, beta, th, pp)
    b = orc.brackets4(dims, beta, U, P, h=1e-4)
    for k in ("SST", "TST", "STSST"):
        assert abs(b[k] - ref[k]) < 1e-12 * abs(ref[k]), k
    for k in ("STTST", "TTSST", "TTTST"):   # central differences at h = 1e-4
        assert abs(b[k] - ref[k]) < 2e-7 * abs(ref[k]), k


def test_brackets4_from_forces_alone(orc):
    """Force-only differences: TTSST = d^2/dt^2 |F|^2 and TTTST = d^3/dt^3
    <p, F> along exp(tP) U, STSST = d/dt |F|^2 along exp(tF) U, and STTST =
    [L_S, L_T] TST with TST = d/dt <p, F(exp(tP) U)> and L_S moving p by s F."""
    dims, beta = (4, 4, 4, 4), 6.0
    U0, P0, _, _ = synth.hot_start(dims, synth.SEED_BASE + 41, fermions=False)

    def F(U):
        return orc.force(dims, beta, U)[0]

    def moved(U, t, V):
        return orc.link_update(dims, t, V, U)

    b = orc.brackets4(dims, beta, U0, P0, h=1e-4)
    h = 2e-3
    n2 = [np.sum(F(moved(U0, k * h, P0)) ** 2) for k in (-2, -1, 0, 1, 2)]
    ttsst = (-n2[0] + 16 * n2[1] - 30 * n2[2] + 16 * n2[3] - n2[4]) / (12 * h * h)
    pf = [np.sum(P0 * F(moved(U0, k * h, P0))) for k in (-2, -1, 1, 2)]
    tttst = (pf[3] - 2 * pf[2] + 2 * pf[1] - pf[0]) / (2 * h ** 3)
    F0 = F(U0)
    fs = [np.sum(F(moved(U0, k * h, F0)) ** 2) for k in (-1, 1)]
    stsst = (fs[1] - fs[0]) / (2 * h)

    def tst(U, P):   # d/dt <P, F(exp(tP) U)>
        return (np.sum(P * F(moved(U, h, P))) - np.sum(P * F(moved(U, -h, P)))) / (2 * h)

    def ls_tst(U, P):   # L_S TST at (U, P): P -> P + s F(U)
        FU = F(U)
        return (tst(U, P + h * FU) - tst(U, P - h * FU)) / (2 * h)
    lslt = (ls_tst(moved(U0, h, P0), P0) - ls_tst(moved(U0, -h, P0), P0)) / (2 * h)   # L_T L_S TST
    F0 = F(U0)

    def lt_tst(P):   # L_T TST at (U0, P)
        return (tst(moved(U0, h, P), P) - tst(moved(U0, -h, P), P)) / (2 * h)
    ltls = (lt_tst(P0 + h * F0) - lt_tst(P0 - h * F0)) / (2 * h)                       # L_S L_T TST
    sttst = ltls - lslt
    assert abs(stsst - b["STSST"]) < 1e-4 * abs(b["STSST"])
    assert abs(ttsst - b["TTSST"]) < 1e-4 * abs(b["TTSST"])
    assert abs(tttst - b["TTTST"]) < 1e-3 * abs(b["TTTST"])
    assert abs(sttst - b["STTST"]) < 1e-3 * abs(b["STTST"])


def fg_row(b):
    return (36 * b["STSST"] + 72 * b["STTST"] + 126 * b["TTSST"] + 54 * b["TTTST"]) / 155520


def campostrini_row(b):
    c2, c4 = 2 ** (1 / 3), 4 ** (1 / 3)
    return -((180 * c4 + 240 * c2 + 312) * b["STSST"] + (60 * c4 + 80 * c2 + 104) * b["STTST"]
             + (20 * c2 + 32) * b["TTSST"] + (5 * c2 + 8) * b["TTTST"]) / 34560


def residuals(orc, dims, beta, U0, P0, name, row, exact, kappa=0.0, phi=None, ns=(8, 16, 32, 64)):
    kw = dict(kappa=kappa, phi=phi) if phi is not None else {}
    b0 = orc.brackets4(dims, beta, U0, P0, h=1e-3, **kw)
    out = []
    for n in ns:
        U1, P1, dH, _, status = orc.trajectory(dims, beta, orc.table(name), 1.0, n, U0, P0, fg_exact=exact, **kw)
        assert status == 0
        b1 = orc.brackets4(dims, beta, U1, P1, h=1e-3, **kw)
        out.append((dH, dH - (1.0 / n) ** 4 * (row(b1) - row(b0))))
    return out


CASES = [("gauge", (4, 4, 4, 4), 6.0, 0.0), ("nf2", (4, 4, 2, 2), 5.6, 0.155)]


@pytest.mark.parametrize("case,dims,beta,kappa", CASES)
@pytest.mark.parametrize("name,row", [("FG", fg_row), ("CAMPOSTRINI", campostrini_row)])
def test_table1_dt4_rows_on_the_lattice(orc, case, dims, beta, kappa, name, row):
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + (0 if case == "gauge" else 3), fermions=kappa != 0)
    phi = orc.pf_heatbath(dims, kappa, U0, eta) if kappa else None
    res = residuals(orc, dims, beta, U0, P0, name, row, True, kappa, phi)
    ratios = [abs(res[i][1] / res[i + 1][1]) for i in range(len(res) - 1)]
    assert all(48 < r < 80 for r in ratios), ratios
    # the prediction carries dH: the residual is a small part of it at the finest step
    assert abs(res[-1][1]) < 0.02 * abs(res[-1][0])


def test_displacement_form_has_another_dt4_coefficient(orc):
    """The FG stage in its displacement form agrees with the exact stage to
    O(dt^5) per step, so dH still falls as dt^4, but with another coefficient:
    the exact form's dt^4 row leaves a residual that falls as dt^4 too."""
    dims, beta = (4, 4, 4, 4), 6.0
    U0, P0, _, _ = synth.hot_start(dims, synth.SEED_BASE, fermions=False)
    res = residuals(orc, dims, beta, U0, P0, "FG", fg_row, False, ns=(16, 32, 64))
    ratios = [abs(res[i][1] / res[i + 1][1]) for i in range(len(res) - 1)]
    assert all(12 < r < 20 for r in ratios), ratios
    assert abs(res[-1][1]) > 0.1 * abs(res[-1][0])
