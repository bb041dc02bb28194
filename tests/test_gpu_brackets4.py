"""The dt^4 Poisson brackets of Table 1 on the GPU (fgi_poisson_brackets4)
against the oracle's (oracle_brackets4, pinned in test_oracle_brackets4.py),
at the same difference step: pure gauge (Wilson and tree-level Symanzik) and
Nf = 2 Wilson fermions, including a lattice with a ragged block tail; and on
the GPU alone, exact force-gradient trajectories whose dH minus Table 1's dt^4
row falls as dt^6."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
EXACT = ("SST", "TST", "STSST")      # products of force gradients at U
DIFF = ("STTST", "TTSST", "TTTST")   # carry one central difference of J_P


@pytest.fixture(scope="module")
def ctx():
    c = fgi.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


CASES = [((4, 4, 4, 4), 6.0, 0.0, 0.0), ((4, 4, 4, 4), 6.0, 0.0, -1.0 / 12.0), ((4, 4, 2, 2), 5.6, 0.155, 0.0),
         ((6, 4, 4, 6), 5.6, 0.155, 0.0)]


@pytest.mark.parametrize("dims,beta,kappa,c1", CASES)
def test_brackets4_match_oracle(ctx, orc, dims, beta, kappa, c1):
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 61, fermions=kappa != 0)
    phi = orc.pf_heatbath(dims, kappa, U0, eta) if kappa else None
    act = Action(beta=beta, kappa=kappa, c1=c1, cg_tol=1e-14)
    g = ctx.poisson_brackets4(dims, act, dev(U0), dev(P0), dev(phi) if kappa else None, h=1e-3)
    o = orc.brackets4(dims, beta, U0, P0, kappa=kappa, phi=phi, h=1e-3, c1=c1)
    print(dims, kappa, c1, {k: "%.10e / %.10e" % (g[k], o[k]) for k in g}, flush=True)
    for k in EXACT:
        assert abs(g[k] - o[k]) < 1e-11 * abs(o[k]), k
    for k in DIFF:
        assert abs(g[k] - o[k]) < 1e-7 * abs(o[k]), k


def fg_row(b):
    return (36 * b["STSST"] + 72 * b["STTST"] + 126 * b["TTSST"] + 54 * b["TTTST"]) / 155520


@pytest.mark.parametrize("dims,beta,kappa", [((4, 4, 4, 4), 6.0, 0.0), ((4, 4, 2, 2), 5.6, 0.155)])
def test_fg_dt4_row_on_gpu(ctx, orc, dims, beta, kappa):
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 62, fermions=kappa != 0)
    phi = dev(orc.pf_heatbath(dims, kappa, U0, eta)) if kappa else None
    act = dataclasses.replace(Action(beta=beta, kappa=kappa, cg_tol=1e-14), fg_exact=True)
    b0 = ctx.poisson_brackets4(dims, act, dev(U0), dev(P0), phi, h=1e-3)
    res = []
    for n in (8, 16, 32, 64):
        U, P = dev(U0), dev(P0)
        if kappa:
            dH, _ = ctx.trajectory(dims, act, "FG", 1.0, n, U, P, phi, pf_is_phi=True)
        else:
            dH, _ = ctx.trajectory(dims, act, "FG", 1.0, n, U, P)
        b1 = ctx.poisson_brackets4(dims, act, U, P, phi, h=1e-3)
        res.append(dH - (1.0 / n) ** 4 * (fg_row(b1) - fg_row(b0)))
    ratios = [abs(res[i] / res[i + 1]) for i in range(3)]
    print(dims, "residuals", res, "ratios", ratios, flush=True)
    assert all(48 < r < 80 for r in ratios), ratios


@pytest.mark.parametrize("dims,beta,kappa", [((4, 4, 4, 4), 6.0, 0.0), ((4, 4, 2, 2), 5.6, 0.155)])
def test_fg_family_member_on_gpu(ctx, orc, dims, beta, kappa):
    """A member P(lam) Q G(1 - 2 lam, xi) Q P(lam) of the tunable force-gradient
    family away from the fourth-order point, with the exact G stage: one
    trajectory matches the oracle's, and dH minus the family's predicted dt^2
    and dt^4 terms (tuning.predicted_dh_fg_family, from the GPU brackets at both
    ends) falls as dt^6."""
    from paper_0910_2950_amd import tuning
    lam, xi = 0.19, 0.008
    stages = tuning.fg_family_stages(lam, xi)
    terms = fgi.TERM_GAUGE | (fgi.TERM_FERMION if kappa else 0)
    integ = fgi.integrator_from_levels([(stages, terms, 1)])
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 63, fermions=kappa != 0)
    phi0 = orc.pf_heatbath(dims, kappa, U0, eta) if kappa else None
    phi = dev(phi0) if kappa else None
    act = dataclasses.replace(Action(beta=beta, kappa=kappa, cg_tol=1e-14), fg_exact=True)
    kw = dict(kappa=kappa, phi=phi0) if kappa else {}
    b0 = ctx.poisson_brackets4(dims, act, dev(U0), dev(P0), phi, h=1e-3)
    res = []
    for n in (8, 16, 32, 64):
        U, P = dev(U0), dev(P0)
        extra = (phi,) if kappa else ()
        dH, _ = ctx.trajectory(dims, act, integ, 1.0, n, U, P, *extra, pf_is_phi=bool(kappa))
        if n == 8:
            Uo, Po, dHo, _, status = orc.trajectory(dims, beta, stages, 1.0, n, U0, P0, fg_exact=True, **kw)
            assert status == 0
            print(dims, "dH gpu %.12e oracle %.12e" % (dH, dHo), flush=True)
            assert abs(dH - dHo) < 1e-9 * max(1.0, abs(dHo))
            assert np.max(np.abs(U.cpu().numpy() - Uo)) < 1e-11
            assert np.max(np.abs(P.cpu().numpy() - Po)) < 1e-10
        b1 = ctx.poisson_brackets4(dims, act, U, P, phi, h=1e-3)
        dB = {k: b1[k] - b0[k] for k in tuning.FG_KEYS2 + tuning.FG_KEYS4}
        res.append(dH - float(tuning.predicted_dh_fg_family(lam, xi, dB, 1.0 / n)))
    ratios = [abs(res[i] / res[i + 1]) for i in range(3)]
    print(dims, "family residuals", res, "ratios", ratios, flush=True)
    assert all(48 < r < 80 for r in ratios), ratios
