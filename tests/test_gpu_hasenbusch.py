"""GPU parity of the Hasenbusch (two-pseudofermion) terms and of the nested
force-gradient integrator against the CPU oracle (row a9)."""
import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
K, K2 = 0.155, 0.140


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def relmax(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def start(dims, seed):
    U, P, eta1, _ = synth.hot_start(dims, seed, fermions=True)
    eta2 = synth.gaussian_noise(synth.rng(seed + 1), dims)
    return U, P, eta1, eta2


@pytest.mark.parametrize("dims", [(4, 4, 2, 2), (6, 4, 4, 6)])
def test_heatbath_action_force(ctx, orc, dims):
    U, _, eta1, eta2 = start(dims, 11)
    act = Action(beta=5.6, kappa=K, kappa_hasen=K2, cg_tol=1e-14)
    phi2 = ctx.hasen_heatbath(dims, act, dev(U), dev(eta2))
    phi2o = orc.hasen_heatbath(dims, K, K2, U, eta2)
    assert relmax(phi2.cpu().numpy(), phi2o) < 1e-12
    S2 = ctx.hasen_action(dims, act, dev(U), phi2)
    e2 = np.vdot(eta2, eta2).real
    assert abs(S2 - e2) < 1e-11 * e2
    phi1 = orc.pf_heatbath(dims, K2, U, eta1)
    _, X2 = orc.hasen_action(dims, K, K2, U, phi2o)
    F2o = orc.hasen_force(dims, K, K2, U, phi2o, X2)
    X1, _, _ = orc.cg(dims, K2, U, phi1)
    F1o = orc.fermion_force(dims, K2, U, X1)
    FGo = orc.gauge_force(dims, 5.6, U)
    for terms, ref in [(fgi.TERM_HASEN, F2o), (fgi.TERM_FERMION, F1o), (fgi.TERM_GAUGE, FGo),
                       (7, F2o + F1o + FGo)]:
        F, st = ctx.force_terms(dims, act, dev(U), dev(phi1), dev(phi2o), terms)
        assert relmax(F.cpu().numpy(), ref) < 1e-12, terms


def levels_fg3():
    FG = [("P", 1 / 6, 0.0), ("Q", 0.5, 0.0), ("G", 2 / 3, 1 / 72), ("Q", 0.5, 0.0), ("P", 1 / 6, 0.0)]
    return [(FG, 4, 1), (FG, 2, 2), (FG, 1, 2)]


@pytest.mark.parametrize("dims", [(4, 4, 2, 2), (6, 4, 4, 6)])
def test_nested_hasenbusch_trajectory_fp64(ctx, orc, dims):
    U0, P0, eta1, eta2 = start(dims, 12)
    act = Action(beta=5.6, kappa=K, kappa_hasen=K2, cg_tol=1e-14)
    levels = levels_fg3()
    integ = fgi.integrator_from_levels(levels)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, integ, 1.0, 3, U, P, dev(eta1), dev(eta2))
    Uo, Po, dHo, sto, _ = orc.trajectory_nested(dims, 5.6, levels, 1.0, 3, U0, P0, kappa=K, kappa2=K2,
                                                eta1=eta1, eta2=eta2)
    assert st["solves"] == sto["solves"]
    assert relmax(U.cpu().numpy(), Uo) < 1e-12
    assert relmax(P.cpu().numpy(), Po) < 1e-12
    assert abs(dH - dHo) < 1e-9, (dH, dHo)


@pytest.mark.parametrize("prec", ["mp32", "mp16"])
def test_nested_hasenbusch_mixed_precision(ctx, orc, prec):
    dims = (8, 8, 8, 8)
    U0, P0, eta1, eta2 = start(dims, 13)
    act = Action(beta=5.6, kappa=K, kappa_hasen=K2, cg_tol=1e-10, prec=prec, link_recon=12)
    levels = levels_fg3()
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, fgi.integrator_from_levels(levels), 1.0, 2, U, P, dev(eta1), dev(eta2))
    Uo, Po, dHo, _, _ = orc.trajectory_nested(dims, 5.6, levels, 1.0, 2, U0, P0, kappa=K, kappa2=K2,
                                              eta1=eta1, eta2=eta2, tol=1e-12)
    assert relmax(U.cpu().numpy(), Uo) < 1e-7 and relmax(P.cpu().numpy(), Po) < 1e-7
    assert abs(dH - dHo) < 1e-6


def test_hasenbusch_requires_second_noise(ctx):
    dims = (4, 4, 2, 2)
    U0, P0, eta1, _ = start(dims, 14)
    act = Action(beta=5.6, kappa=K, kappa_hasen=K2)
    with pytest.raises(fgi.FgiError) as e:
        ctx.trajectory(dims, act, "FG", 1.0, 2, dev(U0), dev(P0), dev(eta1), None)
    assert e.value.code == fgi.FGI_EINVAL
