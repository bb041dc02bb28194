"""A looser tolerance for the solves inside force evaluations (cg_tol_md)
while the heatbath and action solves that enter dH keep cg_tol.

  - the trajectory moves by no more than the MD solver error from the one at
    full tolerance (oracle, FP64 at 1e-14);
  - dH stays exact: the oracle rebuilds it from the GPU's start and end fields
    (gauge and kinetic energy, a fresh 1e-14 solve for S_F at the end) and it
    agrees to the action solves' tolerance, far below the MD tolerance's
    effect on S_F;
  - the MD map reverses to the MD tolerance (every solve starts from zero or
    from a solution at the same links; a solve stopping at a looser threshold
    reacts to last-bit differences of the links by up to that threshold), and
    it takes fewer CG iterations;
  - invalid values are rejected.
"""
import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
K = 0.155


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.cpu().numpy()


def relmax(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("prec", ["fp64", "mp16"])
def test_md_tolerance_keeps_dH_exact(ctx, orc, prec):
    dims = (6, 4, 4, 6)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 700, fermions=True)
    recon = 12 if prec == "mp16" else 18
    full = Action(beta=5.6, kappa=K, cg_tol=1e-12, prec=prec, link_recon=recon)
    loose = Action(beta=5.6, kappa=K, cg_tol=1e-12, prec=prec, link_recon=recon, cg_tol_md=1e-6)
    Ua, Pa, Ub, Pb = dev(U0), dev(P0), dev(U0), dev(P0)
    dHa, sta = ctx.trajectory(dims, full, "FG", 1.0, 4, Ua, Pa, dev(eta))
    dHb, stb = ctx.trajectory(dims, loose, "FG", 1.0, 4, Ub, Pb, dev(eta))
    assert stb["cg_iters"] < 0.8 * sta["cg_iters"], (sta["cg_iters"], stb["cg_iters"])
    Uo, Po, dHo, _, _ = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 4, U0, P0, kappa=K, eta=eta)
    # the MD solver error moves the trajectory by about its size
    assert relmax(host(Ub), Uo) < 1e-4 and relmax(host(Pb), Po) < 1e-4
    assert relmax(host(Ub), Uo) > 1e-9       # and it does move it
    # dH of the loose trajectory rebuilt from its own end fields at full precision
    U1, P1 = host(Ub), host(Pb)
    phi = orc.pf_heatbath(dims, K, U0, eta)
    sf1, _ = orc.pf_action(dims, K, U1, phi, tol=1e-14)
    dH_rebuilt = (orc.gauge_action(dims, 5.6, U1) + orc.kinetic(dims, P1) - orc.gauge_action(dims, 5.6, U0)
                  - orc.kinetic(dims, P0) + sf1 - np.vdot(eta, eta).real)
    assert abs(dHb - dH_rebuilt) < 1e-9 * max(1.0, abs(sf1)), (dHb, dH_rebuilt, sf1)


def test_md_tolerance_reversible(ctx, orc):
    dims = (6, 4, 4, 6)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 701, fermions=True)
    act = Action(beta=5.6, kappa=K, cg_tol=1e-12, prec="mp16", link_recon=12, cg_tol_md=1e-6)
    phi = orc.pf_heatbath(dims, K, U0, eta)
    U, P = dev(U0), dev(P0)
    dH1, _ = ctx.trajectory(dims, act, "FG", 1.0, 4, U, P, dev(phi), pf_is_phi=True)
    P.neg_()
    dH2, _ = ctx.trajectory(dims, act, "FG", 1.0, 4, U, P, dev(phi), pf_is_phi=True)
    # reversible to the MD tolerance: links that differ in the last bits can make
    # a solve stop one iteration earlier or later, a force change of order cg_tol_md
    assert relmax(host(U), U0) < 1e-7 and relmax(-host(P), P0) < 1e-7
    assert abs(dH1 + dH2) < 1e-5


def test_md_tolerance_validated(ctx):
    dims = (4, 4, 4, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 702, fermions=True)
    for bad in (-1e-8, 1.0, float("nan")):
        with pytest.raises(fgi.FgiError) as e:
            ctx.trajectory(dims, Action(beta=5.6, kappa=K, cg_tol_md=bad), "FG", 1.0, 2, dev(U0), dev(P0), dev(eta))
        assert e.value.code == fgi.FGI_EINVAL
