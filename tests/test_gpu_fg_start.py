"""The FG displacement form's displaced solve started from the undisplaced
solution (context option fg_start, on by default) against the oracle's
same reading, and with the option off against the oracle's zero start; the
start saves CG iterations, never solves.  Tolerances as in the trajectory
parity tests (FP64 CG 1e-14: links and momenta 1e-12 relative, dH 1e-9)."""
import numpy as np
import pytest
import torch

from paper_0910_2950_amd import synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.set_option("fg_start", 1)
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.cpu().numpy()


def relmax(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("fg_start", [0, 1])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 6)])
def test_fg_start_parity(ctx, orc, fg_start, dims):
    ctx.set_option("fg_start", fg_start)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 53, fermions=True)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, Action(beta=5.6, kappa=0.155, cg_tol=1e-14), "FG", 1.0, 4, U, P, dev(eta))
    Uo, Po, dHo, sto, _ = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 4, U0, P0, kappa=0.155, eta=eta,
                                         tol=1e-14, fg_start=bool(fg_start))
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12
    assert abs(dH - dHo) < 1e-9
    assert st["solves"] == sto["solves"]


@pytest.mark.parametrize("prec", ["fp64", "mp16"])
def test_fg_start_saves_iterations(ctx, prec):
    dims = (8, 8, 8, 8)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 54, fermions=True)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-10, prec=prec, link_recon=12 if prec == "mp16" else 18)
    res = {}
    for fs in (0, 1):
        ctx.set_option("fg_start", fs)
        U, P = dev(U0), dev(P0)
        dH, st = ctx.trajectory(dims, act, "FG", 1.0, 4, U, P, dev(eta))
        res[fs] = (dH, st, host(U))
    (d0, s0, u0), (d1, s1, u1) = res[0], res[1]
    assert s0["solves"] == s1["solves"] and s1["cg_iters"] < s0["cg_iters"]
    assert s1["max_rel_resid"] <= 1e-10
    assert abs(d0 - d1) < 1e-6 and relmax(u1, u0) < 1e-8
