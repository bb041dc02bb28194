"""GPU: the Chronopoulos-Gear form of the CG iteration (option cg_form = 1:
four launches per iteration instead of five; the operator is applied to the
residual, the direction's image follows by recurrence, and <p, A p> is
expanded exactly from reductions of the update kernel before).

Against the oracle's CG and against the classic form, through the C ABI:
  - FP64 to 1e-14 on geometries with a ragged block tail, the 2^4 edge case
    and anisotropic extents: the oracle's solution to 1e-12;
  - FP32 and FP16 inner solves (12- and 18-real links) with FP64 reliable
    updates to the 1e-10 true residual, on a Haar field and on a pure-gauge
    thermalised 8^4 field (a solve of ~200 iterations), with the iteration
    count within 15 % of the classic form's;
  - graph replays bitwise equal to eager launches; iterates and iteration
    count independent of how many iterations run between host polls;
  - at 16^3x32 (MP16) the oracle's FP64 residual of the GPU's solution meets
    1e-10;
  - an MP16 FG trajectory in either form ends at the same fields and dH to
    the solvers' accuracy; a nested Hasenbusch FG trajectory in this form
    matches the oracle's nested driver.
"""
import contextlib

import numpy as np
import pytest
import torch

from paper_0910_2950_amd import synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
GEOMS = [(2, 2, 2, 2), (6, 4, 4, 6), (4, 6, 2, 8), (8, 8, 8, 8)]
MP = [("mp32", 18), ("mp32", 12), ("mp16", 12), ("mp16", 18)]


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.set_option("cg_form", 0)
    c.close()


@contextlib.contextmanager
def form(ctx, f):
    ctx.set_option("cg_form", f)
    try:
        yield
    finally:
        ctx.set_option("cg_form", 0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.cpu().numpy()


def relmax(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def links(dims, seed):
    return synth.haar_su3(synth.rng(seed), 4 * synth.volume(dims)).reshape(4, -1, 3, 3)


def spinor(dims, seed):
    return synth.gaussian_noise(synth.rng(seed), dims)


@pytest.fixture(scope="module")
def therm8(ctx):
    """A pure-gauge field near equilibrium at beta = 5.83 (8^4, 100 FG
    trajectories from a Haar start on the GPU), on which the Nf = 2 solve at
    kappa = 0.155 takes ~200 iterations."""
    dims = (8, 8, 8, 8)
    U = dev(links(dims, 300))
    ctx.hmc_run(dims, Action(beta=5.83), "FG", 1.0, 10, U, 301, 0, 100, metropolis=False)
    ctx.reunitarize(dims, U)
    return host(U)


def solve(ctx, dims, act, U, phi, f):
    with form(ctx, f):
        X, st = ctx.cg_solve(dims, act, dev(U), dev(phi))
    return host(X), st


@pytest.mark.parametrize("dims", GEOMS)
def test_fp64_matches_oracle(ctx, orc, dims):
    U, phi = links(dims, 310), spinor(dims, 311)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-14)
    X, st = solve(ctx, dims, act, U, phi, 1)
    Xo, it, _ = orc.cg(dims, 0.155, U, phi, tol=1e-14)
    print(dims, "iterations", st["cg_iters"], "oracle", it, flush=True)
    assert st["max_rel_resid"] <= 1e-14
    assert relmax(X, Xo) < 1e-12
    assert st["cg_iters"] <= 1.15 * it + 3


@pytest.mark.parametrize("field", ["haar", "therm"])
@pytest.mark.parametrize("prec,recon", MP)
def test_mixed_precision(ctx, orc, therm8, field, prec, recon):
    dims = (8, 8, 8, 8)
    U = links(dims, 312) if field == "haar" else therm8
    phi = spinor(dims, 313)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-10, prec=prec, link_recon=recon)
    X1, st1 = solve(ctx, dims, act, U, phi, 1)
    _, st0 = solve(ctx, dims, act, U, phi, 0)
    print(field, prec, recon, "iterations: classic", st0["cg_iters"], "CG form", st1["cg_iters"],
          "reliable updates", st0["reliable_updates"], st1["reliable_updates"], flush=True)
    assert st1["max_rel_resid"] <= 1e-10 and st1["reliable_updates"] >= 1
    Xo, _, _ = orc.cg(dims, 0.155, U, phi, tol=1e-13)
    # the error of X is the residual times the condition number
    assert relmax(X1, Xo) < (1e-8 if field == "haar" else 1e-6)
    assert st1["cg_iters"] <= 1.15 * st0["cg_iters"] + 5


@pytest.mark.parametrize("prec", ["fp64", "mp32", "mp16"])
def test_graph_replays_match_eager(ctx, prec):
    dims = (8, 8, 8, 8)
    U = dev(links(dims, 320))
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-10, prec=prec, link_recon=12 if prec != "fp64" else 18)
    phis = [dev(spinor(dims, 321 + k)) for k in range(3)]
    with form(ctx, 1):
        try:
            ctx.set_option("graphs", 0)
            ref = [host(ctx.cg_solve(dims, act, U, ph)[0]) for ph in phis]
            ctx.set_option("graphs", 1)
            for k, ph in enumerate(phis):
                X, st = ctx.cg_solve(dims, act, U, ph)
                ctx.gauge_force(dims, 5.6, U)  # eager work between replays
                assert np.array_equal(host(X), ref[k]), (prec, k)
                assert st["max_rel_resid"] <= 1e-10
        finally:
            ctx.set_option("graphs", 1)


@pytest.mark.parametrize("prec", ["fp64", "mp32", "mp16"])
@pytest.mark.parametrize("dims", [(6, 4, 4, 6), (8, 8, 8, 8), (16, 16, 16, 32)])
def test_independent_of_batch_length(ctx, prec, dims):
    U = dev(links(dims, 330))
    phi = dev(spinor(dims, 331))
    tol = 1e-12 if prec == "fp64" else 1e-10
    act = Action(beta=5.6, kappa=0.155, cg_tol=tol, prec=prec, link_recon=12 if prec != "fp64" else 18)
    out = []
    with form(ctx, 1):
        try:
            for B in (1, 5, 64):
                ctx.set_option("cg_batch", B)
                X, st = ctx.cg_solve(dims, act, U, phi)
                out.append((host(X), st))
        finally:
            ctx.set_option("cg_batch", 8)
    for X, st in out:
        assert st["max_rel_resid"] <= tol
        assert st["cg_iters"] == out[0][1]["cg_iters"]
        assert np.array_equal(X, out[0][0]), prec


@pytest.mark.parametrize("recon", [12, 18])
def test_full_size_residual(ctx, orc, recon):
    dims = (16, 16, 16, 32)
    U = links(dims, 340)
    phi = orc.pf_heatbath(dims, 0.1575, U, spinor(dims, 341))
    act = Action(beta=5.6, kappa=0.1575, cg_tol=1e-10, prec="mp16", link_recon=recon)
    X, st = solve(ctx, dims, act, U, phi, 1)
    AX = orc.mhat(dims, 0.1575, U, orc.mhat(dims, 0.1575, U, X, 0), 1)
    rel = np.linalg.norm(phi - AX) / np.linalg.norm(phi)
    assert rel <= 1.01e-10 and st["max_rel_resid"] <= 1e-10, (rel, st)


def test_fg_trajectory_either_form(ctx, therm8):
    dims = (8, 8, 8, 8)
    _, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 350, fermions=True)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-12, prec="mp16", link_recon=18)
    res = []
    for f in (0, 1):
        U, P = dev(therm8), dev(P0)
        with form(ctx, f):
            dH, st = ctx.trajectory(dims, act, "FG", 1.0, 8, U, P, dev(eta))
        assert st["max_rel_resid"] <= 1e-12
        res.append((host(U), host(P), dH, st["cg_iters"]))
    print("dH classic %.10e CG form %.10e; iterations %d, %d" % (res[0][2], res[1][2], res[0][3], res[1][3]))
    assert relmax(res[1][0], res[0][0]) < 1e-8 and relmax(res[1][1], res[0][1]) < 1e-8
    assert abs(res[1][2] - res[0][2]) < 1e-6


@pytest.mark.parametrize("f", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "mp16"])
def test_repeat_calls_reuse_graphs(ctx, f, prec):
    """The captured CG batches are keyed by everything they capture; a repeated
    call with the same operator and buffers captures nothing new (an unset
    field in the key once made every solve capture afresh, at 1.8 times the
    cost per trajectory)."""
    dims = (8, 8, 8, 8)
    U, phi = dev(links(dims, 360)), dev(spinor(dims, 361))
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-10, prec=prec, link_recon=18)
    _, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 362, fermions=True)
    with form(ctx, f):
        ctx.cg_solve(dims, act, U, phi)
        X, st = ctx.cg_solve(dims, act, U, phi)
        assert st["graph_captures"] == 0, st
        for k in range(2):
            Ut, Pt = U.clone(), dev(P0)
            dH, st = ctx.trajectory(dims, act, "FG", 1.0, 4, Ut, Pt, dev(eta))
        assert st["graph_captures"] == 0, st


@pytest.mark.parametrize("prec", ["fp64", "mp16"])
def test_nested_hasenbusch_either_form(ctx, orc, prec):
    """Nested Hasenbusch FG trajectory (S_2 outer, S_1 middle, gauge inner)
    with every solve in the Chronopoulos-Gear form: the oracle's nested driver
    to the same gates as the classic form (FP64 1e-12 / 1e-9 with solves at
    1e-14; MP16 to the solver tolerance)."""
    from paper_0910_2950_amd import fgi as F
    dims = (6, 4, 4, 6) if prec == "fp64" else (8, 8, 8, 8)
    U0, P0, eta1, _ = synth.hot_start(dims, synth.SEED_BASE + 370, fermions=True)
    eta2 = synth.gaussian_noise(synth.rng(371), dims)
    fg = [("P", 1 / 6, 0.0), ("Q", 0.5, 0.0), ("G", 2 / 3, 1 / 72), ("Q", 0.5, 0.0), ("P", 1 / 6, 0.0)]
    levels = [(fg, F.TERM_HASEN, 1), (fg, F.TERM_FERMION, 2), (fg, F.TERM_GAUGE, 2)]
    tol = 1e-14 if prec == "fp64" else 1e-10
    act = Action(beta=5.6, kappa=0.155, kappa_hasen=0.140, cg_tol=tol, prec=prec,
                 link_recon=12 if prec != "fp64" else 18)
    U, P = dev(U0), dev(P0)
    with form(ctx, 1):
        dH, st = ctx.trajectory(dims, act, F.integrator_from_levels(levels), 1.0, 2, U, P, dev(eta1), dev(eta2))
    Uo, Po, dHo, sto, _ = orc.trajectory_nested(dims, 5.6, levels, 1.0, 2, U0, P0, kappa=0.155, kappa2=0.140,
                                                eta1=eta1, eta2=eta2, tol=1e-14 if prec == "fp64" else 1e-12)
    gate_u, gate_h = (1e-12, 1e-9) if prec == "fp64" else (1e-7, 1e-6)
    assert st["solves"] == sto["solves"]
    assert relmax(host(U), Uo) < gate_u and relmax(host(P), Po) < gate_u
    assert abs(dH - dHo) < gate_h, (dH, dHo)
