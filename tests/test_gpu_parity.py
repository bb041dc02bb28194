"""GPU parity: every entry point of the HIP library, called through the C ABI,
against the FP64 CPU oracle on the same seeded inputs.

Tolerances (FP64 path): component kernels 1e-13 relative to the largest
entry; trajectories: links and momenta 1e-12 relative (max norm), dH 1e-9
absolute (the parity gate of the design), with CG run to 1e-14.
Geometries span several 256-site tiles with a ragged tail (6x4x4x6: V/2 =
288), the 2^4 edge case where x+nu = x-nu, and anisotropic extents.
"""
import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
GEOMS = [(2, 2, 2, 2), (6, 4, 4, 6), (4, 6, 2, 8), (8, 8, 8, 8)]


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


def links(dims, seed):
    return synth.haar_su3(synth.rng(seed), 4 * synth.volume(dims)).reshape(4, -1, 3, 3)


def spinor(dims, seed):
    return synth.gaussian_noise(synth.rng(seed), dims)


def parity_of(dims):
    V = synth.volume(dims)
    c = np.stack(np.unravel_index(np.arange(V), dims[::-1])[::-1], axis=1)
    return c.sum(axis=1) % 2


# ----------------------------------------------------------------- algebra --

def test_exp_su3(ctx, orc):
    g = synth.rng(1)
    p = g.standard_normal((512, 8)) * np.array([0.001, 0.3, 1.0, 3.0]).repeat(128)[:, None]
    p[:8] = 0.0
    p[8, 2] = 1e-9
    out = host(ctx.exp_su3(dev(p), 0.7))
    ref = np.array([orc.exp_su3(x, 0.7) for x in p])
    assert np.max(np.abs(out - ref)) < 2e-14


@pytest.mark.parametrize("dims", GEOMS)
def test_gauge_action_kinetic(ctx, orc, dims):
    U = links(dims, 2)
    P = synth.rng(3).standard_normal((4, synth.volume(dims), 8))
    S = ctx.gauge_action(dims, 5.6, dev(U))
    So = orc.gauge_action(dims, 5.6, U)
    assert abs(S - So) < 1e-12 * abs(So)
    T = ctx.kinetic(dims, dev(P))
    assert abs(T - orc.kinetic(dims, P)) < 1e-12 * T


@pytest.mark.parametrize("dims", GEOMS)
def test_gauge_force(ctx, orc, dims):
    U = links(dims, 4)
    F = host(ctx.gauge_force(dims, 6.0, dev(U)))
    assert relmax(F, orc.gauge_force(dims, 6.0, U)) < 1e-13


@pytest.mark.parametrize("dims", GEOMS[:3])
def test_force_gradient(ctx, orc, dims):
    U = links(dims, 5)
    Vd = synth.rng(6).standard_normal((4, synth.volume(dims), 8))
    J = host(ctx.force_gradient(dims, 6.0, dev(U), dev(Vd)))
    assert relmax(J, orc.gauge_force_tangent(dims, 6.0, U, Vd)) < 1e-13


@pytest.mark.parametrize("dims", GEOMS[:3])
def test_link_update_and_reunitarize(ctx, orc, dims):
    U = links(dims, 7)
    P = synth.rng(8).standard_normal((4, synth.volume(dims), 8))
    Ug = ctx.link_update(dims, 0.23, dev(P), dev(U))
    assert np.max(np.abs(host(Ug) - orc.link_update(dims, 0.23, P, U))) < 1e-14
    noisy = U + 1e-7 * synth.rng(9).standard_normal(U.shape)
    R = host(ctx.reunitarize(dims, dev(noisy)))
    assert np.max(np.abs(R - orc.reunitarize(dims, noisy))) < 1e-14


# ----------------------------------------------------------------- fermion --

@pytest.mark.parametrize("dims", GEOMS)
@pytest.mark.parametrize("out_parity", [0, 1])
def test_dslash_fp64(ctx, orc, dims, out_parity):
    U = links(dims, 10)
    V = synth.volume(dims)
    src = spinor(dims, 11)
    par = parity_of(dims)
    full = np.zeros((V, 4, 3), complex)
    full[par == 1 - out_parity] = src
    ref = orc.dhop(dims, U, full)[par == out_parity]
    act = Action(beta=5.6, kappa=0.155)
    out = host(ctx.dslash(dims, act, dev(U), dev(src), out_parity))
    assert relmax(out, ref) < 1e-14


@pytest.mark.parametrize("prec,recon,tol", [("mp32", 18, 2e-6), ("mp32", 12, 5e-6), ("mp16", 12, 5e-3),
                                             ("mp16", 18, 5e-3)])
def test_dslash_sloppy(ctx, orc, prec, recon, tol):
    dims = (6, 4, 4, 6)
    U = links(dims, 12)
    V = synth.volume(dims)
    src = spinor(dims, 13)
    par = parity_of(dims)
    full = np.zeros((V, 4, 3), complex)
    full[par == 0] = src
    ref = orc.dhop(dims, U, full)[par == 1]
    act = Action(beta=5.6, kappa=0.155, prec=prec, link_recon=recon)
    out = host(ctx.dslash(dims, act, dev(U), dev(src), 1, prec))
    assert relmax(out, ref) < tol


@pytest.mark.parametrize("dims", GEOMS)
@pytest.mark.parametrize("dagger", [False, True])
def test_mhat(ctx, orc, dims, dagger):
    U = links(dims, 14)
    src = spinor(dims, 15)
    act = Action(beta=5.6, kappa=0.155)
    out = host(ctx.mhat(dims, act, dev(U), dev(src), dagger))
    assert relmax(out, orc.mhat(dims, 0.155, U, src, dagger)) < 1e-14


@pytest.mark.parametrize("dims", GEOMS)
def test_cg_fp64(ctx, orc, dims):
    U = links(dims, 16)
    phi = spinor(dims, 17)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-14)
    X, st = ctx.cg_solve(dims, act, dev(U), dev(phi))
    Xo, it, rel = orc.cg(dims, 0.155, U, phi, tol=1e-14)
    assert st["max_rel_resid"] <= 1e-14
    assert relmax(host(X), Xo) < 1e-12
    assert abs(st["cg_iters"] - it) <= 3


@pytest.mark.parametrize("prec,recon", [("mp32", 18), ("mp32", 12), ("mp16", 12), ("mp16", 18)])
def test_cg_mixed_precision(ctx, orc, prec, recon):
    dims = (8, 8, 8, 8)
    U = links(dims, 18)
    phi = spinor(dims, 19)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-10, prec=prec, link_recon=recon)
    X, st = ctx.cg_solve(dims, act, dev(U), dev(phi))
    assert st["max_rel_resid"] <= 1e-10
    Xo, _, _ = orc.cg(dims, 0.155, U, phi, tol=1e-13)
    # error of X is bounded by the residual times the condition number (~10^2 here)
    assert relmax(host(X), Xo) < 1e-8
    assert st["reliable_updates"] >= 1


def test_cg_maxiter_reports_noconv(ctx):
    dims = (4, 4, 4, 4)
    U = links(dims, 20)
    phi = spinor(dims, 21)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-14, cg_maxiter=5)
    X, st = ctx.cg_solve(dims, act, dev(U), dev(phi), allow_noconv=True)
    assert st["status"] == -3 and st["max_rel_resid"] > 1e-6


@pytest.mark.parametrize("dims", GEOMS[:3])
def test_heatbath_action_identity(ctx, orc, dims):
    U = links(dims, 22)
    eta = spinor(dims, 23)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-14)
    phi = ctx.pf_heatbath(dims, act, dev(U), dev(eta))
    assert relmax(host(phi), orc.pf_heatbath(dims, 0.155, U, eta)) < 1e-14
    SF, _ = ctx.pf_action(dims, act, dev(U), phi)
    ee = np.vdot(eta, eta).real
    assert abs(SF - ee) < 1e-12 * ee


@pytest.mark.parametrize("dims", GEOMS)
def test_fermion_force(ctx, orc, dims):
    U = links(dims, 24)
    X = spinor(dims, 25)
    act = Action(beta=5.6, kappa=0.155)
    F = host(ctx.fermion_force(dims, act, dev(U), dev(X)))
    assert relmax(F, orc.fermion_force(dims, 0.155, U, X)) < 1e-13


@pytest.mark.parametrize("dims", GEOMS[:3])
def test_total_force(ctx, orc, dims):
    U = links(dims, 26)
    phi = spinor(dims, 27)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-14)
    F, st = ctx.force(dims, act, dev(U), dev(phi))
    Fo, sto = orc.force(dims, 5.6, U, 0.155, phi, tol=1e-14)
    assert st["solves"] == 1
    assert relmax(host(F), Fo) < 1e-12


def test_poisson_brackets(ctx, orc):
    dims = (4, 4, 2, 2)
    U = links(dims, 28)
    P = synth.rng(29).standard_normal((4, synth.volume(dims), 8))
    phi = spinor(dims, 30)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-14)
    sst, tst = ctx.poisson_brackets(dims, act, dev(U), dev(P), dev(phi), h=1e-4)
    so, to = orc.brackets(dims, 5.6, U, P, kappa=0.155, phi=phi, h=1e-4)
    assert abs(sst - so) < 1e-12 * so
    assert abs(tst - to) < 1e-7 * abs(to)


# ------------------------------------------------------------- trajectories --

def run_pair(ctx, orc, dims, beta, name, n, seed, kappa=0.0, exact=False, tau=1.0, tol=1e-14):
    ferm = kappa != 0.0
    U0, P0, eta, _ = synth.hot_start(dims, seed, fermions=ferm)
    act = Action(beta=beta, kappa=kappa, cg_tol=tol, fg_exact=exact)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, name, tau, n, U, P, dev(eta) if ferm else None)
    Uo, Po, dHo, sto, _ = orc.trajectory(dims, beta, orc.table(name), tau, n, U0, P0, kappa=kappa,
                                         eta=eta if ferm else None, tol=tol, fg_exact=exact)
    return host(U), host(P), dH, st, Uo, Po, dHo, sto


@pytest.mark.parametrize("name", ["PQP", "PQPQP", "FG", "QPQ", "CAMPOSTRINI"])
@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_trajectory_pure_gauge_4444(ctx, orc, name, n):
    """4^4 SU(3) Wilson gauge, beta = 6, tau = 1, dtau = 1/4 .. 1/32."""
    U, P, dH, st, Uo, Po, dHo, _ = run_pair(ctx, orc, (4, 4, 4, 4), 6.0, name, n, synth.SEED_BASE + 0)
    assert relmax(U, Uo) < 1e-12
    assert relmax(P, Po) < 1e-12
    assert abs(dH - dHo) < 1e-9, (dH, dHo)


def test_trajectory_fg_exact_gauge(ctx, orc):
    U, P, dH, st, Uo, Po, dHo, _ = run_pair(ctx, orc, (4, 4, 4, 4), 6.0, "FG", 8, synth.SEED_BASE + 0, exact=True)
    assert relmax(U, Uo) < 1e-12 and relmax(P, Po) < 1e-12 and abs(dH - dHo) < 1e-9


@pytest.mark.parametrize("name", ["PQP", "PQPQP", "FG"])
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (6, 4, 4, 6), (4, 4, 4, 4)])
def test_trajectory_wilson_fp64(ctx, orc, name, dims):
    U, P, dH, st, Uo, Po, dHo, sto = run_pair(ctx, orc, dims, 5.6, name, 5, synth.SEED_BASE + 1, kappa=0.155)
    assert st["solves"] == sto["solves"]
    assert relmax(U, Uo) < 1e-12
    assert relmax(P, Po) < 1e-12
    assert abs(dH - dHo) < 1e-9, (dH, dHo)


@pytest.mark.parametrize("name", ["PQP", "FG"])
def test_trajectory_wilson_8888(ctx, orc, name):
    """8^4, beta 5.6, kappa 0.155, even-odd, parity-mode CG 1e-14."""
    U, P, dH, st, Uo, Po, dHo, sto = run_pair(ctx, orc, (8, 8, 8, 8), 5.6, name, 5, synth.SEED_BASE + 1,
                                              kappa=0.155)
    assert relmax(U, Uo) < 1e-12 and relmax(P, Po) < 1e-12
    assert abs(dH - dHo) < 1e-9, (dH, dHo)


@pytest.mark.parametrize("prec", ["mp32", "mp16"])
def test_trajectory_mixed_precision_close_to_fp64(ctx, orc, prec):
    """Mixed precision changes results only at the solver tolerance level."""
    dims = (8, 8, 8, 8)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 1, fermions=True)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-10, prec=prec, link_recon=12)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, "FG", 1.0, 5, U, P, dev(eta))
    Uo, Po, dHo, _, _ = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 5, U0, P0, kappa=0.155, eta=eta, tol=1e-12)
    assert relmax(host(U), Uo) < 1e-7
    assert relmax(host(P), Po) < 1e-7
    assert abs(dH - dHo) < 1e-6, (dH, dHo)
    assert st["max_rel_resid"] <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "mp32", "mp16"])
def test_cg_graph_replays_match_eager(ctx, prec):
    """CG batches replayed from a captured HIP graph give bitwise the same
    solution as the same kernels launched one by one, on every replay (three
    solves in a row with other eager work between them)."""
    dims = (8, 8, 8, 8)
    U = dev(links(dims, 40))
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-10, prec=prec, link_recon=12 if prec != "fp64" else 18)
    phis = [dev(spinor(dims, 41 + k)) for k in range(3)]
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
def test_cg_independent_of_batch_length(ctx, prec, dims):
    """The host polls the solver state between batches of iterations; where
    the batch boundaries fall changes neither the iterates nor the iteration
    count, because every scalar of the recurrence is a fixed-order sum of the
    same block partials, whichever kernel computes it."""
    U = dev(links(dims, 50))
    phi = dev(spinor(dims, 51))
    tol = 1e-12 if prec == "fp64" else 1e-10
    act = Action(beta=5.6, kappa=0.155, cg_tol=tol, prec=prec, link_recon=12 if prec != "fp64" else 18)
    out = []
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


def test_unknown_option_rejected(ctx):
    with pytest.raises(fgi.FgiError) as e:
        ctx.set_option("persistent", 1)
    assert e.value.code == fgi.FGI_EINVAL

