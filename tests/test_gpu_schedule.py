"""Schedules of the CG kernels (Dslash block size 64/128/256, XCD-aware or
linear block order, iterations per host poll) and the autotuner that picks
them.  Every schedule must give oracle-exact results (FP64: 1e-14 for the
Dslash, the solver tolerance for CG); a fixed schedule is bitwise
repeatable; batched chains stay bitwise equal to single-chain runs under the
same schedule.  Geometries: 6x4x4x6 (288 even sites: a ragged last block for
every block size) and 8^4."""
import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
SCHEDULES = [(bs, x) for bs in (64, 128, 256) for x in (0, 1)]


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(autouse=True)
def default_schedule(ctx):
    yield
    ctx.set_option("dslash_block", 256)
    ctx.set_option("xcd_order", 1)
    ctx.set_option("cg_batch", 8)
    ctx.set_option("cg_form", 0)


def set_schedule(ctx, bs, x):
    ctx.set_option("dslash_block", bs)
    ctx.set_option("xcd_order", x)


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


@pytest.mark.parametrize("bs,x", SCHEDULES)
@pytest.mark.parametrize("dims", [(6, 4, 4, 6), (8, 8, 8, 8)])
def test_dslash_each_schedule(ctx, orc, bs, x, dims):
    set_schedule(ctx, bs, x)
    U = links(dims, 80)
    V = synth.volume(dims)
    src = spinor(dims, 81)
    par = parity_of(dims)
    full = np.zeros((V, 4, 3), complex)
    full[par == 0] = src
    ref = orc.dhop(dims, U, full)[par == 1]
    out = host(ctx.dslash(dims, Action(beta=5.6, kappa=0.155), dev(U), dev(src), 1))
    assert relmax(out, ref) < 1e-14


@pytest.mark.parametrize("bs,x", SCHEDULES)
@pytest.mark.parametrize("prec", ["fp64", "mp16"])
def test_cg_each_schedule(ctx, orc, bs, x, prec):
    set_schedule(ctx, bs, x)
    dims = (6, 4, 4, 6)
    U0, phi0 = links(dims, 82), spinor(dims, 83)
    tol = 1e-12 if prec == "fp64" else 1e-10
    act = Action(beta=5.6, kappa=0.155, cg_tol=tol, prec=prec, link_recon=12 if prec != "fp64" else 18)
    X, st = ctx.cg_solve(dims, act, dev(U0), dev(phi0))
    X2, _ = ctx.cg_solve(dims, act, dev(U0), dev(phi0))
    assert np.array_equal(host(X), host(X2))
    assert st["max_rel_resid"] <= tol
    Xo, _, _ = orc.cg(dims, 0.155, U0, phi0, tol=1e-13)
    assert relmax(host(X), Xo) < (1e-10 if prec == "fp64" else 1e-8)


def test_fg_trajectory_linear_small_blocks(ctx, orc):
    set_schedule(ctx, 64, 0)
    dims = (4, 4, 4, 4)
    U0, P0, eta, _ = synth.hot_start(dims, 0x09102950 + 84, fermions=True)
    U, P = dev(U0), dev(P0)
    dH, _ = ctx.trajectory(dims, Action(beta=5.6, kappa=0.155, cg_tol=1e-14), "FG", 1.0, 4, U, P, dev(eta))
    Uo, Po, dHo, _, _ = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 4, U0, P0, kappa=0.155, eta=eta, tol=1e-14)
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12
    assert abs(dH - dHo) < 1e-9


def test_autotune_single(ctx, orc):
    dims = (8, 8, 8, 8)
    U0, phi0 = links(dims, 85), spinor(dims, 86)
    act = Action(beta=5.6, kappa=0.155, cg_tol=1e-10, prec="mp16", link_recon=12)
    t = ctx.autotune_cg(dims, act, dev(U0), dev(phi0))
    assert t["dslash_block"] in (64, 128, 256) and t["xcd_order"] in (0, 1)
    assert t["cg_batch"] in (4, 8, 16, 32, 64)
    assert all(v > 0 for v in t["sched_us_per_iter"]) and all(v > 0 for v in t["batch_ms_per_solve"])
    k = [64, 128, 256].index(t["dslash_block"])
    assert t["sched_us_per_iter"][2 * k + t["xcd_order"]] == min(t["sched_us_per_iter"])
    # both CG forms timed on full solves, the faster kept
    assert t["cg_form"] in (0, 1) and all(v > 0 for v in t["form_ms_per_solve"])
    assert t["form_ms_per_solve"][t["cg_form"]] == min(t["form_ms_per_solve"])
    # the context now runs the chosen schedule, and still solves correctly
    X, st = ctx.cg_solve(dims, act, dev(U0), dev(phi0))
    assert st["max_rel_resid"] <= 1e-10
    Xo, _, _ = orc.cg(dims, 0.155, U0, phi0, tol=1e-13)
    assert relmax(host(X), Xo) < 1e-8


MIX = [((4, 4, 4, 4), 5.6, 0.150), ((2, 2, 2, 2), 6.0, 0.157), ((6, 4, 4, 6), 5.8, 0.153), ((4, 6, 2, 8), 5.9, 0.151)]


def chains(seed):
    out = []
    for k, (dims, beta, kappa) in enumerate(MIX):
        U, P, eta, _ = synth.hot_start(dims, seed + k, fermions=True)
        out.append(dict(dims=dims, beta=beta, kappa=kappa, U0=U, P0=P, eta0=eta))
    return out


def as_args(chs):
    return [dict(dims=c["dims"], beta=c["beta"], kappa=c["kappa"], U=dev(c["U0"]), P=dev(c["P0"]), eta=dev(c["eta0"]))
            for c in chs]


@pytest.mark.parametrize("bs,x", [(64, 0), (128, 1)])
def test_batch_equals_single_under_schedule(ctx, bs, x):
    set_schedule(ctx, bs, x)
    chs = chains(0x09102950 + 87)
    act = Action(beta=0.0, cg_tol=1e-10, prec="mp16", link_recon=12)
    args = as_args(chs)
    dH, _ = ctx.trajectory_batched(args, act, "FG", 1.0, 3)
    for c, a, d in zip(chs, args, dH):
        a1 = Action(beta=c["beta"], kappa=c["kappa"], cg_tol=1e-10, prec="mp16", link_recon=12)
        U, P = dev(c["U0"]), dev(c["P0"])
        d1, _ = ctx.trajectory(c["dims"], a1, "FG", 1.0, 3, U, P, dev(c["eta0"]))
        assert np.array_equal(host(U), host(a["U"])) and np.array_equal(host(P), host(a["P"]))
        assert d1 == d


def test_autotune_batched(ctx, orc):
    chs = chains(0x09102950 + 88)
    act = Action(beta=0.0, cg_tol=1e-10, prec="mp16", link_recon=12)
    t = ctx.autotune_batched(as_args(chs), act)
    assert t["dslash_block"] in (64, 128, 256) and t["cg_batch"] in (4, 8, 16, 32, 64)
    args = as_args(chs)
    dH, st = ctx.trajectory_batched(args, Action(beta=0.0, cg_tol=1e-14), "FG", 1.0, 3)
    for c, a, d in zip(chs, args, dH):
        Uo, Po, dHo, _, _ = orc.trajectory(c["dims"], c["beta"], orc.table("FG"), 1.0, 3, c["U0"], c["P0"],
                                           kappa=c["kappa"], eta=c["eta0"], tol=1e-14)
        assert relmax(host(a["U"]), Uo) < 1e-12 and abs(d - dHo) < 1e-9


def test_schedule_options_validated(ctx):
    with pytest.raises(fgi.FgiError) as e:
        ctx.set_option("dslash_block", 96)
    assert e.value.code == fgi.FGI_EINVAL
