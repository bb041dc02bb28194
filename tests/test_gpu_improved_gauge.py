"""The improved gauge action (plaquettes at c0 = 1 - 8 c1, 2x1 rectangles at
c1) on the GPU against the oracle, through the C ABI.

  - action, force, force gradient J_V[F], Poisson brackets at c1 = -1/12 and
    -0.331 on lattices with extents 2 (rectangles that wrap onto themselves),
    mixed extents and several tiles, 1e-13 relative (1e-12 for J);
  - trajectories with every Table 1 integrator, the FG displacement and
    exact forms, pure gauge and with Wilson fermions: U and P to 1e-12,
    dH to 1e-9;
  - an on-device chain against the oracle's chain (identical decisions);
  - at 16^3x32 in the benchmark's launch configuration (block 256, XCD
    order): action, force on every link and the tangent, against the oracle;
  - batched chains of uneven sizes with c1: each bitwise equal to its own
    single-chain run (FP64 and MP16) and to the oracle;
  - c1 = 0 leaves the Wilson results bitwise unchanged; non-finite c1 is
    rejected.
"""
import math

import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
C1S = [-1.0 / 12.0, -0.331]
DIMS = [(2, 2, 2, 2), (4, 2, 2, 4), (6, 4, 4, 6), (8, 8, 8, 16)]


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


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("c1", C1S)
def test_action_and_force(ctx, orc, dims, c1):
    U = links(dims, 400)
    S = ctx.improved_gauge_action(dims, 5.6, c1, dev(U))
    So = orc.gauge_action(dims, 5.6, U, c1)
    assert abs(S - So) < 1e-13 * abs(So)
    F, _ = ctx.force(dims, Action(beta=5.6, c1=c1), dev(U))
    assert relmax(host(F), orc.gauge_force(dims, 5.6, U, c1)) < 1e-13


@pytest.mark.parametrize("dims", DIMS[:3])
@pytest.mark.parametrize("c1", C1S)
def test_force_gradient(ctx, orc, dims, c1):
    U = links(dims, 401)
    Vd = synth.rng(402).standard_normal((4, synth.volume(dims), 8))
    J, _ = ctx.total_force_gradient(dims, Action(beta=5.6, c1=c1), dev(U), V=dev(Vd))
    assert relmax(host(J), orc.gauge_force_tangent(dims, 5.6, U, Vd, c1)) < 1e-12
    # V = F: the force gradient itself
    F = orc.gauge_force(dims, 5.6, U, c1)
    J2, _ = ctx.total_force_gradient(dims, Action(beta=5.6, c1=c1), dev(U))
    assert relmax(host(J2), orc.gauge_force_tangent(dims, 5.6, U, F, c1)) < 1e-12


@pytest.mark.parametrize("fermions", [False, True])
def test_poisson_brackets(ctx, orc, fermions):
    dims, c1, kappa = (4, 4, 2, 2), -0.331, 0.155
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 403, fermions=True)
    act = Action(beta=5.6, kappa=kappa if fermions else 0.0, cg_tol=1e-14, c1=c1)
    phi = orc.pf_heatbath(dims, kappa, U0, eta) if fermions else None
    sst, tst = ctx.poisson_brackets(dims, act, dev(U0), dev(P0), dev(phi) if fermions else None, h=1e-4)
    so, to = orc.brackets(dims, 5.6, U0, P0, kappa=kappa if fermions else 0.0, phi=phi, h=1e-4, c1=c1)
    assert abs(sst - so) < 1e-11 * so and abs(tst - to) < 1e-7 * abs(to)


@pytest.mark.parametrize("name", ["PQP", "QPQ", "PQPQP", "CAMPOSTRINI", "FG"])
def test_trajectory_pure_gauge(ctx, orc, name):
    dims, c1 = (4, 4, 4, 4), -1 / 12
    U0, P0, _, _ = synth.hot_start(dims, synth.SEED_BASE + 404, fermions=False)
    U, P = dev(U0), dev(P0)
    dH, _ = ctx.trajectory(dims, Action(beta=5.6, c1=c1), name, 1.0, 4, U, P)
    Uo, Po, dHo, _, _ = orc.trajectory(dims, 5.6, orc.table(name), 1.0, 4, U0, P0, c1=c1)
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12 and abs(dH - dHo) < 1e-9


@pytest.mark.parametrize("fg_exact", [False, True])
@pytest.mark.parametrize("c1", C1S)
def test_fg_trajectory_with_fermions(ctx, orc, fg_exact, c1):
    dims, kappa = (4, 4, 2, 2), 0.155
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 405, fermions=True)
    act = Action(beta=5.6, kappa=kappa, cg_tol=1e-14, fg_exact=fg_exact, c1=c1)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, "FG", 1.0, 3, U, P, dev(eta))
    Uo, Po, dHo, sto, status = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 3, U0, P0, kappa=kappa, eta=eta,
                                              fg_exact=fg_exact, c1=c1)
    assert status == 0 and st["solves"] == sto["solves"]
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12 and abs(dH - dHo) < 1e-9


def test_mixed_precision_fg_trajectory(ctx, orc):
    """MP16 inner solves with the improved action: dH and fields within the
    solver tolerance of the FP64 oracle"""
    dims, kappa, c1 = (6, 4, 4, 6), 0.155, -0.331
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 406, fermions=True)
    act = Action(beta=5.6, kappa=kappa, cg_tol=1e-12, prec="mp16", link_recon=12, c1=c1)
    U, P = dev(U0), dev(P0)
    dH, _ = ctx.trajectory(dims, act, "FG", 1.0, 4, U, P, dev(eta))
    Uo, Po, dHo, _, _ = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 4, U0, P0, kappa=kappa, eta=eta, c1=c1)
    assert relmax(host(U), Uo) < 1e-8 and relmax(host(P), Po) < 1e-8 and abs(dH - dHo) < 1e-6


def test_chain_matches_oracle(ctx, orc):
    dims, c1, seed = (4, 4, 4, 4), -0.331, 23
    act = Action(beta=2.5, c1=c1)
    U0, _, _, _ = synth.hot_start(dims, synth.SEED_BASE + 407, fermions=False)
    U = dev(U0)
    dH, acc, plaq, _ = ctx.hmc_run(dims, act, "PQPQP", 1.0, 2, U, seed, 0, 12)
    Uo, dHo, acco, plo, _ = orc.hmc_run(dims, 2.5, orc.table("PQPQP"), 1.0, 2, U0, seed, 0, 12, c1=c1)
    for k in range(12):
        assert abs(orc.metropolis_uniform(seed, k) - np.exp(-dHo[k])) > 1e-6
    assert relmax(host(U), Uo) < 1e-11
    assert np.max(np.abs(np.array(dH) - dHo)) < 1e-9 and acc == acco
    assert np.max(np.abs(np.array(plaq) - plo)) < 1e-12
    assert 0 < sum(acc) < 12


def test_zero_c1_is_wilson_bitwise(ctx):
    dims = (6, 4, 4, 6)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 408, fermions=True)
    assert ctx.improved_gauge_action(dims, 5.6, 0.0, dev(U0)) == ctx.gauge_action(dims, 5.6, dev(U0))
    F1 = ctx.gauge_force(dims, 5.6, dev(U0))
    F2, _ = ctx.force(dims, Action(beta=5.6, c1=0.0), dev(U0))
    assert torch.equal(F1, F2)


def test_bad_c1_rejected(ctx):
    dims = (4, 4, 4, 4)
    U0, P0, _, _ = synth.hot_start(dims, synth.SEED_BASE + 409, fermions=False)
    for bad in (math.nan, math.inf):
        with pytest.raises(fgi.FgiError) as e:
            ctx.improved_gauge_action(dims, 5.6, bad, dev(U0))
        assert e.value.code == fgi.FGI_EINVAL
        U, P = dev(U0), dev(P0)
        with pytest.raises(fgi.FgiError) as e:
            ctx.trajectory(dims, Action(beta=5.6, c1=bad), "FG", 1.0, 2, U, P)
        assert e.value.code == fgi.FGI_EINVAL
        assert np.array_equal(host(U), U0)


@pytest.mark.parametrize("prec", ["fp64", "mp16"])
def test_batched_chains_equal_single_runs(ctx, orc, prec):
    """Chains of uneven sizes and couplings in one batched call, each bitwise
    equal to its own single-chain trajectory with the same c1; FP64 also
    against the oracle."""
    c1 = -0.331
    mix = [((4, 4, 4, 4), 5.6, 0.155), ((6, 4, 4, 6), 5.8, 0.150), ((4, 4, 2, 2), 5.5, 0.156)]
    tol = 1e-14 if prec == "fp64" else 1e-10
    chs = []
    for k, (dims, beta, kappa) in enumerate(mix):
        U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 420 + k, fermions=True)
        chs.append((dims, beta, kappa, U0, P0, eta))
    args = [dict(dims=d, beta=b, kappa=k, U=dev(U0), P=dev(P0), eta=dev(e)) for d, b, k, U0, P0, e in chs]
    act = Action(beta=0.0, cg_tol=tol, prec=prec, link_recon=12 if prec == "mp16" else 18, c1=c1)
    dH, _ = ctx.trajectory_batched(args, act, "FG", 1.0, 3)
    for (dims, beta, kappa, U0, P0, eta), a, d in zip(chs, args, dH):
        a1 = Action(beta=beta, kappa=kappa, cg_tol=tol, prec=prec, link_recon=act.link_recon, c1=c1)
        U, P = dev(U0), dev(P0)
        d1, _ = ctx.trajectory(dims, a1, "FG", 1.0, 3, U, P, dev(eta))
        assert torch.equal(U, a["U"]) and torch.equal(P, a["P"]) and d1 == d
        if prec == "fp64":
            Uo, Po, dHo, _, _ = orc.trajectory(dims, beta, orc.table("FG"), 1.0, 3, U0, P0, kappa=kappa, eta=eta,
                                               c1=c1)
            assert relmax(host(U), Uo) < 1e-12 and abs(d - dHo) < 1e-9


@pytest.fixture(scope="module")
def ctx_bench():
    c = Context(0)
    c.set_option("dslash_block", 256)
    c.set_option("xcd_order", 1)
    yield c
    c.close()


def test_full_size_16x32(ctx_bench, orc):
    dims, c1 = (16, 16, 16, 32), -0.331
    U = links(dims, 410)
    S = ctx_bench.improved_gauge_action(dims, 5.6, c1, dev(U))
    So = orc.gauge_action(dims, 5.6, U, c1)
    assert abs(S - So) < 1e-12 * abs(So)
    F, _ = ctx_bench.force(dims, Action(beta=5.6, c1=c1), dev(U))
    Fo = orc.gauge_force(dims, 5.6, U, c1)
    assert relmax(host(F), Fo) < 1e-13
    J, _ = ctx_bench.total_force_gradient(dims, Action(beta=5.6, c1=c1), dev(U))
    assert relmax(host(J), orc.gauge_force_tangent(dims, 5.6, U, Fo, c1)) < 1e-12
