"""Stout-smeared fermion links on the GPU against the oracle, through the C ABI.

  - the smearing (1-3 levels, rho 0.1 and 0.25) on 2^4, 4.2.2.4, 6.4.4.6 and
    8.8.8.16 to 1e-13, its adjoint (a smeared-link force carried to the thin
    links) to 1e-12;
  - the total force with Nf=2 fermions on smeared links, the Poisson
    brackets, trajectories with four integrators (FP64: U, P to 1e-12, dH to
    1e-9; MP16 within the solver tolerance), nested Hasenbusch FG scales, and
    a chain with identical decisions;
  - 16^3x32 in the benchmark's launch configuration: the smearing and its
    adjoint against the oracle;
  - batched chains of uneven sizes with smearing: each bitwise equal to its
    own single-chain run (FP64 and MP16) and to the oracle;
  - zero levels leave the thin-link path bitwise; the exact G stage with
    smearing and out-of-range parameters are rejected.
"""
import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
DIMS = [(2, 2, 2, 2), (4, 2, 2, 4), (6, 4, 4, 6), (8, 8, 8, 16)]
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


def links(dims, seed):
    return synth.haar_su3(synth.rng(seed), 4 * synth.volume(dims)).reshape(4, -1, 3, 3)


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("rho,n", [(0.1, 1), (0.1, 3), (0.25, 2)])
def test_smear_and_adjoint(ctx, orc, dims, rho, n):
    U = links(dims, 600)
    Us = host(ctx.stout_smear(dims, rho, n, dev(U)))
    assert np.max(np.abs(Us - orc.stout_smear(dims, rho, n, U))) < 1e-13
    Fs = synth.rng(601).standard_normal((4, synth.volume(dims), 8))
    F = host(ctx.stout_force(dims, rho, n, dev(U), dev(Fs)))
    assert relmax(F, orc.stout_vjp(dims, rho, n, U, Fs)) < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 2, 2), (6, 4, 4, 6)])
def test_total_force(ctx, orc, dims):
    U0, _, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 602, fermions=True)
    phi = orc.pf_heatbath(dims, K, orc.stout_smear(dims, 0.12, 2, U0), eta)
    act = Action(beta=5.6, kappa=K, cg_tol=1e-14, stout_rho=0.12, stout_n=2)
    F, st = ctx.force(dims, act, dev(U0), dev(phi))
    Fo, _ = orc.force(dims, 5.6, U0, kappa=K, phi=phi, stout_rho=0.12, stout_n=2)
    assert relmax(host(F), Fo) < 1e-12


def test_poisson_brackets(ctx, orc):
    dims = (4, 4, 2, 2)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 603, fermions=True)
    phi = orc.pf_heatbath(dims, K, orc.stout_smear(dims, 0.1, 1, U0), eta)
    act = Action(beta=5.6, kappa=K, cg_tol=1e-14, stout_rho=0.1, stout_n=1)
    sst, tst = ctx.poisson_brackets(dims, act, dev(U0), dev(P0), dev(phi), h=1e-4)
    so, to = orc.brackets(dims, 5.6, U0, P0, kappa=K, phi=phi, h=1e-4, stout_rho=0.1, stout_n=1)
    assert abs(sst - so) < 1e-11 * so and abs(tst - to) < 1e-7 * abs(to)


@pytest.mark.parametrize("name", ["QPQ", "PQPQP", "CAMPOSTRINI", "FG"])
def test_trajectory(ctx, orc, name):
    dims = (4, 4, 2, 2)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 604, fermions=True)
    act = Action(beta=5.6, kappa=K, cg_tol=1e-14, stout_rho=0.12, stout_n=2)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, name, 1.0, 3, U, P, dev(eta))
    Uo, Po, dHo, sto, status = orc.trajectory(dims, 5.6, orc.table(name), 1.0, 3, U0, P0, kappa=K, eta=eta,
                                              stout_rho=0.12, stout_n=2)
    assert status == 0 and st["solves"] == sto["solves"]
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12 and abs(dH - dHo) < 1e-9


def test_trajectory_phi_given(ctx, orc):
    dims = (6, 4, 4, 6)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 605, fermions=True)
    phi = orc.pf_heatbath(dims, K, orc.stout_smear(dims, 0.1, 1, U0), eta)
    act = Action(beta=5.6, kappa=K, cg_tol=1e-14, stout_rho=0.1, stout_n=1, c1=-1 / 12)
    U, P = dev(U0), dev(P0)
    dH, _ = ctx.trajectory(dims, act, "FG", 1.0, 2, U, P, dev(phi), pf_is_phi=True)
    Uo, Po, dHo, _, _ = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 2, U0, P0, kappa=K, phi=phi,
                                       stout_rho=0.1, stout_n=1, c1=-1 / 12)
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12 and abs(dH - dHo) < 1e-9


def test_mixed_precision_trajectory(ctx, orc):
    dims = (6, 4, 4, 6)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 606, fermions=True)
    act = Action(beta=5.6, kappa=K, cg_tol=1e-12, prec="mp16", link_recon=12, stout_rho=0.1, stout_n=2)
    U, P = dev(U0), dev(P0)
    dH, _ = ctx.trajectory(dims, act, "FG", 1.0, 3, U, P, dev(eta))
    Uo, Po, dHo, _, _ = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 3, U0, P0, kappa=K, eta=eta,
                                       stout_rho=0.1, stout_n=2)
    assert relmax(host(U), Uo) < 1e-8 and relmax(host(P), Po) < 1e-8 and abs(dH - dHo) < 1e-6


@pytest.mark.parametrize("c1", [0.0, -0.331])
def test_nested_hasenbusch(ctx, orc, c1):
    dims = (4, 4, 2, 2)
    FG = orc.table("FG")
    levels = [(FG, 4, 1), (FG, 2, 2), (FG, 1, 2)]
    U0, P0, _, _ = synth.hot_start(dims, synth.SEED_BASE + 607, fermions=False)
    e1 = synth.gaussian_noise(synth.rng(608), dims)
    e2 = synth.gaussian_noise(synth.rng(609), dims)
    act = Action(beta=5.6, kappa=K, kappa_hasen=0.14, cg_tol=1e-14, stout_rho=0.1, stout_n=1, c1=c1)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, fgi.integrator_from_levels(levels), 1.0, 2, U, P, dev(e1), dev(e2))
    Uo, Po, dHo, sto, status = orc.trajectory_nested(dims, 5.6, levels, 1.0, 2, U0, P0, kappa=K, kappa2=0.14,
                                                     eta1=e1, eta2=e2, stout_rho=0.1, stout_n=1, c1=c1)
    assert status == 0 and st["solves"] == sto["solves"]
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12 and abs(dH - dHo) < 1e-9


def test_chain_matches_oracle(ctx, orc):
    dims, seed = (4, 4, 4, 4), 29
    act = Action(beta=5.6, kappa=K, cg_tol=1e-14, stout_rho=0.1, stout_n=2)
    U0, _, _, _ = synth.hot_start(dims, synth.SEED_BASE + 610, fermions=False)
    U = dev(U0)
    dH, acc, plaq, _ = ctx.hmc_run(dims, act, "FG", 1.0, 3, U, seed, 0, 3)
    Uo, dHo, acco, plo, _ = orc.hmc_run(dims, 5.6, orc.table("FG"), 1.0, 3, U0, seed, 0, 3, kappa=K,
                                        fermions=True, stout_rho=0.1, stout_n=2)
    for k in range(3):
        assert abs(orc.metropolis_uniform(seed, k) - np.exp(-dHo[k])) > 1e-6
    assert relmax(host(U), Uo) < 1e-11
    assert np.max(np.abs(np.array(dH) - dHo)) < 1e-9 and acc == acco


def test_zero_levels_bitwise_and_rejections(ctx):
    dims = (6, 4, 4, 6)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 611, fermions=True)
    a0 = Action(beta=5.6, kappa=K, cg_tol=1e-12)
    a1 = Action(beta=5.6, kappa=K, cg_tol=1e-12, stout_rho=0.2, stout_n=0)
    Ua, Pa, Ub, Pb = dev(U0), dev(P0), dev(U0), dev(P0)
    dHa, _ = ctx.trajectory(dims, a0, "FG", 1.0, 2, Ua, Pa, dev(eta))
    dHb, _ = ctx.trajectory(dims, a1, "FG", 1.0, 2, Ub, Pb, dev(eta))
    assert dHa == dHb and torch.equal(Ua, Ub) and torch.equal(Pa, Pb)
    bad = [Action(beta=5.6, kappa=K, stout_rho=0.1, stout_n=1, fg_exact=True),
           Action(beta=5.6, kappa=K, stout_rho=0.6, stout_n=1),
           Action(beta=5.6, kappa=K, stout_rho=0.1, stout_n=9),
           Action(beta=5.6, kappa=K, stout_rho=-0.1, stout_n=1)]
    for act in bad:
        U, P = dev(U0), dev(P0)
        with pytest.raises(fgi.FgiError) as e:
            ctx.trajectory(dims, act, "FG", 1.0, 2, U, P, dev(eta))
        assert e.value.code == fgi.FGI_EINVAL
        assert torch.equal(U, dev(U0))
    with pytest.raises(fgi.FgiError) as e:
        ctx.stout_smear(dims, 0.1, 9, dev(U0))
    assert e.value.code == fgi.FGI_EINVAL


@pytest.mark.parametrize("prec", ["fp64", "mp16"])
def test_batched_chains_equal_single_runs(ctx, orc, prec):
    """Chains of uneven sizes and couplings with smeared fermion links (and the
    improved gauge action) in one batched call, each bitwise equal to its own
    single-chain run; FP64 also against the oracle."""
    mix = [((4, 4, 4, 4), 5.6, 0.155), ((6, 4, 4, 6), 5.8, 0.150), ((4, 4, 2, 2), 5.5, 0.140)]
    tol = 1e-14 if prec == "fp64" else 1e-10
    sm = dict(stout_rho=0.12, stout_n=2, c1=-1 / 12)
    chs = []
    for k, (dims, beta, kappa) in enumerate(mix):
        U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 620 + k, fermions=True)
        chs.append((dims, beta, kappa, U0, P0, eta))
    args = [dict(dims=d, beta=b, kappa=k, U=dev(U0), P=dev(P0), eta=dev(e)) for d, b, k, U0, P0, e in chs]
    act = Action(beta=0.0, cg_tol=tol, prec=prec, link_recon=12 if prec == "mp16" else 18, **sm)
    dH, _ = ctx.trajectory_batched(args, act, "FG", 1.0, 3)
    for (dims, beta, kappa, U0, P0, eta), a, d in zip(chs, args, dH):
        a1 = Action(beta=beta, kappa=kappa, cg_tol=tol, prec=prec, link_recon=act.link_recon, **sm)
        U, P = dev(U0), dev(P0)
        d1, _ = ctx.trajectory(dims, a1, "FG", 1.0, 3, U, P, dev(eta))
        assert torch.equal(U, a["U"]) and torch.equal(P, a["P"]) and d1 == d
        if prec == "fp64":
            Uo, Po, dHo, _, _ = orc.trajectory(dims, beta, orc.table("FG"), 1.0, 3, U0, P0, kappa=kappa, eta=eta,
                                               **sm)
            assert relmax(host(U), Uo) < 1e-12 and abs(d - dHo) < 1e-9


@pytest.fixture(scope="module")
def ctx_bench():
    c = Context(0)
    c.set_option("dslash_block", 256)
    c.set_option("xcd_order", 1)
    yield c
    c.close()


def test_full_size_16x32(ctx_bench, orc):
    dims = (16, 16, 16, 32)
    U = links(dims, 612)
    Us = host(ctx_bench.stout_smear(dims, 0.1, 1, dev(U)))
    assert np.max(np.abs(Us - orc.stout_smear(dims, 0.1, 1, U))) < 1e-13
    Fs = synth.rng(613).standard_normal((4, synth.volume(dims), 8))
    F = host(ctx_bench.stout_force(dims, 0.1, 1, dev(U), dev(Fs)))
    assert relmax(F, orc.stout_vjp(dims, 0.1, 1, U, Fs)) < 1e-12
