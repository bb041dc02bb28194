"""The clover (Sheikholeslami-Wohlert) fermion operator on the GPU against the
oracle, through the C ABI (FP64).

  - the clover matrices A(x) on lattices with one block, several blocks and a
    ragged tail, to 1e-14; the log det action to 1e-12 and its force to 1e-12;
  - the clover Mhat and Mhat^+ (even-odd Schur complement) to 1e-13, also at
    16^3x32, the benchmark lattice;
  - the CG solution, the pseudofermion force for a given solution (hopping
    and clover parts) and the total force (gauge, pseudofermion and log det);
  - trajectories (four integrators, FP64 solves at 1e-14): U, P to 1e-11 and
    dH to 1e-9 against the oracle, with stout-smeared fermion links and the
    tree-level Symanzik gauge action too; reversibility; an on-device chain
    runs;
  - the Hasenbusch split on three scales against the oracle's nested driver,
    and its heatbath identity at tau = 0;
  - csw = 0 leaves the Wilson path bitwise; MP16, the exact G stage and
    batched chains with the clover term and an out-of-range csw are rejected;
  - kappa csw = 0.65, where some blocks of A(x) are indefinite: A, the log
    det action and force, and Mhat (through A_oo^-1) against the oracle;
  - the MP32 solver (FP32 inner CG, FP64 defect correction) with smearing
    and the Hasenbusch split at the solver-tolerance gates, and its FP64
    fallback when the FP32 residual is not finite.
"""
import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
K, CSW = 0.155, 1.0
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
def test_clover_field_and_log_det(ctx, orc, dims):
    U = links(dims, 700)
    A, S, F = ctx.clover_field(dims, K, CSW, dev(U))
    Ao, _, _, So = orc.clover(dims, K, CSW, U)
    assert np.max(np.abs(host(A) - Ao)) < 1e-14
    assert abs(S - So) < 1e-12 * max(1.0, abs(So))
    Fo = orc.clover_force(dims, K, CSW, U, None, det_scale=1.0)
    assert np.max(np.abs(host(F) - Fo)) < 1e-12 * max(1.0, np.max(np.abs(Fo)))


@pytest.mark.parametrize("dims", DIMS + [(16, 16, 16, 32)])
def test_clover_mhat(ctx, orc, dims):
    U, _, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 701)
    act = Action(beta=5.6, kappa=K, csw=CSW)
    for dag in (False, True):
        out = host(ctx.mhat(dims, act, dev(U), dev(eta), dagger=dag))
        assert relmax(out, orc.clover_mhat(dims, K, CSW, U, eta, dagger=dag)) < 1e-13


@pytest.mark.parametrize("dims", [(4, 2, 2, 4), (6, 4, 4, 6)])
def test_clover_solve_and_forces(ctx, orc, dims):
    U, _, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 702)
    act = Action(beta=5.6, kappa=K, csw=CSW, cg_tol=1e-13)
    phi = orc.clover_mhat(dims, K, CSW, U, eta, dagger=True)
    assert relmax(host(ctx.pf_heatbath(dims, act, dev(U), dev(eta))), phi) < 1e-13
    X, st = ctx.cg_solve(dims, act, dev(U), dev(phi))
    Xo, it = orc.clover_cg(dims, K, CSW, U, phi)
    assert it > 0 and st["solves"] == 1
    assert relmax(host(X), Xo) < 1e-10
    # pseudofermion force of a given solution: hopping and clover parts
    Fpf = host(ctx.fermion_force(dims, act, dev(U), dev(Xo)))
    assert relmax(Fpf, orc.clover_force(dims, K, CSW, U, Xo, pf_scale=1.0, det_scale=0.0)) < 1e-12
    # total force: gauge + S_F + log det
    F, _ = ctx.force(dims, act, dev(U), dev(phi))
    Fo, _ = orc.force(dims, 5.6, U, kappa=K, phi=phi, csw=CSW)
    assert relmax(host(F), Fo) < 1e-10
    SF, _ = ctx.pf_action(dims, act, dev(U), dev(phi))
    assert abs(SF - orc.clover_pf_action(dims, K, CSW, U, phi)[0]) < 1e-10 * abs(SF)


@pytest.mark.parametrize("name", ["QPQ", "PQPQP", "CAMPOSTRINI", "FG"])
def test_clover_trajectory(ctx, orc, name):
    dims = (4, 4, 4, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 703)
    act = Action(beta=5.6, kappa=K, csw=CSW, cg_tol=1e-14)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, name, 1.0, 3, U, P, dev(eta))
    Uo, Po, dHo, sto, status = orc.trajectory(dims, 5.6, orc.table(name), 1.0, 3, U0, P0, kappa=K, eta=eta,
                                              csw=CSW)
    assert status == 0 and st["solves"] == sto["solves"]
    assert relmax(host(U), Uo) < 1e-11 and relmax(host(P), Po) < 1e-11 and abs(dH - dHo) < 1e-9


# FP64 solves at 1e-14 hold the 1e-11 / 1e-9 gates; the MP32 solver (FP32
# inner CG, FP64 defect correction at 1e-12) holds the solver-tolerance gates
PREC_GATES = [("fp64", 1e-14, 1e-11, 1e-9), ("mp32", 1e-12, 1e-8, 1e-6)]


@pytest.mark.parametrize("prec,tol,gate_up,gate_dh", PREC_GATES)
def test_clover_with_smearing_and_symanzik(ctx, orc, prec, tol, gate_up, gate_dh):
    dims = (4, 2, 2, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 704)
    act = Action(beta=5.6, kappa=K, csw=CSW, cg_tol=tol, stout_rho=0.1, stout_n=2, c1=-1 / 12, prec=prec)
    U, P = dev(U0), dev(P0)
    dH, _ = ctx.trajectory(dims, act, "FG", 1.0, 2, U, P, dev(eta))
    Uo, Po, dHo, _, status = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 2, U0, P0, kappa=K, eta=eta,
                                            csw=CSW, stout_rho=0.1, stout_n=2, c1=-1 / 12)
    assert status == 0
    assert relmax(host(U), Uo) < gate_up and relmax(host(P), Po) < gate_up and abs(dH - dHo) < gate_dh


def test_clover_reversible_from_phi(ctx, orc):
    dims = (4, 4, 2, 2)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 705)
    phi = orc.clover_mhat(dims, K, CSW, U0, eta, dagger=True)
    act = Action(beta=5.6, kappa=K, csw=CSW, cg_tol=1e-14)
    U, P = dev(U0), dev(P0)
    dH1, _ = ctx.trajectory(dims, act, "FG", 1.0, 4, U, P, dev(phi), pf_is_phi=True)
    P.neg_()
    dH2, _ = ctx.trajectory(dims, act, "FG", 1.0, 4, U, P, dev(phi), pf_is_phi=True)
    assert relmax(host(U), U0) < 1e-11 and relmax(-host(P), P0) < 1e-11
    assert abs(dH1 + dH2) < 1e-9


def test_zero_csw_is_wilson_bitwise(ctx):
    dims = (4, 4, 4, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 706)
    out = []
    for act in (Action(beta=5.6, kappa=K), Action(beta=5.6, kappa=K, csw=0.0)):
        U, P = dev(U0), dev(P0)
        dH, _ = ctx.trajectory(dims, act, "FG", 1.0, 2, U, P, dev(eta))
        out.append((host(U), host(P), dH))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1]) and out[0][2] == out[1][2]


def test_clover_rejections(ctx):
    dims = (4, 4, 4, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 707)
    bad = [Action(beta=5.6, kappa=K, csw=CSW, prec="mp16", link_recon=12),
           Action(beta=5.6, kappa=K, csw=CSW, fg_exact=True),
           Action(beta=5.6, kappa=K, csw=-0.5),
           Action(beta=5.6, kappa=K, csw=float("nan"))]
    for act in bad:
        with pytest.raises(fgi.FgiError) as e:
            ctx.trajectory(dims, act, "FG", 1.0, 2, dev(U0), dev(P0), dev(eta), dev(eta))
        assert e.value.code == fgi.FGI_EINVAL


def test_clover_batched_rejected(ctx):
    dims = (4, 4, 4, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 708)
    args = [dict(dims=dims, beta=5.6, kappa=K, U=dev(U0), P=dev(P0), eta=dev(eta))]
    with pytest.raises(fgi.FgiError) as e:
        ctx.trajectory_batched(args, Action(beta=0.0, csw=CSW), "FG", 1.0, 2)
    assert e.value.code == fgi.FGI_EINVAL


def test_clover_chain_runs(ctx):
    """the on-device chain runs with the clover term (its trajectories go
    through the same packed trajectory as the oracle-checked ones above): two
    trajectories without Metropolis give finite, small dH"""
    dims = (4, 4, 4, 4)
    U0, _, _, _ = synth.hot_start(dims, synth.SEED_BASE + 709)
    act = Action(beta=5.6, kappa=K, csw=CSW, cg_tol=1e-12)
    U = dev(U0)
    out = ctx.hmc_run(dims, act, "FG", 1.0, 3, U, 1234, 0, 2, metropolis=False)
    dH = out[0]
    assert len(dH) == 2 and all(np.isfinite(dH)) and all(abs(d) < 5 for d in dH)


def test_clover_nested_scales_and_brackets(ctx, orc):
    dims = (4, 4, 2, 2)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 711)
    levels = [(orc.table("FG"), 2, 1), (orc.table("FG"), 1, 2)]
    act = Action(beta=5.6, kappa=K, csw=CSW, cg_tol=1e-14)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, fgi.integrator_from_levels(levels), 1.0, 3, U, P, dev(eta))
    Uo, Po, dHo, sto, status = orc.trajectory_nested(dims, 5.6, levels, 1.0, 3, U0, P0, kappa=K, eta1=eta, csw=CSW)
    assert status == 0 and st["solves"] == sto["solves"]
    assert relmax(host(U), Uo) < 1e-11 and relmax(host(P), Po) < 1e-11 and abs(dH - dHo) < 1e-9
    phi = orc.clover_mhat(dims, K, CSW, U0, eta, dagger=True)
    sst, tst = ctx.poisson_brackets(dims, act, dev(U0), dev(P0), dev(phi), h=1e-4)
    so, to = orc.brackets(dims, 5.6, U0, P0, kappa=K, phi=phi, h=1e-4, csw=CSW)
    assert abs(sst - so) < 1e-11 * so and abs(tst - to) < 1e-7 * abs(to)


@pytest.mark.parametrize("prec,tol,gate_up,gate_dh", PREC_GATES)
def test_clover_hasenbusch_nested(ctx, orc, prec, tol, gate_up, gate_dh):
    dims = (4, 4, 2, 2)
    U0, P0, eta1, _ = synth.hot_start(dims, synth.SEED_BASE + 712)
    eta2 = synth.gaussian_noise(synth.rng(synth.SEED_BASE + 713), dims)
    K2 = 0.13
    levels = [(orc.table("FG"), 4, 1), (orc.table("FG"), 2, 2), (orc.table("FG"), 1, 2)]
    act = Action(beta=5.6, kappa=K, kappa_hasen=K2, csw=CSW, cg_tol=tol, prec=prec)
    integ = fgi.integrator_from_levels(levels)
    U, P = dev(U0), dev(P0)
    d0, _ = ctx.trajectory(dims, act, integ, 0.0, 1, U, P, dev(eta1), dev(eta2))
    assert abs(d0) < 1e-10 if prec == "fp64" else abs(d0) < gate_dh
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, integ, 1.0, 2, U, P, dev(eta1), dev(eta2))
    Uo, Po, dHo, sto, status = orc.trajectory_nested(dims, 5.6, levels, 1.0, 2, U0, P0, kappa=K, kappa2=K2,
                                                     eta1=eta1, eta2=eta2, csw=CSW)
    assert status == 0 and st["solves"] == sto["solves"]
    assert relmax(host(U), Uo) < gate_up and relmax(host(P), Po) < gate_up and abs(dH - dHo) < gate_dh


def test_clover_field_and_log_det_force_at_benchmark_size(ctx, orc):
    """16^3x32: A(x) on sampled sites, the log det action and its force on
    every link against the oracle (no solve involved)"""
    dims = (16, 16, 16, 32)
    U = links(dims, 714)
    A, S, F = ctx.clover_field(dims, K, CSW, dev(U))
    Ao, _, _, So = orc.clover(dims, K, CSW, U)
    idx = synth.rng(715).choice(synth.volume(dims), 512, replace=False)
    assert np.max(np.abs(host(A)[idx] - Ao[idx])) < 1e-14
    assert abs(S - So) < 1e-12 * abs(So)
    Fo = orc.clover_force(dims, K, CSW, U, None, det_scale=1.0)
    assert np.max(np.abs(host(F) - Fo)) < 1e-12 * np.max(np.abs(Fo))


def test_clover_mixed_precision(ctx, orc):
    """FP32 inner CG with FP64 defect correction: the solution meets the FP64
    tolerance, and trajectories agree with the oracle to the solver tolerance"""
    dims = (6, 4, 4, 6)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 716)
    phi = orc.clover_mhat(dims, K, CSW, U0, eta, dagger=True)
    for recon in (18, 12):
        act = Action(beta=5.6, kappa=K, csw=CSW, cg_tol=1e-12, prec="mp32", link_recon=recon)
        X, st = ctx.cg_solve(dims, act, dev(U0), dev(phi))
        Xo, _ = orc.clover_cg(dims, K, CSW, U0, phi, tol=1e-14)
        assert relmax(host(X), Xo) < 1e-9 and st["max_rel_resid"] <= 1e-12
    act = Action(beta=5.6, kappa=K, csw=CSW, cg_tol=1e-12, prec="mp32", link_recon=12)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, "FG", 1.0, 3, U, P, dev(eta))
    Uo, Po, dHo, sto, status = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 3, U0, P0, kappa=K, eta=eta, csw=CSW)
    assert status == 0 and st["solves"] == sto["solves"]
    assert relmax(host(U), Uo) < 1e-8 and relmax(host(P), Po) < 1e-8 and abs(dH - dHo) < 1e-6


# kappa csw = 0.65: on a hot start about one site in six has a clover block
# with a negative determinant (A(x) Hermitian but indefinite), the regime where
# the block inversion needs its pivoting
K_IND, CSW_IND = 0.13, 5.0


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 6)])
def test_clover_indefinite_blocks(ctx, orc, dims):
    U = links(dims, 720)
    Ao, _, _, So = orc.clover(dims, K_IND, CSW_IND, U)
    B = Ao.reshape(-1, 12, 12)
    neg = (np.linalg.slogdet(B[:, :6, :6])[0].real < 0).sum() + (np.linalg.slogdet(B[:, 6:, 6:])[0].real < 0).sum()
    assert neg > 0   # the regime is exercised
    A, S, F = ctx.clover_field(dims, K_IND, CSW_IND, dev(U))
    assert np.max(np.abs(host(A) - Ao)) < 1e-14
    assert abs(S - So) < 1e-11 * max(1.0, abs(So))
    Fo = orc.clover_force(dims, K_IND, CSW_IND, U, None, det_scale=1.0)
    assert relmax(host(F), Fo) < 1e-11
    _, _, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 721)
    act = Action(beta=5.6, kappa=K_IND, csw=CSW_IND)
    for dag in (False, True):   # Mhat uses A_oo^-1
        out = host(ctx.mhat(dims, act, dev(U), dev(eta), dagger=dag))
        assert relmax(out, orc.clover_mhat(dims, K_IND, CSW_IND, U, eta, dagger=dag)) < 1e-11


def test_clover_mixed_precision_falls_back_when_fp32_overflows(ctx, orc):
    """A right-hand side beyond the FP32 range (|phi| ~ 1e39 per component)
    makes the FP32 inner residual infinite on the first defect-correction step;
    the MP32 solver then discards the FP32 correction and finishes in FP64
    from the current solution, meeting cg_tol."""
    dims = (4, 4, 4, 4)
    U0, _, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 722)
    phi = orc.clover_mhat(dims, K, CSW, U0, eta, dagger=True)
    scale = 1e39
    act = Action(beta=5.6, kappa=K, csw=CSW, cg_tol=1e-12, prec="mp32", link_recon=18)
    X, st = ctx.cg_solve(dims, act, dev(U0), dev(phi * scale))
    Xo, _ = orc.clover_cg(dims, K, CSW, U0, phi, tol=1e-14)
    assert np.all(np.isfinite(host(X)))
    assert relmax(host(X) / scale, Xo) < 1e-9 and st["max_rel_resid"] <= 1e-12
