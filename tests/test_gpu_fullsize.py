"""Parity at the benchmark lattices, in the launch configuration bench.py
times (block 256, XCD-aware order, cg_batch 16, MP16 inner solves with
12-real FP16 links; streamed links where the field exceeds the L2 caches).

16^3x32 (the FG trajectory workload) and 32^3x64 (the large-lattice Dslash
and Hasenbusch workload), on seeded Haar fields generated at full size (not
tiled, so an index that wraps with the wrong extent cannot hide):
  - hopping term, FP64 storage: every output site against the oracle, 1e-14
    relative to the largest entry; FP16 storage (spinor and links rounded to
    FP16 with per-site scales, FP32 arithmetic): 4e-3;
  - gauge force (32^3x64) and fermion force (16^3x32) against the oracle,
    1e-13;
  - CG at 16^3x32: the oracle's own FP64 evaluation of |phi - A X| for the
    GPU's mixed-precision solution meets the 1e-10 target;
  - one FG trajectory at 16^3x32 (n = 12, the benchmark's step count): the
    oracle rebuilds dH from the GPU's start and end fields (its gauge action,
    kinetic energy and a fresh FP64 solve for S_F at the end) and it agrees
    with the GPU's dH to the solver error of S_F; the final links are SU(3).
"""
import numpy as np
import pytest
import torch

from paper_0910_2950_amd import synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
L16 = (16, 16, 16, 32)
L32 = (32, 32, 32, 64)


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    c.set_option("dslash_block", 256)
    c.set_option("xcd_order", 1)
    c.set_option("cg_batch", 16)
    yield c
    c.set_option("cg_batch", 8)
    c.close()


@pytest.fixture(scope="module")
def fields():
    out = {}
    for k, dims in enumerate((L16, L32)):
        V = synth.volume(dims)
        U = synth.haar_su3(synth.rng(900 + k), 4 * V).reshape(4, V, 3, 3)
        out[dims] = U
    return out


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.cpu().numpy()


def relmax(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def parity_of(dims):
    V = synth.volume(dims)
    c = np.stack(np.unravel_index(np.arange(V), dims[::-1])[::-1], axis=1)
    return c.sum(axis=1) % 2


@pytest.mark.parametrize("dims", [L16, L32])
def test_dslash_full_size(ctx, orc, fields, dims):
    U = fields[dims]
    V = synth.volume(dims)
    src = synth.gaussian_noise(synth.rng(910), dims)
    par = parity_of(dims)
    full = np.zeros((V, 4, 3), complex)
    full[par == 0] = src
    ref = orc.dhop(dims, U, full)[par == 1]
    Ud, sd = dev(U), dev(src)
    out = host(ctx.dslash(dims, Action(beta=5.6, kappa=0.1575), Ud, sd, 1))
    assert relmax(out, ref) < 1e-14
    for recon in (12, 18):
        act16 = Action(beta=5.6, kappa=0.1575, prec="mp16", link_recon=recon)
        out16 = host(ctx.dslash(dims, act16, Ud, sd, 1, prec="mp16"))
        assert relmax(out16, ref) < 4e-3, recon


def test_gauge_force_full_size(ctx, orc, fields):
    U = fields[L32]
    F = host(ctx.gauge_force(L32, 5.6, dev(U)))
    assert relmax(F, orc.gauge_force(L32, 5.6, U)) < 1e-13


def test_fermion_force_full_size(ctx, orc, fields):
    U = fields[L16]
    X = synth.gaussian_noise(synth.rng(911), L16)
    act = Action(beta=5.6, kappa=0.1575)
    F = host(ctx.fermion_force(L16, act, dev(U), dev(X)))
    assert relmax(F, orc.fermion_force(L16, 0.1575, U, X)) < 1e-13


@pytest.mark.parametrize("recon", [12, 18])
def test_cg_full_size_residual(ctx, orc, fields, recon):
    U = fields[L16]
    eta = synth.gaussian_noise(synth.rng(912), L16)
    phi = orc.pf_heatbath(L16, 0.1575, U, eta)
    act = Action(beta=5.6, kappa=0.1575, cg_tol=1e-10, prec="mp16", link_recon=recon)
    X, st = ctx.cg_solve(L16, act, dev(U), dev(phi))
    X = host(X)
    AX = orc.mhat(L16, 0.1575, U, orc.mhat(L16, 0.1575, U, X, 0), 1)
    rel = np.linalg.norm(phi - AX) / np.linalg.norm(phi)
    assert rel <= 1.01e-10 and st["max_rel_resid"] <= 1e-10, (rel, st)


def test_fg_trajectory_full_size(ctx, orc):
    dims = L16
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 913, fermions=True)
    kappa, beta = 0.1575, 5.6
    act = Action(beta=beta, kappa=kappa, cg_tol=1e-12, prec="mp16", link_recon=12)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, act, "FG", 1.0, 12, U, P, dev(eta))
    U1, P1 = host(U), host(P)
    assert st["solves"] == 3 * 12 + 1 + 1 and st["max_rel_resid"] <= 1e-12
    phi = orc.pf_heatbath(dims, kappa, U0, eta)
    sf1, _ = orc.pf_action(dims, kappa, U1, phi, tol=1e-13)
    dH_o = (orc.gauge_action(dims, beta, U1) + orc.kinetic(dims, P1) - orc.gauge_action(dims, beta, U0)
            - orc.kinetic(dims, P0) + sf1 - np.vdot(eta, eta).real)
    # S_F ~ 8e5 here: a 1e-12 relative solve leaves ~1e-5 in dH on each side
    assert abs(dH - dH_o) < 1e-3, (dH, dH_o)
    assert np.max(np.abs(np.einsum("...ij,...kj->...ik", U1, U1.conj()) - np.eye(3))) < 1e-12


@pytest.mark.parametrize("recon", [12, 18])
def test_mp16_trajectory_tracks_fp64_full_size(ctx, recon):
    """At the benchmark lattice the mixed-precision FG trajectory (FP16 inner
    solves, FP64 reliable updates to the same 1e-10 true residual) ends where
    the FP64 one does: the solves differ only below their tolerance."""
    dims = L16
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 914, fermions=True)
    res = {}
    for prec, rc in (("fp64", 18), ("mp16", recon)):
        act = Action(beta=5.6, kappa=0.1575, cg_tol=1e-10, prec=prec, link_recon=rc)
        U, P = dev(U0), dev(P0)
        dH, st = ctx.trajectory(dims, act, "FG", 1.0, 12, U, P, dev(eta))
        assert st["max_rel_resid"] <= 1e-10
        res[prec] = (dH, host(U), host(P))
    (d64, U64, P64), (d16, U16, P16) = res["fp64"], res["mp16"]
    assert abs(d16 - d64) < 1e-5, (d16, d64)
    assert np.max(np.abs(U16 - U64)) < 1e-6
    assert np.max(np.abs(P16 - P64)) < 1e-6 * np.max(np.abs(P64))
