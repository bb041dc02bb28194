"""Degenerate and invalid inputs through the C ABI.

  - tau = 0: every stage is the identity, so U and P come back bitwise and
    dH is zero up to the final solve's tolerance;
  - eta = 0 (phi = 0): the pseudofermion force and action vanish (CG returns
    X = 0 at once) and the trajectory is the pure-gauge one;
  - beta = 0 with fermions: the fermion-only Hamiltonian against the oracle;
  - the smallest lattice 2^4 with fermions and every integrator;
  - invalid geometry, step count, tau, precision and action arguments are
    rejected before any launch, leaving the outputs untouched.
"""
import math

import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


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


@pytest.mark.parametrize("name", ["PQP", "QPQ", "PQPQP", "CAMPOSTRINI", "FG"])
def test_zero_tau_is_identity(ctx, name):
    dims = (4, 4, 4, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 80, fermions=True)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, Action(beta=5.6, kappa=0.155, cg_tol=1e-14), name, 0.0, 3, U, P, dev(eta))
    assert np.array_equal(host(U), U0) and np.array_equal(host(P), P0)
    assert abs(dH) < 1e-8


def test_zero_noise_is_pure_gauge(ctx, orc):
    dims = (6, 4, 4, 6)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 81, fermions=True)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, Action(beta=5.6, kappa=0.155, cg_tol=1e-12), "FG", 1.0, 4, U, P,
                            dev(np.zeros_like(eta)))
    Uo, Po, dHo, _, _ = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 4, U0, P0)
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12 and abs(dH - dHo) < 1e-9
    assert st["cg_iters"] == 0


def test_fermions_without_gauge_action(ctx, orc):
    dims = (4, 4, 4, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 82, fermions=True)
    U, P = dev(U0), dev(P0)
    dH, _ = ctx.trajectory(dims, Action(beta=0.0, kappa=0.155, cg_tol=1e-14), "PQPQP", 1.0, 5, U, P, dev(eta))
    Uo, Po, dHo, _, _ = orc.trajectory(dims, 0.0, orc.table("PQPQP"), 1.0, 5, U0, P0, kappa=0.155, eta=eta)
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12 and abs(dH - dHo) < 1e-9


@pytest.mark.parametrize("name", ["PQP", "QPQ", "PQPQP", "CAMPOSTRINI", "FG"])
def test_smallest_lattice_with_fermions(ctx, orc, name):
    dims = (2, 2, 2, 2)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 83, fermions=True)
    U, P = dev(U0), dev(P0)
    dH, st = ctx.trajectory(dims, Action(beta=5.6, kappa=0.155, cg_tol=1e-14), name, 1.0, 4, U, P, dev(eta))
    Uo, Po, dHo, sto, _ = orc.trajectory(dims, 5.6, orc.table(name), 1.0, 4, U0, P0, kappa=0.155, eta=eta)
    assert relmax(host(U), Uo) < 1e-12 and relmax(host(P), Po) < 1e-12 and abs(dH - dHo) < 1e-9
    assert st["solves"] == sto["solves"]


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, -2, 4), (4, 5, 4, 4)])
def test_bad_geometry_rejected(ctx, dims):
    """The library's own check (called directly, past the binding's shape check)."""
    import ctypes
    U = dev(synth.hot_start((4, 4, 4, 4), 1, fermions=False)[0])
    S = ctypes.c_double(-1.0)
    rc = fgi.lib().fgi_gauge_action(ctx.h, fgi._geom(dims), 5.6, ctypes.c_void_p(U.data_ptr()), ctypes.byref(S),
                                    None)
    assert rc == fgi.FGI_EINVAL and S.value == -1.0


def test_bad_trajectory_arguments_leave_fields_untouched(ctx):
    dims = (4, 4, 4, 4)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 84, fermions=True)
    U, P = dev(U0), dev(P0)
    bad = [dict(act=Action(beta=5.6), tau=1.0, n=0),
           dict(act=Action(beta=5.6), tau=math.nan, n=2),
           dict(act=Action(beta=5.6, kappa=0.155, cg_tol=0.0), tau=1.0, n=2),
           dict(act=Action(beta=5.6, kappa=0.155, link_recon=8), tau=1.0, n=2),
           dict(act=Action(beta=5.6, kappa=0.155, kappa_hasen=0.16), tau=1.0, n=2)]
    for b in bad:
        with pytest.raises(fgi.FgiError) as e:
            ctx.trajectory(dims, b["act"], "FG", b["tau"], b["n"], U, P, dev(eta), dev(eta))
        assert e.value.code == fgi.FGI_EINVAL, b
        assert np.array_equal(host(U), U0) and np.array_equal(host(P), P0)


def test_missing_noise_rejected(ctx):
    dims = (4, 4, 4, 4)
    U0, P0, _, _ = synth.hot_start(dims, synth.SEED_BASE + 85, fermions=False)
    with pytest.raises(fgi.FgiError) as e:
        ctx.trajectory(dims, Action(beta=5.6, kappa=0.155), "FG", 1.0, 2, dev(U0), dev(P0), None)
    assert e.value.code == fgi.FGI_EINVAL
