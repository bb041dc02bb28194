"""The 8^4 Nf = 2 step-size sweep on the GPU (Figure 1's dH against dtau):
beta = 5.6, kappa = 0.155, even-odd Wilson fermions, tau = 1, one trajectory
per integrator (leapfrog PQP, Omelyan PQPQP(0.1932), FG) and step count
n in {5, 7, 10, 14, 20, 28, 40}, from the seeded Haar start.

  - FP64 (CG 1e-14): dH at every point against the oracle's
    (tests/golden/config2_dH_sweep.json, written by make_config2_sweep.py
    from the oracle alone), 1e-9 absolute plus 1e-11 relative;
  - FP64, MP32 and MP16 (CG 1e-10 with FP64 reliable updates): the slope of
    log |dH| against log dtau over n >= 10 is 2 +- 0.3 for PQP and PQPQP and
    4 +- 0.3 for FG (the paper's n = 2 and n = 4);
  - mixed precision statistically: over 24 fresh (P, eta) draws at FG n = 10
    the MP32 and MP16 <dH^2> and acceptance lie within 2 sigma of FP64's, and
    each trajectory's dH agrees with FP64's to the solver tolerance."""
import json
import os

import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth
from paper_0910_2950_amd.fgi import Action

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "config2_dH_sweep.json")))
DIMS = tuple(GOLD["dims"])
NS = GOLD["ns"]
SLOPE = {"PQP": 2.0, "PQPQP": 2.0, "FG": 4.0}


@pytest.fixture(scope="module")
def ctx():
    c = fgi.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def start():
    return synth.hot_start(DIMS, GOLD["seed"], fermions=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def sweep(ctx, start, name, act):
    U0, P0, eta, _ = start
    out = []
    for n in NS:
        U, P = dev(U0), dev(P0)
        dH, _ = ctx.trajectory(DIMS, act, name, 1.0, n, U, P, dev(eta))
        out.append(dH)
    return np.array(out)


def slope(dh):
    k = [i for i, n in enumerate(NS) if n >= 10]
    x = np.log(1.0 / np.array(NS)[k])
    return np.polyfit(x, np.log(np.abs(dh[k])), 1)[0]


@pytest.mark.parametrize("name", ["PQP", "PQPQP", "FG"])
def test_sweep_fp64_matches_oracle(ctx, start, name):
    act = Action(beta=GOLD["beta"], kappa=GOLD["kappa"], cg_tol=GOLD["tol"])
    dh = sweep(ctx, start, name, act)
    ref = np.array(GOLD["dH"][name])
    print(name, "dH", dh.tolist(), flush=True)
    assert np.all(np.abs(dh - ref) <= 1e-9 + 1e-11 * np.abs(ref)), np.abs(dh - ref).max()
    assert abs(slope(dh) - SLOPE[name]) < 0.3


@pytest.mark.parametrize("prec", ["fp64", "mp32", "mp16"])
@pytest.mark.parametrize("name", ["PQP", "PQPQP", "FG"])
def test_sweep_slopes(ctx, start, name, prec):
    act = Action(beta=GOLD["beta"], kappa=GOLD["kappa"], cg_tol=1e-10, prec=prec,
                 link_recon=12 if prec == "mp16" else 18)
    dh = sweep(ctx, start, name, act)
    q = slope(dh)
    print(name, prec, "slope %.3f" % q, flush=True)
    assert abs(q - SLOPE[name]) < 0.3
    # the solver tolerance, not the precision, sets the distance to the oracle's dH
    ref = np.array(GOLD["dH"][name])
    assert np.all(np.abs(dh - ref) <= 1e-4 + 1e-6 * np.abs(ref))


def test_mixed_precision_statistics(ctx, start):
    U0, _, _, _ = start
    draws = [synth.refresh(DIMS, synth.SEED_BASE + 5000 + k) for k in range(24)]
    res = {}
    for prec in ("fp64", "mp32", "mp16"):
        act = Action(beta=GOLD["beta"], kappa=GOLD["kappa"], cg_tol=1e-10, prec=prec,
                     link_recon=12 if prec == "mp16" else 18)
        dh = []
        for P0, eta in draws:
            U, P = dev(U0), dev(P0)
            d, _ = ctx.trajectory(DIMS, act, "FG", 1.0, 10, U, P, dev(eta))
            dh.append(d)
        res[prec] = np.array(dh)
    d64 = res["fp64"]
    m2, s2 = np.mean(d64 ** 2), np.std(d64 ** 2) / np.sqrt(len(d64))
    acc = np.minimum(1.0, np.exp(-d64))
    ma, sa = acc.mean(), max(acc.std() / np.sqrt(len(acc)), 1e-12)
    for prec in ("mp32", "mp16"):
        d = res[prec]
        print(prec, "<dH^2> %.6e vs %.6e +- %.1e" % (np.mean(d ** 2), m2, s2), flush=True)
        assert abs(np.mean(d ** 2) - m2) <= 2 * s2
        assert abs(np.minimum(1.0, np.exp(-d)).mean() - ma) <= 2 * sa
        assert np.max(np.abs(d - d64)) < 1e-4
