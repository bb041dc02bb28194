"""Pins of the oracle's Markov chain (no GPU): the counter-based draws have
the distributions HMC needs (unit Gaussian momenta, noise with Re, Im ~
N(0, 1/2), uniform Metropolis draws) and are independent across counters and
streams; the chain obeys the Creutz identity <exp(-dH)> = 1 in equilibrium
(which needs a reversible, area-preserving integrator and the right
Metropolis rule); a resumed chain repeats an uninterrupted one bitwise."""
import numpy as np
import pytest
import scipy.stats

from paper_0910_2950_amd import synth
from oracle.oracle import table

L8 = (8, 8, 8, 8)


def test_momenta_are_unit_gaussian(orc):
    P, _, _ = orc.refresh(L8, seed=11, traj=0, eta1=False)
    x = P.ravel()
    n = x.size
    assert abs(x.mean()) < 5 / np.sqrt(n)
    assert abs(x.var() - 1) < 5 * np.sqrt(2 / n)
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-4
    # every component and direction on its own
    for a in range(8):
        assert abs(P[..., a].var() - 1) < 6 * np.sqrt(2 / P[..., a].size)


def test_noise_has_half_variance_per_real_part(orc):
    _, e1, e2 = orc.refresh(L8, seed=12, traj=3, momenta=False, eta1=True, eta2=True)
    for e in (e1, e2):
        z = np.concatenate([e.real.ravel(), e.imag.ravel()])
        assert abs(z.var() - 0.5) < 5 * 0.5 * np.sqrt(2 / z.size)
        assert scipy.stats.kstest(z * np.sqrt(2), "norm").pvalue > 1e-4


def test_streams_and_trajectories_are_independent(orc):
    P0, e1, e2 = orc.refresh(L8, seed=13, traj=7, eta2=True)
    P1, f1, _ = orc.refresh(L8, seed=13, traj=8)
    Q0, _, _ = orc.refresh(L8, seed=14, traj=7, eta1=False)
    lim = lambda n: 5 / np.sqrt(n)
    pairs = [(P0.ravel(), P1.ravel()), (P0.ravel(), Q0.ravel()), (e1.real.ravel(), e2.real.ravel()),
             (e1.real.ravel(), f1.real.ravel()), (e1.real.ravel(), e1.imag.ravel()),
             (P0[..., 0].ravel(), P0[..., 1].ravel()), (P0[..., 1].ravel(), P0[..., 2].ravel())]
    for a, b in pairs:
        assert abs(np.corrcoef(a, b)[0, 1]) < lim(a.size)


def test_metropolis_uniforms(orc):
    u = np.array([orc.metropolis_uniform(99, t) for t in range(4000)])
    assert u.min() > 0 and u.max() < 1
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-4


def test_philox_avalanche(orc):
    """Flipping one counter or key bit flips about half of the 128 output bits."""
    g = np.random.default_rng(5)
    flips = []
    for _ in range(64):
        c = [int(x) for x in g.integers(0, 2 ** 32, 4)]
        k = [int(x) for x in g.integers(0, 2 ** 32, 2)]
        base = orc.philox(c, k)
        for w in range(6):
            for bit in (0, 13, 31):
                c2, k2 = list(c), list(k)
                if w < 4:
                    c2[w] ^= 1 << bit
                else:
                    k2[w - 4] ^= 1 << bit
                out = orc.philox(c2, k2)
                flips.append(sum(bin(a ^ b).count("1") for a, b in zip(base, out)))
    flips = np.array(flips)
    assert abs(flips.mean() - 64) < 1.5 and flips.min() > 30


def test_chain_resume_is_bitwise(orc):
    dims = (4, 4, 2, 2)
    U0, _, _, _ = synth.hot_start(dims, synth.SEED_BASE + 60, fermions=False)
    args = dict(kappa=0.155, fermions=True, tol=1e-12)
    Ua, dHa, acca, _, _ = orc.hmc_run(dims, 5.6, table("FG"), 0.5, 3, U0, 77, 0, 4, **args)
    Ub, dHb, accb, _, _ = orc.hmc_run(dims, 5.6, table("FG"), 0.5, 3, U0, 77, 0, 2, **args)
    Ub, dHc, accc, _, _ = orc.hmc_run(dims, 5.6, table("FG"), 0.5, 3, Ub, 77, 2, 2, **args)
    assert np.array_equal(Ua, Ub) and dHa == dHb + dHc and acca == accb + accc


def test_chain_without_metropolis_accepts_all(orc):
    dims = (2, 2, 2, 2)
    U0, _, _, _ = synth.hot_start(dims, synth.SEED_BASE + 61, fermions=False)
    _, dH, acc, _, _ = orc.hmc_run(dims, 6.0, table("PQP"), 1.0, 2, U0, 5, 0, 6, metropolis=False)
    assert all(acc) and max(abs(d) for d in dH) > 1e-3


def test_creutz_identity_on_an_equilibrated_chain(orc):
    """<exp(-dH)> = 1 over an equilibrium chain (pure gauge 2^4, beta 6, a coarse
    PQPQP step so that dH is O(1)); the Metropolis acceptance is the mean of
    min(1, exp(-dH))."""
    dims = (2, 2, 2, 2)
    U0, _, _, _ = synth.hot_start(dims, synth.SEED_BASE + 62, fermions=False)
    st = table("PQPQP")
    U, _, _, _, _ = orc.hmc_run(dims, 6.0, st, 1.0, 2, U0, 31, 0, 300)
    _, dH, acc, _, _ = orc.hmc_run(dims, 6.0, st, 1.0, 2, U, 31, 300, 3000)
    w = np.exp(-np.array(dH))
    err = w.std() / np.sqrt(w.size)
    assert abs(w.mean() - 1) < 4 * err, (w.mean(), err)
    assert 0.05 < np.mean(acc) < 0.95
    pacc = np.mean(np.minimum(1, w))
    assert abs(np.mean(acc) - pacc) < 4 * np.sqrt(pacc * (1 - pacc) / w.size)
    # the same chain without the accept/reject step leaves equilibrium and the
    # identity fails (measured 1.157 +- 0.018)
    _, dH2, _, _, _ = orc.hmc_run(dims, 6.0, st, 1.0, 2, U, 31, 300, 3000, metropolis=False)
    w2 = np.exp(-np.array(dH2))
    assert abs(w2.mean() - 1) > 4 * w2.std() / np.sqrt(w2.size)
