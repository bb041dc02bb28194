"""The host-side logic of bench.py (CPU): the step counts it reads from the
committed calibration, its per-leg statistics, and the two-fold
cross-validation of its bracket-tuning legs, driven by a stand-in context that
returns designed bracket changes and records what each trajectory was run with.
"""
import math
import types

import numpy as np
import pytest

import bench
from paper_0910_2950_amd import fgi, tuning


def test_n_star_follows_the_rule():
    """n* = the smallest swept n from which every swept point has <dH^2> at or
    below the target, for every leg of the committed calibration."""
    import json
    with open(bench.CALIBRATION_FILE) as fh:
        cal = json.load(fh)
    target = cal["target_dH2"]
    assert target == pytest.approx(0.257)
    for leg, v in cal["legs"].items():
        pts = sorted(v["points"], key=lambda p: p["n"])
        ok = [p["n"] for i, p in enumerate(pts) if all(q["mean_dH2"] <= target for q in pts[i:])]
        assert v["n_star"] == min(ok), leg
        if leg in bench.LEGS:
            assert bench.n_star(leg) == (min(ok), "calibration")
    assert {k: bench.n_star(k)[0] for k in bench.LEGS} == {"fg_mp16": 16, "fg_mp32": 16, "fg_fp64": 16,
                                                          "pqpqp_fp64": 22, "lf_fp64": 80}


def test_summarise():
    dh = [0.3, -0.2, 1.5, 0.05]
    recs = [dict(dH=d, solves=50, cg_iters=1000 + k, cg_iters_max=40, max_rel_resid=1e-11, reliable_updates=3,
                 force_evals=49) for k, d in enumerate(dh)]
    s = bench.summarise(recs)
    x = np.array(dh)
    assert s["trajectories"] == 4
    assert s["mean_dH2"] == pytest.approx(np.mean(x ** 2))
    assert s["mean_dH2_err"] == pytest.approx(np.std(x ** 2, ddof=1) / 2)
    assert s["acceptance"] == pytest.approx(np.mean(np.minimum(1, np.exp(-x))))
    assert s["exp_minus_dH"] == pytest.approx(np.mean(np.exp(-x)))
    assert s["cg_iters_per_traj"] == pytest.approx(1001.5)


class Field:
    """A stand-in device tensor: clone() gives a new object carrying the same tag."""

    def __init__(self, tag):
        self.tag = tag

    def clone(self):
        return Field(self.tag)


class FakeCtx:
    """Brackets are zero at every start measurement and take designed values
    at the k-th end measurement; trajectories move the links to a new tag,
    return dH = -0.01 (always accepted) and log what they were run with."""

    def __init__(self, ends):
        self.ends = ends
        self.calls = 0
        self.runs = []

    def pf_heatbath(self, dims, act, U, eta):
        return Field(("phi", U.tag))

    def _bracket(self):   # the legs measure start, end, start, end, ...
        c, self.calls = self.calls, self.calls + 1
        return None if c % 2 == 0 else self.ends[c // 2]

    def poisson_brackets(self, dims, act, U, P, phi, h=1e-4):
        b = self._bracket()
        return (0.0, 0.0) if b is None else (b["SST"], b["TST"])

    def poisson_brackets4(self, dims, act, U, P, phi, h=1e-3):
        b = self._bracket()
        return {k: 0.0 for k in tuning.FG_KEYS2 + tuning.FG_KEYS4} if b is None else dict(b)

    def trajectory(self, dims, act, integ, tau, n, U, P, *a, **k):
        self.runs.append((U.tag, integ))
        U.tag = ("end", len(self.runs) - 1)
        return -0.01, {}

    def reunitarize(self, dims, U):
        pass


def fake_runner(ctx, k):
    starts = [(Field(("P", i)), Field(("eta", i))) for i in range(2 * k)]
    R = types.SimpleNamespace(ctx=ctx, dims=(4, 4, 4, 4), fgi=fgi,
                              args=types.SimpleNamespace(seed=1, prec="mp16", recon=18),
                              fresh_inputs=lambda n, base: starts[:n],
                              action=lambda p, r: fgi.Action(beta=5.6, kappa=0.155))
    return R


def test_alpha_leg_cross_validates(monkeypatch):
    """alpha is fitted on each half from that half's brackets only and run on
    the other half's starts, along the chain's links."""
    monkeypatch.setattr(bench, "log", lambda *a: None)
    monkeypatch.setattr(fgi, "integrator_builtin", lambda name, alpha=0.1932: ("PQPQP", alpha))
    k = 3
    # half 0: only {T,{S,T}} changes (best alpha 1/6); half 1: only {S,{S,T}} (the root of a(alpha))
    ends = [dict(SST=0.0, TST=1.0 + i) if i < k else dict(SST=1.0 + i, TST=0.0) for i in range(2 * k)]
    ctx = FakeCtx(ends)
    out = bench.tune_alpha_leg(fake_runner(ctx, k), Field(("start", None)), k, 44)
    a0, a1 = out["alpha_folds"]
    assert a0 == pytest.approx(1 / 6, abs=1e-9)
    assert a1 == pytest.approx((3 - math.sqrt(3)) / 6, abs=1e-9)
    # the first 2k runs measure at 0.1932 along the chain, the next 2k are the held-out reruns
    measure, cv = ctx.runs[:2 * k], ctx.runs[2 * k:]
    assert all(integ == ("PQPQP", 0.1932) for _, integ in measure)
    assert [integ[1] for _, integ in cv] == [a0] * k + [a1] * k   # half 1 run at half 0's alpha, then back
    # each held-out rerun starts from the links its measured trajectory started from
    assert [tag for tag, _ in cv] == [measure[i][0] for i in list(range(k, 2 * k)) + list(range(k))]
    assert out["chain_accepted"] == [True] * (2 * k)
    assert len(out["dH"]["cross_validated"]) == 2 * k


def test_family_leg_cross_validates(monkeypatch):
    """The family member is fitted on each half and run on the other; with
    only the dt^2 brackets changing, every fit is the fourth-order point."""
    monkeypatch.setattr(bench, "log", lambda *a: None)
    captured = []

    def from_levels(levels):
        captured.append(levels[0][0])
        return ("member", len(captured) - 1)
    monkeypatch.setattr(fgi, "integrator_from_levels", from_levels)
    k = 3
    rng = np.random.default_rng(3)
    ends = [dict({kk: float(rng.normal()) for kk in tuning.FG_KEYS2}, **{kk: 0.0 for kk in tuning.FG_KEYS4})
            for _ in range(2 * k)]
    ctx = FakeCtx(ends)
    act = fgi.Action(beta=5.6, kappa=0.155)
    out = bench.fg_family_leg(fake_runner(ctx, k), Field(("start", None)), act, 32, k)
    for lam, xi in out["fold_fits"] + [(out["lam"], out["xi"])]:
        assert lam == pytest.approx(1 / 6, abs=1e-3) and xi == pytest.approx(1 / 72, abs=1e-4)
    # the first member built is FG itself; the held-out reruns use the fold members
    assert captured[0] == tuning.fg_family_stages(1 / 6, 1 / 72)
    measure, cv = ctx.runs[:2 * k], ctx.runs[2 * k:]
    assert all(integ == ("member", 0) for _, integ in measure)
    assert [integ for _, integ in cv] == [("member", 1)] * k + [("member", 2)] * k
    assert [tag for tag, _ in cv] == [measure[i][0] for i in list(range(k, 2 * k)) + list(range(k))]
    assert len(out["dH"]["cross_validated_predicted"]) == 2 * k


def test_ensemble_leg_batches_the_headline_starts(monkeypatch):
    """K chains built from the headline's first K timed starts on clones of the
    thermalised links, one untimed batched call before the timed ones, and
    each chain's dH compared with the single run of its start."""
    monkeypatch.setattr(bench, "log", lambda *a: None)
    calls = []

    class Ctx:
        def trajectory_batched(self, chains, act, integ, tau, n):
            calls.append([(c["dims"], c["beta"], c["kappa"], c["U"].tag, c["P"].tag, c["eta"].tag) for c in chains])
            return [0.01 * i for i in range(len(chains))], {}

    requested = []

    def fresh_inputs(n, base):
        requested.append((n, base))
        return [(Field(("P", base + i)), Field(("eta", base + i))) for i in range(n)]
    R = types.SimpleNamespace(ctx=Ctx(), dims=(4, 4, 4, 8), fgi=fgi, fresh_inputs=fresh_inputs,
                              torch=types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None)),
                              args=types.SimpleNamespace(seed=10, warmup=1, beta=5.6, kappa=0.1575, tol=1e-10))
    act = fgi.Action(beta=5.6, kappa=0.1575, prec="mp16", link_recon=18)
    out = bench.ensemble_leg(R, Field("Utherm"), act, 16, [2, 3], [0.0, 0.01, 0.5], steps=2)
    assert requested == [(2, 100011), (3, 100011)]        # the headline's timed starts begin at seed + 100000 + warmup
    assert [len(c) for c in calls] == [2, 2, 2, 3, 3, 3]   # per K: one untimed call, then two timed
    for chains in calls:
        assert [c[3] for c in chains] == ["Utherm"] * len(chains)
        assert [(c[4], c[5]) for c in chains] == [(("P", 100011 + i), ("eta", 100011 + i)) for i in range(len(chains))]
        assert all(c[:3] == ((4, 4, 4, 8), 5.6, 0.1575) for c in chains)
    assert out["chains"]["2"]["max_abs_dH_diff_vs_single"] == 0.0
    assert out["chains"]["3"]["max_abs_dH_diff_vs_single"] == pytest.approx(0.48)
    assert out["timed"] == 2
