"""Integrator tuning from measured Poisson brackets (Section 3).

To order dt^2 the Omelyan integrator PQPQP(alpha) conserves the shadow
Hamiltonian H + dt^2 [a(alpha) {S,{S,T}} + b(alpha) {T,{S,T}}] with the
Table 1 coefficients a = (6 alpha^2 - 6 alpha + 1) / 12, b = (1 - 6 alpha) / 24,
so over a trajectory dH = -dt^2 [a dSST + b dTST] + O(dt^4), where dSST, dTST
are the changes of the two brackets between its ends.  Given those changes
measured on an ensemble, the alpha that minimises the predicted <dH^2> is the
minimum of the quartic f(alpha) = mean((a dSST + b dTST)^2) on [0, 1/2];
the paper's conclusions name this tuning as the next step.

The same is done for a force-gradient family whose fourth-order shadow terms
are known in closed form (fg_family_*, below): with the four dt^4 brackets
measured as well, its two parameters are chosen to minimise the predicted
<dH^2> at the step size in use.
"""
import numpy as np


def pqpqp_dt2_coeffs(alpha):
    """(a, b): the dt^2 coefficients of {S,{S,T}} and {T,{S,T}} for PQPQP(alpha)."""
    return (6 * alpha ** 2 - 6 * alpha + 1) / 12, (1 - 6 * alpha) / 24


def predicted_dh2(alpha, dsst, dtst, dt=1.0):
    """dt^4 mean((a dSST + b dTST)^2) at this alpha (arrays of per-trajectory changes)."""
    a, b = pqpqp_dt2_coeffs(alpha)
    return dt ** 4 * float(np.mean((a * np.asarray(dsst) + b * np.asarray(dtst)) ** 2))


def tune_omelyan_alpha(dsst, dtst, lo=0.0, hi=0.5):
    """alpha in [lo, hi] minimising the predicted <dH^2> of PQPQP(alpha).

    f(alpha) = mean((a dS + b dT)^2) with a, b quadratic and linear in alpha is
    a quartic; its minimum is at a real root of f' in the interval or at an end."""
    dS, dT = np.asarray(dsst, float), np.asarray(dtst, float)
    if dS.shape != dT.shape or dS.size == 0:
        raise ValueError("need equal, non-empty arrays of bracket changes")
    # a dS + b dT = c2 alpha^2 + c1 alpha + c0 per sample
    c2 = dS / 2.0
    c1 = -dS / 2.0 - dT / 4.0
    c0 = dS / 12.0 + dT / 24.0
    # f = mean of the squared quadratic: coefficients of alpha^4 .. alpha^0
    f = np.array([np.mean(c2 * c2), np.mean(2 * c2 * c1), np.mean(c1 * c1 + 2 * c2 * c0),
                  np.mean(2 * c1 * c0), np.mean(c0 * c0)])
    cand = [lo, hi] + [r.real for r in np.roots(np.polyder(f)) if abs(r.imag) < 1e-12 and lo <= r.real <= hi]
    return float(min(cand, key=lambda x: np.polyval(f, x)))


# ---------------------------------------------------------------------------
# The force-gradient family P(lam) Q(1/2) G(1 - 2 lam, xi) Q(1/2) P(lam) with
# the exact G stage (p += w dt F + 2 xi dt^3 J_F[F]); (1/6, 1/72) is Table 1's
# FG integrator, (alpha, 0) is PQPQP(alpha).  Its shadow Hamiltonian to dt^4,
# from the BCH series to fifth order (derived and checked by bch.py):
#   H~ = H + dt^2 sum_k c2_k B_k + dt^4 sum_k c4_k B_k,
# so over a trajectory dH = -dt^2 sum c2_k dB_k - dt^4 sum c4_k dB_k + O(dt^6).
# The dt^4 brackets {S,{S,{S,{S,T}}}} and {T,{S,{S,{S,T}}}} vanish for T
# quadratic in p and are left out.
FG_KEYS2 = ("SST", "TST")
FG_KEYS4 = ("STSST", "STTST", "TTSST", "TTTST")


def fg_family_stages(lam, xi):
    """One step of the family as a stage table (kind, w, xi)."""
    return [("P", lam, 0.0), ("Q", 0.5, 0.0), ("G", 1.0 - 2.0 * lam, xi), ("Q", 0.5, 0.0), ("P", lam, 0.0)]


def fg_family_coeffs(lam, xi):
    """(c2, c4): the dt^2 and dt^4 shadow-Hamiltonian coefficients of the family."""
    c2 = {"SST": lam ** 2 / 2 - lam / 2 - xi + 1.0 / 12, "TST": 1.0 / 24 - lam / 4}
    c4 = {"STSST": lam ** 3 / 8 - 7 * lam ** 2 / 48 - lam * xi / 2 + lam / 16 + xi / 6 - 1.0 / 120,
          "STTST": -lam ** 2 / 24 + lam / 48 - 1.0 / 360,
          "TTSST": lam / 48 + xi / 24 - 7.0 / 1440,
          "TTTST": lam / 192 - 7.0 / 5760}
    return c2, c4


def predicted_dh_fg_family(lam, xi, dB, dt):
    """Per-trajectory dH predicted to O(dt^6) from the bracket changes dB (a dict
    of arrays, end minus start, for FG_KEYS2 + FG_KEYS4)."""
    c2, c4 = fg_family_coeffs(lam, xi)
    s2 = sum(c2[k] * np.asarray(dB[k], float) for k in FG_KEYS2)
    s4 = sum(c4[k] * np.asarray(dB[k], float) for k in FG_KEYS4)
    return -(dt ** 2) * s2 - (dt ** 4) * s4


def tune_fg_family(dB, dt, lam_range=(0.12, 0.22), xi_range=(0.0, 0.03), grid=121):
    """(lam, xi) in the given ranges minimising the predicted <dH^2> at step dt.

    The prediction is linear in xi and cubic in lam per trajectory, so the
    objective is a polynomial; it is minimised on a grid and refined by
    successive finer grids around the best point (no derivative needed).  The
    expansion describes dH only where its leading terms dominate: tune at a
    step where the FG integrator's measured dH follows its dt^4 row."""
    for k in FG_KEYS2 + FG_KEYS4:
        if np.asarray(dB[k]).size == 0:
            raise ValueError("need bracket changes of at least one trajectory")
    lo_l, hi_l = lam_range
    lo_x, hi_x = xi_range
    best = None
    for _ in range(4):
        ls = np.linspace(lo_l, hi_l, grid)
        xs = np.linspace(lo_x, hi_x, grid)
        for lam in ls:
            vals = [float(np.mean(predicted_dh_fg_family(lam, xi, dB, dt) ** 2)) for xi in xs]
            j = int(np.argmin(vals))
            if best is None or vals[j] < best[0]:
                best = (vals[j], float(lam), float(xs[j]))
        dl, dx = (hi_l - lo_l) / (grid - 1), (hi_x - lo_x) / (grid - 1)
        lo_l, hi_l = max(lam_range[0], best[1] - 2 * dl), min(lam_range[1], best[1] + 2 * dl)
        lo_x, hi_x = max(xi_range[0], best[2] - 2 * dx), min(xi_range[1], best[2] + 2 * dx)
    return best[1], best[2]
