"""Integrator tuning from measured Poisson brackets (Section 3).

To order dt^2 the Omelyan integrator PQPQP(alpha) conserves the shadow
Hamiltonian H + dt^2 [a(alpha) {S,{S,T}} + b(alpha) {T,{S,T}}] with the
Table 1 coefficients a = (6 alpha^2 - 6 alpha + 1) / 12, b = (1 - 6 alpha) / 24,
so over a trajectory dH = -dt^2 [a dSST + b dTST] + O(dt^4), where dSST, dTST
are the changes of the two brackets between its ends.  Given those changes
measured on an ensemble, the alpha that minimises the predicted <dH^2> is the
minimum of the quartic f(alpha) = mean((a dSST + b dTST)^2) on [0, 1/2];
the paper's conclusions name this tuning as the next step.
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
