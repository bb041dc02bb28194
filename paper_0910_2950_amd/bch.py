"""Shadow Hamiltonians of symmetric splitting integrators, derived by the
Baker-Campbell-Hausdorff series to fifth order (Section 3).

One step of an integrator is a product of exponentials of the two flows: the
P step exp(w dt X) (the S-hat flow, p += w dt F) and the Q step exp(w dt Y)
(the T-hat flow, U <- exp(w dt P) U), and the force-gradient stage
G(w, xi) = exp(w dt X - xi dt^3 [X,[X,Y]]) (p += w dt F + 2 xi dt^3 J_F[F]).
The logarithm of the product, computed here in the free associative algebra
over {X, Y} truncated at words of length five (each letter carries one power
of dt), is dt (X + Y) + dt^3 L3 + dt^5 L5 for a symmetric step; writing L3 and
L5 in the nested commutators that correspond to the Poisson brackets,

  H~ = H + dt^2 (c_SST {S,{S,T}} + c_TST {T,{S,T}})
         + dt^4 (c_SSSST {S,{S,{S,{S,T}}}} + c_TSSST {T,{S,{S,{S,T}}}}
                 + c_STSST {{S,T},{S,{S,T}}} + c_STTST {{S,T},{T,{S,T}}}
                 + c_TTSST {T,{T,{S,{S,T}}}} + c_TTTST {T,{T,{T,{S,T}}}}) + O(dt^6),

with the bracket of two functions taken as the commutator of their flows.
This module needs sympy and is used to derive and check the closed forms in
tuning.py; it reproduces Table 1's rows (the dt^2 coefficients of PQPQP(alpha)
and the dt^4 rows of the force-gradient and Campostrini integrators).
"""
import sympy as sp

MAXLEN = 5
ONE = {(): sp.Integer(1)}
X = {("X",): sp.Integer(1)}
Y = {("Y",): sp.Integer(1)}


def _mul(a, b):
    out = {}
    for wa, ca in a.items():
        for wb, cb in b.items():
            if len(wa) + len(wb) <= MAXLEN:
                out[wa + wb] = out.get(wa + wb, 0) + ca * cb
    return out


def _add(a, b, s=1):
    out = dict(a)
    for w, c in b.items():
        out[w] = out.get(w, 0) + s * c
    return out


def _scale(a, s):
    return {w: s * c for w, c in a.items()}


def _exp(z):
    out, term = dict(ONE), dict(ONE)
    for k in range(1, MAXLEN + 1):
        term = _scale(_mul(term, z), sp.Rational(1, k))
        out = _add(out, term)
    return out


def _log(g):
    m = _add(g, ONE, -1)
    out, term = {}, dict(ONE)
    for k in range(1, MAXLEN + 1):
        term = _mul(term, m)
        out = _add(out, _scale(term, sp.Rational((-1) ** (k + 1), k)))
    out = {w: sp.cancel(c) for w, c in out.items()}  # weights may be rational functions of a parameter
    return {w: c for w, c in out.items() if c != 0}


def comm(a, b):
    return _add(_mul(a, b), _mul(b, a), -1)


_XY = comm(X, Y)
BASIS3 = {"SST": comm(X, _XY), "TST": comm(Y, _XY)}
BASIS5 = {"SSSST": comm(X, comm(X, BASIS3["SST"])), "TSSST": comm(Y, comm(X, BASIS3["SST"])),
          "STSST": comm(_XY, BASIS3["SST"]), "STTST": comm(_XY, BASIS3["TST"]),
          "TTSST": comm(Y, comm(Y, BASIS3["SST"])), "TTTST": comm(Y, comm(Y, BASIS3["TST"]))}


def _coords(z, basis, length):
    names = list(basis)
    cs = sp.symbols("c0:%d" % len(names))
    words = {w for b in basis.values() for w in b} | {w for w in z if len(w) == length}
    sol = sp.solve([sum(c * basis[n].get(w, 0) for c, n in zip(cs, names)) - z.get(w, 0) for w in words],
                   cs, dict=True)
    if len(sol) != 1:
        raise ValueError("not a Lie element of the expected degree")
    return {n: sp.cancel(sol[0][c]) for c, n in zip(cs, names)}


def shadow_coefficients(stages):
    """stages: list of (kind, w, xi) with kind in 'PQG' (sympy or Python numbers);
    returns (c2, c4): the dt^2 and dt^4 coefficient dicts of H~ - H."""
    g = dict(ONE)
    for kind, w, xi in stages:
        if kind == "P":
            z = _scale(X, w)
        elif kind == "Q":
            z = _scale(Y, w)
        elif kind == "G":
            z = _add(_scale(X, w), _scale(BASIS3["SST"], -xi))
        else:
            raise ValueError(kind)
        g = _mul(g, _exp(z))
    L = _log(g)
    if any(len(w) % 2 == 0 for w in L):
        raise ValueError("the step is not symmetric")
    if {w: c for w, c in L.items() if len(w) == 1} != {("X",): 1, ("Y",): 1}:
        raise ValueError("the weights of the P and of the Q stages must each sum to one")
    return (_coords({w: c for w, c in L.items() if len(w) == 3}, BASIS3, 3),
            _coords({w: c for w, c in L.items() if len(w) == 5}, BASIS5, 5))
