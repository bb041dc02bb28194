"""ctypes wrapper of the FP64 CPU oracle (fgi_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The GPU library never imports it.

Array conventions (numpy, C order, lexicographic site i = x + Lx(y + Ly(z + Lz t))):
  U    complex128 (4, V, 3, 3)   links U_mu(x)
  P    float64    (4, V, 8)      momentum components p_a, P = sum p_a T^a, T^a = i lambda^a / 2
  eta, phi, X  complex128 (V/2, 4, 3)  even-site spinors, k-th even site in lexicographic order
  full spinors complex128 (V, 4, 3)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fgi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force=True):
    """Compile the oracle with gcc (plain C99 + OpenMP, -O2, no fast-math)."""
    cmd = ["gcc", "-std=gnu99", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB):
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_long)
_vp = ctypes.c_void_p
_d = ctypes.c_double
_i = ctypes.c_int


def _declare(L):
    L.oracle_threads.argtypes = []
    L.oracle_threads.restype = _i
    L.oracle_gauge_action.argtypes = [_ip, _d, _d, _vp]
    L.oracle_gauge_action.restype = _d
    L.oracle_plaquette.argtypes = [_ip, _vp]
    L.oracle_plaquette.restype = _d
    L.oracle_gauge_force.argtypes = [_ip, _d, _d, _vp, _vp]
    L.oracle_gauge_force_tangent.argtypes = [_ip, _d, _d, _vp, _vp, _vp]
    L.oracle_kinetic.argtypes = [_ip, _vp]
    L.oracle_kinetic.restype = _d
    L.oracle_exp_su3.argtypes = [_vp, _d, _vp]
    L.oracle_link_update.argtypes = [_ip, _d, _vp, _vp]
    L.oracle_reunitarize.argtypes = [_ip, _vp]
    L.oracle_gamma.argtypes = [_i, _vp]
    L.oracle_dhop.argtypes = [_ip, _vp, _vp, _vp]
    L.oracle_wilson.argtypes = [_ip, _d, _vp, _vp, _vp]
    L.oracle_mhat.argtypes = [_ip, _d, _vp, _vp, _vp, _i]
    L.oracle_cg.argtypes = [_ip, _d, _vp, _vp, _vp, _d, _i, _dp]
    L.oracle_cg.restype = _i
    L.oracle_pf_heatbath.argtypes = [_ip, _d, _vp, _vp, _vp]
    L.oracle_pf_action.argtypes = [_ip, _d, _vp, _vp, _d, _i, _ip]
    L.oracle_pf_action.restype = _d
    L.oracle_fermion_force_add.argtypes = [_ip, _d, _vp, _vp, _d, _vp]
    L.oracle_force.argtypes = [_ip, _d, _d, _i, _d, _i, _vp, _vp, _vp, _lp, _d, _d, _i, _d]
    L.oracle_force_tangent.argtypes = [_ip, _d, _d, _i, _d, _i, _vp, _vp, _vp, _vp, _lp, _d]
    L.oracle_fermion_force_tangent_add.argtypes = [_ip, _d, _vp, _vp, _vp, _d, _i, _d, _vp]
    L.oracle_fermion_force_tangent_add.restype = _i
    L.oracle_trajectory.argtypes = [_ip, _d, _d, _i, _d, _i, _i, _i, ctypes.c_char_p, _vp, _vp,
                                    _d, _i, _vp, _vp, _vp, _vp, _dp, _lp, _i, _d, _d, _i, _d]
    L.oracle_sigma.argtypes = [_i, _i, _vp]
    L.oracle_clover.argtypes = [_ip, _d, _d, _vp, _vp, _vp, _vp]
    L.oracle_clover.restype = _d
    L.oracle_clover_wilson.argtypes = [_ip, _d, _d, _vp, _vp, _vp]
    L.oracle_clover_mhat.argtypes = [_ip, _d, _d, _vp, _vp, _vp, _i]
    L.oracle_clover_pf_action.argtypes = [_ip, _d, _d, _vp, _vp, _d, _i, _ip]
    L.oracle_clover_pf_action.restype = _d
    L.oracle_clover_force_add.argtypes = [_ip, _d, _d, _vp, _vp, _d, _d, _vp]
    L.oracle_clover_cg.argtypes = [_ip, _d, _d, _vp, _vp, _vp, _d, _i]
    L.oracle_trajectory.restype = _i
    L.oracle_brackets.argtypes = [_ip, _d, _d, _i, _d, _i, _vp, _vp, _vp, _d, _dp, _dp, _d, _d, _i, _d]
    L.oracle_hasen_heatbath.argtypes = [_ip, _d, _d, _vp, _vp, _vp, _d, _i]
    L.oracle_hasen_heatbath.restype = _i
    L.oracle_hasen_action.argtypes = [_ip, _d, _d, _vp, _vp, _d, _i, _vp, _ip]
    L.oracle_hasen_action.restype = _d
    L.oracle_hasen_force_add.argtypes = [_ip, _d, _d, _vp, _vp, _vp, _d, _vp]
    L.oracle_hasen_force_tangent_add.argtypes = [_ip, _d, _d, _vp, _vp, _vp, _vp, _d, _i, _d, _vp]
    L.oracle_hasen_force_tangent_add.restype = _i
    L.oracle_trajectory_nested.argtypes = [_ip, _d, _d, _d, _d, _i, _i, _vp, _vp, _vp, ctypes.c_char_p, _vp, _vp,
                                           _d, _i, _vp, _vp, _vp, _vp, _dp, _lp, _i, _d, _d, _i, _i, _d]
    L.oracle_trajectory_nested.restype = _i
    L.oracle_philox.argtypes = [_vp, _vp, _vp]
    L.oracle_brackets4.argtypes = [_ip, _d, _d, _i, _d, _i, _vp, _vp, _vp, _d, _d, _vp]
    L.oracle_brackets4.restype = _i
    L.oracle_refresh.argtypes = [_ip, ctypes.c_uint64, ctypes.c_uint32, _vp, _vp, _vp]
    L.oracle_metropolis_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    L.oracle_metropolis_uniform.restype = _d
    L.oracle_hmc_run.argtypes = [_ip, _d, _d, _i, _d, _i, _i, _i, ctypes.c_char_p, _vp, _vp, _d, _i, _vp,
                                 ctypes.c_uint64, ctypes.c_uint32, _i, _i, _vp, _vp, _vp, _i, _d, _d, _i]
    L.oracle_cg_from.argtypes = [_ip, _d, _vp, _vp, _vp, _d, _i, _dp, _i]
    L.oracle_cg_from.restype = _i
    L.oracle_hmc_run.restype = _i
    L.oracle_stout_smear.argtypes = [_ip, _d, _i, _vp, _vp]
    L.oracle_stout_jvp.argtypes = [_ip, _d, _i, _vp, _vp, _vp]
    L.oracle_stout_vjp.argtypes = [_ip, _d, _i, _vp, _vp, _vp]


def _dims(dims):
    return (ctypes.c_int * 4)(*[int(d) for d in dims])


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads():
    return lib().oracle_threads()


def volume(dims):
    return int(np.prod(dims))


def gauge_action(dims, beta, U, c1=0.0):
    """S_G with plaquettes (weight c0 = 1 - 8 c1) and 2x1 rectangles (weight c1)"""
    U = _c(U, np.complex128)
    return lib().oracle_gauge_action(_dims(dims), beta, c1, _ptr(U))


def plaquette(dims, U):
    U = _c(U, np.complex128)
    return lib().oracle_plaquette(_dims(dims), _ptr(U))


def gauge_force(dims, beta, U, c1=0.0):
    U = _c(U, np.complex128)
    F = np.zeros((4, volume(dims), 8))
    lib().oracle_gauge_force(_dims(dims), beta, c1, _ptr(U), _ptr(F))
    return F


def gauge_force_tangent(dims, beta, U, Vdir, c1=0.0):
    """J_V[F_G] = d/dt F_G(exp(t V) U) at t = 0."""
    U = _c(U, np.complex128)
    Vdir = _c(Vdir, np.float64)
    J = np.zeros((4, volume(dims), 8))
    lib().oracle_gauge_force_tangent(_dims(dims), beta, c1, _ptr(U), _ptr(Vdir), _ptr(J))
    return J


def kinetic(dims, P):
    P = _c(P, np.float64)
    return lib().oracle_kinetic(_dims(dims), _ptr(P))


def exp_su3(p, h=1.0):
    p = _c(p, np.float64)
    out = np.zeros((3, 3), np.complex128)
    lib().oracle_exp_su3(_ptr(p), h, _ptr(out))
    return out


def link_update(dims, h, P, U):
    """returns exp(h P) U (U not modified)"""
    U = np.array(U, dtype=np.complex128, copy=True, order="C")
    P = _c(P, np.float64)
    lib().oracle_link_update(_dims(dims), h, _ptr(P), _ptr(U))
    return U


def reunitarize(dims, U):
    U = np.array(U, dtype=np.complex128, copy=True, order="C")
    lib().oracle_reunitarize(_dims(dims), _ptr(U))
    return U


def gamma(mu):
    out = np.zeros((4, 4), np.complex128)
    lib().oracle_gamma(mu, _ptr(out))
    return out


def dhop(dims, U, psi):
    U = _c(U, np.complex128)
    psi = _c(psi, np.complex128)
    out = np.zeros_like(psi)
    lib().oracle_dhop(_dims(dims), _ptr(U), _ptr(psi), _ptr(out))
    return out


def wilson(dims, kappa, U, psi):
    U = _c(U, np.complex128)
    psi = _c(psi, np.complex128)
    out = np.zeros_like(psi)
    lib().oracle_wilson(_dims(dims), kappa, _ptr(U), _ptr(psi), _ptr(out))
    return out


def mhat(dims, kappa, U, psi_e, dagger=False):
    U = _c(U, np.complex128)
    psi_e = _c(psi_e, np.complex128)
    out = np.zeros_like(psi_e)
    lib().oracle_mhat(_dims(dims), kappa, _ptr(U), _ptr(psi_e), _ptr(out), int(bool(dagger)))
    return out


def cg(dims, kappa, U, phi, tol=1e-14, maxiter=10000):
    """returns (X, iterations or -1, true relative residual)"""
    U = _c(U, np.complex128)
    phi = _c(phi, np.complex128)
    X = np.zeros_like(phi)
    rr = ctypes.c_double(0)
    it = lib().oracle_cg(_dims(dims), kappa, _ptr(U), _ptr(phi), _ptr(X), tol, maxiter,
                         ctypes.byref(rr))
    return X, it, rr.value


def pf_heatbath(dims, kappa, U, eta):
    U = _c(U, np.complex128)
    eta = _c(eta, np.complex128)
    phi = np.zeros_like(eta)
    lib().oracle_pf_heatbath(_dims(dims), kappa, _ptr(U), _ptr(eta), _ptr(phi))
    return phi


def pf_action(dims, kappa, U, phi, tol=1e-14, maxiter=10000):
    U = _c(U, np.complex128)
    phi = _c(phi, np.complex128)
    it = ctypes.c_int(0)
    s = lib().oracle_pf_action(_dims(dims), kappa, _ptr(U), _ptr(phi), tol, maxiter,
                               ctypes.byref(it))
    return s, it.value


def fermion_force(dims, kappa, U, Xe):
    U = _c(U, np.complex128)
    Xe = _c(Xe, np.complex128)
    F = np.zeros((4, volume(dims), 8))
    lib().oracle_fermion_force_add(_dims(dims), kappa, _ptr(U), _ptr(Xe), 1.0, _ptr(F))
    return F


def cg_from(dims, kappa, U, phi, x0, tol=1e-10, maxiter=10000):
    """CG started from x0; returns (X, iterations or -1, final relative residual)."""
    U = _c(U, np.complex128)
    phi = _c(phi, np.complex128)
    X = np.array(x0, dtype=np.complex128, copy=True, order="C")
    rel = ctypes.c_double(0)
    it = lib().oracle_cg_from(_dims(dims), kappa, _ptr(U), _ptr(phi), _ptr(X), tol, maxiter, ctypes.byref(rel), 1)
    return X, it, rel.value


def force(dims, beta, U, kappa=0.0, phi=None, tol=1e-14, maxiter=10000, c1=0.0, stout_rho=0.0, stout_n=0,
          csw=0.0):
    """total force F = F_G (+ F_F when phi is given, on stout_n levels of
    stout-smeared links, carried back to the thin links; with csw != 0 the
    clover operator and its -2 log det A_oo term); returns (F, stats)"""
    U = _c(U, np.complex128)
    F = np.zeros((4, volume(dims), 8))
    st = (ctypes.c_long * 3)()
    ferm = phi is not None
    phi_a = _c(phi, np.complex128) if ferm else None
    lib().oracle_force(_dims(dims), beta, kappa, int(ferm), tol, maxiter, _ptr(U),
                       _ptr(phi_a) if ferm else None, _ptr(F), st, c1, stout_rho, int(stout_n), csw)
    return F, dict(solves=st[0], cg_iters=st[1], cg_fail=st[2])


def force_tangent(dims, beta, U, V, kappa=0.0, phi=None, tol=1e-14, maxiter=10000, c1=0.0):
    """J_V[F] = d/dt F(exp(t V) U) at t = 0 for the total force (gauge, plus the
    pseudofermion force when phi is given); returns (J, stats)"""
    U = _c(U, np.complex128)
    V = _c(V, np.float64)
    J = np.zeros((4, volume(dims), 8))
    st = (ctypes.c_long * 3)()
    ferm = phi is not None
    phi_a = _c(phi, np.complex128) if ferm else None
    lib().oracle_force_tangent(_dims(dims), beta, kappa, int(ferm), tol, maxiter, _ptr(U),
                               _ptr(phi_a) if ferm else None, _ptr(V), _ptr(J), st, c1)
    return J, dict(solves=st[0], cg_iters=st[1], cg_fail=st[2])


def fermion_force_tangent(dims, kappa, U, X, V, tol=1e-14, maxiter=10000):
    """J_V[F_F] given X = (Mhat^+ Mhat)^-1 phi (one more solve inside)"""
    U = _c(U, np.complex128)
    X = _c(X, np.complex128)
    V = _c(V, np.float64)
    J = np.zeros((4, volume(dims), 8))
    lib().oracle_fermion_force_tangent_add(_dims(dims), kappa, _ptr(U), _ptr(X), _ptr(V), tol, maxiter, 1.0,
                                           _ptr(J))
    return J


def trajectory(dims, beta, stages, tau, nsteps, U, P, kappa=0.0, eta=None, tol=1e-14,
               maxiter=10000, fg_exact=False, phi=None, fg_start=True, c1=0.0, stout_rho=0.0, stout_n=0, csw=0.0):
    """One MD trajectory.  stages: list of (kind, w, xi) with kind in 'PQG'.
    Fermions: give eta (phi = Mhat^+ eta) or phi itself.  fg_start: the
    displaced force's solve of a G stage starts from the undisplaced solution.
    Returns (U_final, P_final, dH, stats, status)."""
    U = np.array(U, dtype=np.complex128, copy=True, order="C")
    P = np.array(P, dtype=np.float64, copy=True, order="C")
    kinds = "".join(s[0] for s in stages).encode()
    ws = np.array([s[1] for s in stages], np.float64)
    xis = np.array([s[2] if len(s) > 2 else 0.0 for s in stages], np.float64)
    ferm = eta is not None or phi is not None
    eta_a = _c(eta, np.complex128) if eta is not None else None
    phi_a = _c(phi, np.complex128) if phi is not None else None
    dH = ctypes.c_double(0)
    st = (ctypes.c_long * 3)()
    status = lib().oracle_trajectory(_dims(dims), beta, kappa, int(ferm), tol, maxiter,
                                     int(bool(fg_exact)), len(stages), kinds, _ptr(ws), _ptr(xis),
                                     tau, nsteps, _ptr(U), _ptr(P),
                                     _ptr(eta_a) if eta_a is not None else None,
                                     _ptr(phi_a) if phi_a is not None else None,
                                     ctypes.byref(dH), st, int(bool(fg_start)), c1, stout_rho, int(stout_n), csw)
    return U, P, dH.value, dict(solves=st[0], cg_iters=st[1], cg_fail=st[2]), status


def brackets(dims, beta, U, P, kappa=0.0, phi=None, h=1e-4, tol=1e-14, maxiter=10000, c1=0.0, stout_rho=0.0,
             stout_n=0, csw=0.0):
    """(SST, TST) = ({S,{S,T}}, {T,{S,T}}) at (U, P); TST by central difference."""
    U = _c(U, np.complex128)
    P = _c(P, np.float64)
    ferm = phi is not None
    phi_a = _c(phi, np.complex128) if ferm else None
    sst = ctypes.c_double(0)
    tst = ctypes.c_double(0)
    lib().oracle_brackets(_dims(dims), beta, kappa, int(ferm), tol, maxiter, _ptr(U), _ptr(P),
                          _ptr(phi_a) if ferm else None, h, ctypes.byref(sst), ctypes.byref(tst), c1, stout_rho,
                          int(stout_n), csw)
    return sst.value, tst.value


def brackets4(dims, beta, U, P, kappa=0.0, phi=None, h=1e-3, tol=1e-14, maxiter=10000, c1=0.0):
    """The dt^4 brackets of Table 1 at (U, P) (oracle_brackets4): dict with
    SST, TST and STSST = {{S,T},{S,{S,T}}}, STTST = {{S,T},{T,{S,T}}},
    TTSST = {T,{T,{S,{S,T}}}}, TTTST = {T,{T,{T,{S,T}}}}; the derivatives of
    the force gradient along P and F by central differences with step h."""
    U = _c(U, np.complex128)
    P = _c(P, np.float64)
    ferm = phi is not None
    phi_a = _c(phi, np.complex128) if ferm else None
    out = np.zeros(6)
    rc = lib().oracle_brackets4(_dims(dims), beta, kappa, int(ferm), tol, maxiter, _ptr(U), _ptr(P),
                                _ptr(phi_a) if ferm else None, h, c1, _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle_brackets4: a CG solve did not converge")
    return dict(zip(("SST", "TST", "STSST", "STTST", "TTSST", "TTTST"), out.tolist()))


def hasen_heatbath(dims, kappa, kappa2, U, eta2, tol=1e-14, maxiter=10000):
    """phi2 = Mhat2 (Mhat2^+ Mhat2)^-1 Mhat^+ eta2 (Mhat2 at kappa2)"""
    U = _c(U, np.complex128)
    eta2 = _c(eta2, np.complex128)
    phi2 = np.zeros_like(eta2)
    lib().oracle_hasen_heatbath(_dims(dims), kappa, kappa2, _ptr(U), _ptr(eta2), _ptr(phi2), tol, maxiter)
    return phi2


def hasen_action(dims, kappa, kappa2, U, phi2, tol=1e-14, maxiter=10000):
    """(S_2, X2) with S_2 = chi^+ (Mhat^+ Mhat)^-1 chi, chi = Mhat2^+ phi2"""
    U = _c(U, np.complex128)
    phi2 = _c(phi2, np.complex128)
    X2 = np.zeros_like(phi2)
    it = ctypes.c_int(0)
    s = lib().oracle_hasen_action(_dims(dims), kappa, kappa2, _ptr(U), _ptr(phi2), tol, maxiter, _ptr(X2),
                                  ctypes.byref(it))
    return s, X2


def hasen_force(dims, kappa, kappa2, U, phi2, X2):
    U = _c(U, np.complex128)
    F = np.zeros((4, volume(dims), 8))
    lib().oracle_hasen_force_add(_dims(dims), kappa, kappa2, _ptr(U), _ptr(_c(phi2, np.complex128)),
                                 _ptr(_c(X2, np.complex128)), 1.0, _ptr(F))
    return F


def hasen_force_tangent(dims, kappa, kappa2, U, phi2, X2, V, tol=1e-14, maxiter=10000):
    """J_V[F_2] = d/dt F_2(exp(tV) U) at t = 0 for the S_2 force, given X2 at U (one more solve)"""
    U = _c(U, np.complex128)
    J = np.zeros((4, volume(dims), 8))
    lib().oracle_hasen_force_tangent_add(_dims(dims), kappa, kappa2, _ptr(U), _ptr(_c(phi2, np.complex128)),
                                         _ptr(_c(X2, np.complex128)), _ptr(_c(V, np.float64)), tol, maxiter, 1.0,
                                         _ptr(J))
    return J


def trajectory_nested(dims, beta, levels, tau, nsteps, U, P, kappa=0.0, kappa2=0.0, eta1=None, eta2=None,
                      tol=1e-14, maxiter=10000, fg_start=True, c1=0.0, stout_rho=0.0, stout_n=0, fg_exact=False,
                      csw=0.0):
    """levels: list of (stages, terms, nsub), level 0 outermost; terms bit 1 gauge,
    2 S_F (or S_1 with Hasenbusch), 4 S_2.  Returns (U, P, dH, stats, status)."""
    U = np.array(U, dtype=np.complex128, copy=True, order="C")
    P = np.array(P, dtype=np.float64, copy=True, order="C")
    ns = np.array([len(l[0]) for l in levels], np.int32)
    terms = np.array([l[1] for l in levels], np.int32)
    nsub = np.array([l[2] for l in levels], np.int32)
    kinds = "".join(s[0] for l in levels for s in l[0]).encode()
    ws = np.array([s[1] for l in levels for s in l[0]], np.float64)
    xis = np.array([s[2] if len(s) > 2 else 0.0 for l in levels for s in l[0]], np.float64)
    dH = ctypes.c_double(0)
    st = (ctypes.c_long * 3)()
    e1 = _c(eta1, np.complex128) if eta1 is not None else None
    e2 = _c(eta2, np.complex128) if eta2 is not None else None
    status = lib().oracle_trajectory_nested(_dims(dims), beta, kappa, kappa2, tol, maxiter, len(levels), _ptr(ns),
                                            _ptr(terms), _ptr(nsub), kinds, _ptr(ws), _ptr(xis), tau, nsteps,
                                            _ptr(U), _ptr(P), _ptr(e1) if e1 is not None else None,
                                            _ptr(e2) if e2 is not None else None, ctypes.byref(dH), st,
                                            int(bool(fg_start)), c1, stout_rho, int(stout_n),
                                            int(bool(fg_exact)), csw)
    return U, P, dH.value, dict(solves=st[0], cg_iters=st[1], cg_fail=st[2]), status


# ---------------------------------------------------------------------------
# stout smearing (Morningstar and Peardon 2004)
# ---------------------------------------------------------------------------

def stout_smear(dims, rho, n, U):
    """n levels of U <- exp(TA(C U^+)) U, C = rho * (sum of the 6 staples)"""
    U = _c(U, np.complex128)
    out = np.empty_like(U)
    lib().oracle_stout_smear(_dims(dims), rho, n, _ptr(U), _ptr(out))
    return out


def stout_jvp(dims, rho, n, U, v):
    """tangent of the smearing: thin-link su(3) components v -> smeared-link components"""
    U = _c(U, np.complex128)
    v = _c(v, np.float64)
    out = np.zeros_like(v)
    lib().oracle_stout_jvp(_dims(dims), rho, n, _ptr(U), _ptr(v), _ptr(out))
    return out


def stout_vjp(dims, rho, n, U, g):
    """adjoint of stout_jvp: a force on the smeared links -> the force on the thin links"""
    U = _c(U, np.complex128)
    g = _c(g, np.float64)
    out = np.zeros_like(g)
    lib().oracle_stout_vjp(_dims(dims), rho, n, _ptr(U), _ptr(g), _ptr(out))
    return out


# ---------------------------------------------------------------------------
# Markov chain: Philox4x32-10 draws and the HMC accept/reject loop
# ---------------------------------------------------------------------------

def philox(ctr, key):
    """Philox4x32-10 of one counter (four uint32) under a key (two uint32)."""
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox(_ptr(c), _ptr(k), _ptr(o))
    return [int(x) for x in o]


def refresh(dims, seed, traj, momenta=True, eta1=True, eta2=False):
    """(P, eta1, eta2) drawn for trajectory traj of the chain `seed` (None where not asked)."""
    V = volume(dims)
    P = np.zeros((4, V, 8)) if momenta else None
    e1 = np.zeros((V // 2, 4, 3), np.complex128) if eta1 else None
    e2 = np.zeros((V // 2, 4, 3), np.complex128) if eta2 else None
    lib().oracle_refresh(_dims(dims), int(seed), int(traj), _ptr(P) if momenta else None,
                         _ptr(e1) if eta1 else None, _ptr(e2) if eta2 else None)
    return P, e1, e2


def metropolis_uniform(seed, traj):
    return lib().oracle_metropolis_uniform(int(seed), int(traj))


def hmc_run(dims, beta, stages, tau, nsteps, U, seed, traj0, ntraj, kappa=0.0, fermions=False, tol=1e-14,
            maxiter=10000, fg_exact=False, metropolis=True, fg_start=True, c1=0.0, stout_rho=0.0, stout_n=0):
    """HMC chain of ntraj trajectories from U; returns (U_final, dH list, accepted list, plaquettes, status)."""
    U = np.array(U, dtype=np.complex128, copy=True, order="C")
    kinds = "".join(s[0] for s in stages).encode()
    ws = np.array([s[1] for s in stages], np.float64)
    xis = np.array([s[2] if len(s) > 2 else 0.0 for s in stages], np.float64)
    n = max(int(ntraj), 1)
    dH = np.zeros(n)
    acc = np.zeros(n, np.int32)
    plaq = np.zeros(n)
    status = lib().oracle_hmc_run(_dims(dims), beta, kappa, int(bool(fermions)), tol, maxiter, int(bool(fg_exact)),
                                  len(stages), kinds, _ptr(ws), _ptr(xis), tau, nsteps, _ptr(U), int(seed),
                                  int(traj0), int(ntraj), int(bool(metropolis)), _ptr(dH), _ptr(acc), _ptr(plaq),
                                  int(bool(fg_start)), c1, stout_rho, int(stout_n))
    k = int(ntraj)
    return U, list(dH[:k]), [bool(a) for a in acc[:k]], list(plaq[:k]), status


# ---------------------------------------------------------------------------
# integrator tables (Table 1), written as step stage lists (kind, w, xi)
# ---------------------------------------------------------------------------

def table(name, alpha=0.1932):
    """Stage table of one step for the integrators of Table 1."""
    if name == "PQP":
        return [("P", 0.5, 0.0), ("Q", 1.0, 0.0), ("P", 0.5, 0.0)]
    if name == "QPQ":
        return [("Q", 0.5, 0.0), ("P", 1.0, 0.0), ("Q", 0.5, 0.0)]
    if name == "PQPQP":
        return [("P", alpha, 0.0), ("Q", 0.5, 0.0), ("P", 1.0 - 2.0 * alpha, 0.0),
                ("Q", 0.5, 0.0), ("P", alpha, 0.0)]
    if name == "FG":
        return [("P", 1.0 / 6.0, 0.0), ("Q", 0.5, 0.0), ("G", 2.0 / 3.0, 1.0 / 72.0),
                ("Q", 0.5, 0.0), ("P", 1.0 / 6.0, 0.0)]
    if name == "CAMPOSTRINI":
        c = 2.0 ** (1.0 / 3.0)
        w1 = 1.0 / (2.0 - c)
        w0 = -c / (2.0 - c)
        return [("Q", w1 / 2, 0.0), ("P", w1, 0.0), ("Q", (w1 + w0) / 2, 0.0), ("P", w0, 0.0),
                ("Q", (w1 + w0) / 2, 0.0), ("P", w1, 0.0), ("Q", w1 / 2, 0.0)]
    raise ValueError(name)


# ---- clover term -------------------------------------------------------


def sigma(mu, nu):
    """sigma_{mu nu} = (i/2)[g_mu, g_nu] (mu, nu = 0..3), 4x4"""
    out = np.zeros((4, 4), np.complex128)
    lib().oracle_sigma(mu, nu, _ptr(out))
    return out


def clover(dims, kappa, csw, U):
    """per-site clover matrices A(x), A(x)^-1 ([V, 12, 12], index spin*3 +
    colour), log det A(x) [V], and the action term -2 sum_{x odd} log det A(x)"""
    U = _c(U, np.complex128)
    V = volume(dims)
    A = np.zeros((V, 12, 12), np.complex128)
    Ai = np.zeros((V, 12, 12), np.complex128)
    ld = np.zeros(V)
    s = lib().oracle_clover(_dims(dims), kappa, csw, _ptr(U), _ptr(A), _ptr(Ai), _ptr(ld))
    return A, Ai, ld, s


def clover_wilson(dims, kappa, csw, U, psi):
    """full-lattice M psi = A psi - kappa D psi"""
    U = _c(U, np.complex128)
    psi = _c(psi, np.complex128)
    out = np.zeros_like(psi)
    lib().oracle_clover_wilson(_dims(dims), kappa, csw, _ptr(U), _ptr(psi), _ptr(out))
    return out


def clover_mhat(dims, kappa, csw, U, psi, dagger=False):
    """Mhat psi_e = A_ee psi_e - kappa^2 D_eo A_oo^-1 D_oe psi_e (or Mhat^+)"""
    U = _c(U, np.complex128)
    psi = _c(psi, np.complex128)
    out = np.zeros_like(psi)
    lib().oracle_clover_mhat(_dims(dims), kappa, csw, _ptr(U), _ptr(psi), _ptr(out), int(bool(dagger)))
    return out


def clover_pf_action(dims, kappa, csw, U, phi, tol=1e-14, maxiter=10000):
    """S_F = phi^+ (Mhat^+ Mhat)^-1 phi with the clover Mhat; (S_F, iterations)"""
    U = _c(U, np.complex128)
    phi = _c(phi, np.complex128)
    it = ctypes.c_int(0)
    s = lib().oracle_clover_pf_action(_dims(dims), kappa, csw, _ptr(U), _ptr(phi), tol, maxiter, ctypes.byref(it))
    return s, it.value


def clover_cg(dims, kappa, csw, U, phi, tol=1e-14, maxiter=10000):
    """X_e = (Mhat^+ Mhat)^-1 phi with the clover Mhat; (X_e, iterations)"""
    U = _c(U, np.complex128)
    phi = _c(phi, np.complex128)
    X = np.zeros_like(phi)
    it = lib().oracle_clover_cg(_dims(dims), kappa, csw, _ptr(U), _ptr(phi), _ptr(X), tol, maxiter)
    return X, it


def clover_force(dims, kappa, csw, U, Xe=None, pf_scale=1.0, det_scale=1.0):
    """the clover pseudofermion force for the solution Xe (hopping and clover
    parts, times pf_scale) plus the -2 log det A_oo force (times det_scale)"""
    U = _c(U, np.complex128)
    F = np.zeros((4, volume(dims), 8))
    xa = _c(Xe, np.complex128) if Xe is not None else None
    lib().oracle_clover_force_add(_dims(dims), kappa, csw, _ptr(U), _ptr(xa) if xa is not None else None,
                                  pf_scale if xa is not None else 0.0, det_scale, _ptr(F))
    return F
