"""Python binding of libfgi.so (include/fgi.h): argument marshalling only.

Every C entry point fgi_<name> is exposed as Context.<name> (or a module
function for the context-free ones) with the same arguments, taking torch
tensors that already live on the GPU.  All arithmetic happens in the HIP
library; if libfgi.so is missing this module raises instead of falling back.

Tensor layouts (C-contiguous, on the context's device):
  U    complex128 (4, V, 3, 3)    links, site i = x + Lx(y + Ly(z + Lz t))
  P    float64    (4, V, 8)       momentum / force components
  even/odd fields complex128 (V/2, 4, 3)
"""
import ctypes
import os
from dataclasses import dataclass

import torch  # noqa: F401  (loads the HIP runtime torch uses before libfgi)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfgi.so")

FGI_OK, FGI_EINVAL, FGI_EHIP, FGI_ENOCONV, FGI_ENONFINITE = 0, -1, -2, -3, -4
PREC = {"fp64": 0, "mp32": 1, "mp16": 2}
INTEGRATORS = {"PQP": 0, "QPQ": 1, "PQPQP": 2, "CAMPOSTRINI": 3, "FG": 4}
TERM_GAUGE, TERM_FERMION, TERM_HASEN = 1, 2, 4
MAX_STAGES, MAX_LEVELS = 16, 4


class FgiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fgi error %d: %s" % (code, msg))
        self.code = code


class fgi_geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4)]


class fgi_action(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("kappa", ctypes.c_double), ("kappa_hasen", ctypes.c_double),
                ("cg_tol", ctypes.c_double), ("cg_maxiter", ctypes.c_int), ("prec", ctypes.c_int),
                ("link_recon", ctypes.c_int), ("fg_exact", ctypes.c_int), ("c1", ctypes.c_double),
                ("stout_rho", ctypes.c_double), ("stout_n", ctypes.c_int), ("pad", ctypes.c_int),
                ("cg_tol_md", ctypes.c_double), ("csw", ctypes.c_double)]


class fgi_stage(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("pad", ctypes.c_int), ("w", ctypes.c_double), ("xi", ctypes.c_double)]


class fgi_level(ctypes.Structure):
    _fields_ = [("nstages", ctypes.c_int), ("terms", ctypes.c_int), ("nsub", ctypes.c_int), ("pad", ctypes.c_int),
                ("st", fgi_stage * MAX_STAGES)]


class fgi_integrator(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int), ("pad", ctypes.c_int), ("lev", fgi_level * MAX_LEVELS)]


class fgi_chain(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("pad", ctypes.c_int), ("beta", ctypes.c_double),
                ("kappa", ctypes.c_double), ("U", ctypes.c_void_p), ("P", ctypes.c_void_p),
                ("eta", ctypes.c_void_p)]


class fgi_tuning(ctypes.Structure):
    _fields_ = [("dslash_block", ctypes.c_int), ("xcd_order", ctypes.c_int), ("cg_batch", ctypes.c_int),
                ("cg_form", ctypes.c_int), ("sched_us_per_iter", ctypes.c_double * 6),
                ("batch_ms_per_solve", ctypes.c_double * 5), ("form_ms_per_solve", ctypes.c_double * 2)]

    def as_dict(self):
        return dict(dslash_block=self.dslash_block, xcd_order=self.xcd_order, cg_batch=self.cg_batch,
                    cg_form=self.cg_form, sched_us_per_iter=list(self.sched_us_per_iter),
                    batch_ms_per_solve=list(self.batch_ms_per_solve), form_ms_per_solve=list(self.form_ms_per_solve))


class fgi_halo_timing(ctypes.Structure):
    _fields_ = [("pack_us", ctypes.c_double), ("interior_us", ctypes.c_double), ("faces_us", ctypes.c_double),
                ("all_us", ctypes.c_double), ("local_us", ctypes.c_double), ("face_sites", ctypes.c_long),
                ("halo_bytes", ctypes.c_long)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def philox4x32_10(ctr, key):
    """The library's Philox4x32-10 of one counter (host)."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (ctypes.c_uint32 * 4)()
    _check(lib().fgi_philox4x32_10(c, k, o))
    return [int(x) for x in o]


class fgi_stats(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_long), ("cg_iters", ctypes.c_long), ("cg_iters_max", ctypes.c_int),
                ("reliable_updates", ctypes.c_int), ("max_rel_resid", ctypes.c_double),
                ("force_evals", ctypes.c_long), ("seconds", ctypes.c_double), ("graph_captures", ctypes.c_long)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp, _d, _i = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
_P = ctypes.POINTER

SIGNATURES = {
    "fgi_create": (_i, [_P(_vp), _i]),
    "fgi_destroy": (_i, [_vp]),
    "fgi_last_error": (ctypes.c_char_p, []),
    "fgi_set_option": (_i, [_vp, ctypes.c_char_p, _d]),
    "fgi_get_profile": (_i, [_vp, _P(_d), _P(ctypes.c_long), _P(ctypes.c_long)]),
    "fgi_gauge_action": (_i, [_vp, _P(fgi_geom), _d, _vp, _P(_d), _vp]),
    "fgi_improved_gauge_action": (_i, [_vp, _P(fgi_geom), _d, _d, _vp, _P(_d), _vp]),
    "fgi_improved_gauge_hvp": (_i, [_vp, _P(fgi_geom), _d, _d, _vp, _vp, _vp, _vp]),
    "fgi_stout_smear": (_i, [_vp, _P(fgi_geom), _d, _i, _vp, _vp, _vp]),
    "fgi_stout_force": (_i, [_vp, _P(fgi_geom), _d, _i, _vp, _vp, _vp, _vp]),
    "fgi_clover_field": (_i, [_vp, _P(fgi_geom), _d, _d, _vp, _vp, _P(_d), _vp, _vp]),
    "fgi_kinetic": (_i, [_vp, _P(fgi_geom), _vp, _P(_d), _vp]),
    "fgi_gauge_force": (_i, [_vp, _P(fgi_geom), _d, _vp, _vp, _vp]),
    "fgi_force_gradient": (_i, [_vp, _P(fgi_geom), _d, _vp, _vp, _vp, _vp]),
    "fgi_gauge_hvp": (_i, [_vp, _P(fgi_geom), _d, _vp, _vp, _vp, _vp]),
    "fgi_hasen_heatbath": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _P(fgi_stats), _vp]),
    "fgi_hasen_action": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _P(_d), _P(fgi_stats), _vp]),
    "fgi_force_terms": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _i, _vp, _P(fgi_stats), _vp]),
    "fgi_force": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _P(fgi_stats), _vp]),
    "fgi_fermion_force": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _vp]),
    "fgi_total_force_gradient": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _vp, _P(fgi_stats), _vp]),
    "fgi_dslash": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _i, _i, _vp]),
    "fgi_mhat": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _i, _vp]),
    "fgi_mhat_packed_noalloc": (_i, [_vp, _P(fgi_geom), ctypes.c_double, _vp, _vp, _vp, _i, _vp]),
    "fgi_halo_bytes": (_i, [_P(fgi_geom), _i, _P(ctypes.c_size_t)]),
    "fgi_halo_pack": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _i, _d, _d, _vp, _vp, _i, _vp]),
    "fgi_dslash_halo": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _i, _vp, _vp, _i, _i, _vp]),
    "fgi_halo_time": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _i, _P(fgi_halo_timing), _vp]),
    "fgi_cg_solve": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _P(fgi_stats), _vp]),
    "fgi_pf_heatbath": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _vp]),
    "fgi_pf_action": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _P(_d), _P(fgi_stats), _vp]),
    "fgi_poisson_brackets": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _d, _P(_d), _P(_d),
                                  _P(fgi_stats), _vp]),
    "fgi_poisson_brackets4": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _vp, _d, _P(_d), _P(fgi_stats),
                                   _vp]),
    "fgi_integrator_builtin": (_i, [_i, _d, _P(fgi_integrator)]),
    "fgi_trajectory": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _P(fgi_integrator), _d, _i, _vp, _vp, _vp, _vp,
                            _i, _P(_d), _P(fgi_stats), _vp]),
    "fgi_refresh": (_i, [_vp, _P(fgi_geom), ctypes.c_uint64, ctypes.c_uint64, _vp, _vp, _vp, _vp]),
    "fgi_field_bytes": (_i, [_P(fgi_geom), _i, _P(ctypes.c_size_t)]),
    "fgi_field_pack": (_i, [_vp, _P(fgi_geom), _i, _vp, _vp, _vp]),
    "fgi_field_unpack": (_i, [_vp, _P(fgi_geom), _i, _vp, _vp, _vp]),
    "fgi_trajectory_packed": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _P(fgi_integrator), _d, _i, _vp, _vp, _vp,
                                   _vp, _i, _P(_d), _P(fgi_stats), _vp]),
    "fgi_philox4x32_10": (_i, [_P(ctypes.c_uint32), _P(ctypes.c_uint32), _P(ctypes.c_uint32)]),
    "fgi_hmc_run": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _P(fgi_integrator), _d, _i, _vp, ctypes.c_uint64,
                         ctypes.c_uint64, _i, _i, _P(_d), _P(_i), _P(_d), _P(fgi_stats), _vp]),
    "fgi_trajectory_batched": (_i, [_vp, _i, _vp, _P(fgi_action), _P(fgi_integrator), _d, _i, _P(_d),
                                    _P(fgi_stats), _vp]),
    "fgi_autotune_cg": (_i, [_vp, _P(fgi_geom), _P(fgi_action), _vp, _vp, _P(fgi_tuning), _vp]),
    "fgi_autotune_batched": (_i, [_vp, _i, _vp, _P(fgi_action), _P(fgi_tuning), _vp]),
    "fgi_link_update": (_i, [_vp, _P(fgi_geom), _d, _vp, _vp, _vp]),
    "fgi_reunitarize": (_i, [_vp, _P(fgi_geom), _vp, _vp]),
    "fgi_exp_su3": (_i, [_vp, _i, _vp, _d, _vp, _vp]),
}


def lib():
    """Load libfgi.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FgiError(FGI_EINVAL, "libfgi.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, allow=()):
    if rc != FGI_OK and rc not in allow:
        raise FgiError(rc, lib().fgi_last_error().decode())
    return rc


def _geom(dims):
    return fgi_geom((ctypes.c_int * 4)(*[int(d) for d in dims]))


@dataclass
class Action:
    beta: float
    kappa: float = 0.0
    kappa_hasen: float = 0.0
    cg_tol: float = 1e-10
    cg_maxiter: int = 20000
    prec: str = "fp64"
    link_recon: int = 18
    fg_exact: bool = False
    c1: float = 0.0      # rectangle coefficient of the gauge action (0: Wilson)
    stout_rho: float = 0.0
    stout_n: int = 0     # stout levels of the links the fermion operator sees (0: thin links)
    cg_tol_md: float = 0.0   # tolerance of the solves inside force evaluations (0: cg_tol)
    csw: float = 0.0     # clover coefficient of the fermion matrix (0: Wilson; prec fp64 or mp32)

    def c(self):
        return fgi_action(self.beta, self.kappa, self.kappa_hasen, self.cg_tol, int(self.cg_maxiter),
                          PREC[self.prec], int(self.link_recon), int(bool(self.fg_exact)), float(self.c1),
                          float(self.stout_rho), int(self.stout_n), 0, float(self.cg_tol_md), float(self.csw))


def integrator_builtin(which, alpha=0.1932):
    out = fgi_integrator()
    _check(lib().fgi_integrator_builtin(INTEGRATORS[which] if isinstance(which, str) else int(which),
                                        float(alpha), ctypes.byref(out)))
    return out


def integrator_from_levels(levels):
    """levels: list of (stages, terms, nsub), stages a list of (kind, w, xi); level 0 outermost."""
    I = fgi_integrator()
    I.nlevels = len(levels)
    for l, (stages, terms, nsub) in enumerate(levels):
        L = I.lev[l]
        L.nstages = len(stages)
        L.terms = terms
        L.nsub = nsub
        for k, s in enumerate(stages):
            L.st[k].kind = ord(s[0])
            L.st[k].w = s[1]
            L.st[k].xi = s[2] if len(s) > 2 else 0.0
    return I


def _ptr(t, dtype, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise FgiError(FGI_EINVAL, "%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise FgiError(FGI_EINVAL, "%s must have dtype %s" % (name, dtype))
    if not t.is_contiguous():
        raise FgiError(FGI_EINVAL, "%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise FgiError(FGI_EINVAL, "%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _vol(dims):
    v = 1
    for d in dims:
        v *= int(d)
    return v


class Context:
    """One fgi_ctx on a HIP device (owns the library's scratch memory)."""

    def __init__(self, device=0):
        self.device = device
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            _check(lib().fgi_create(ctypes.byref(h), int(device)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().fgi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- options / profile
    def set_option(self, name, value):
        _check(lib().fgi_set_option(self.h, name.encode(), float(value)))

    def get_profile(self):
        ms, n, s = ctypes.c_double(), ctypes.c_long(), ctypes.c_long()
        _check(lib().fgi_get_profile(self.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(s)))
        return ms.value, n.value, s.value

    # ---- shapes
    @staticmethod
    def _shapes(dims):
        V = _vol(dims)
        return (4, V, 3, 3), (4, V, 8), (V // 2, 4, 3)

    # ---- Hamiltonian
    def gauge_action(self, dims, beta, U):
        su, _, _ = self._shapes(dims)
        S = ctypes.c_double()
        _check(lib().fgi_gauge_action(self.h, _geom(dims), beta, _ptr(U, torch.complex128, su, "U"),
                                      ctypes.byref(S), _stream()))
        return S.value

    def improved_gauge_action(self, dims, beta, c1, U):
        su, _, _ = self._shapes(dims)
        S = ctypes.c_double()
        _check(lib().fgi_improved_gauge_action(self.h, _geom(dims), beta, c1, _ptr(U, torch.complex128, su, "U"),
                                               ctypes.byref(S), _stream()))
        return S.value

    def stout_smear(self, dims, rho, n, U, Us=None):
        su, _, _ = self._shapes(dims)
        Us = torch.empty(su, dtype=torch.complex128, device=U.device) if Us is None else Us
        _check(lib().fgi_stout_smear(self.h, _geom(dims), rho, int(n), _ptr(U, torch.complex128, su, "U"),
                                     _ptr(Us, torch.complex128, su, "Us"), _stream()))
        return Us

    def stout_force(self, dims, rho, n, U, Fs, F=None):
        su, sp, _ = self._shapes(dims)
        F = torch.empty(sp, dtype=torch.float64, device=U.device) if F is None else F
        _check(lib().fgi_stout_force(self.h, _geom(dims), rho, int(n), _ptr(U, torch.complex128, su, "U"),
                                     _ptr(Fs, torch.float64, sp, "Fs"), _ptr(F, torch.float64, sp, "F"), _stream()))
        return F

    def clover_field(self, dims, kappa, csw, U, A=True, F_det=True):
        """(A [V,12,12] complex or None, S_det = -2 sum_{x odd} log det A(x), F_det or None)"""
        su, sp, _ = self._shapes(dims)
        V = dims[0] * dims[1] * dims[2] * dims[3]
        Aout = torch.empty((V, 12, 12), dtype=torch.complex128, device=U.device) if A else None
        Fout = torch.empty(sp, dtype=torch.float64, device=U.device) if F_det else None
        S = ctypes.c_double()
        _check(lib().fgi_clover_field(self.h, _geom(dims), kappa, csw, _ptr(U, torch.complex128, su, "U"),
                                      _ptr(Aout, torch.complex128, (V, 12, 12), "A") if A else None,
                                      ctypes.byref(S), _ptr(Fout, torch.float64, sp, "F_det") if F_det else None,
                                      _stream()))
        return Aout, S.value, Fout

    def kinetic(self, dims, P):
        _, sp, _ = self._shapes(dims)
        T = ctypes.c_double()
        _check(lib().fgi_kinetic(self.h, _geom(dims), _ptr(P, torch.float64, sp, "P"), ctypes.byref(T), _stream()))
        return T.value

    # ---- forces
    def gauge_force(self, dims, beta, U, F=None):
        su, sp, _ = self._shapes(dims)
        F = torch.empty(sp, dtype=torch.float64, device=U.device) if F is None else F
        _check(lib().fgi_gauge_force(self.h, _geom(dims), beta, _ptr(U, torch.complex128, su, "U"),
                                     _ptr(F, torch.float64, sp, "F"), _stream()))
        return F

    def force_gradient(self, dims, beta, U, V, J=None):
        su, sp, _ = self._shapes(dims)
        J = torch.empty(sp, dtype=torch.float64, device=U.device) if J is None else J
        _check(lib().fgi_force_gradient(self.h, _geom(dims), beta, _ptr(U, torch.complex128, su, "U"),
                                        _ptr(V, torch.float64, sp, "V"), _ptr(J, torch.float64, sp, "J"),
                                        _stream()))
        return J

    def gauge_hvp(self, dims, beta, U, V, HV=None):
        su, sp, _ = self._shapes(dims)
        HV = torch.empty(sp, dtype=torch.float64, device=U.device) if HV is None else HV
        _check(lib().fgi_gauge_hvp(self.h, _geom(dims), beta, _ptr(U, torch.complex128, su, "U"),
                                   _ptr(V, torch.float64, sp, "V"), _ptr(HV, torch.float64, sp, "HV"), _stream()))
        return HV

    def improved_gauge_hvp(self, dims, beta, c1, U, V, HV=None):
        su, sp, _ = self._shapes(dims)
        HV = torch.empty(sp, dtype=torch.float64, device=U.device) if HV is None else HV
        _check(lib().fgi_improved_gauge_hvp(self.h, _geom(dims), beta, c1, _ptr(U, torch.complex128, su, "U"),
                                            _ptr(V, torch.float64, sp, "V"), _ptr(HV, torch.float64, sp, "HV"),
                                            _stream()))
        return HV

    def force(self, dims, act, U, phi=None, F=None, allow_noconv=False):
        su, sp, se = self._shapes(dims)
        F = torch.empty(sp, dtype=torch.float64, device=U.device) if F is None else F
        st = fgi_stats()
        _check(lib().fgi_force(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                               _ptr(phi, torch.complex128, se, "phi"), _ptr(F, torch.float64, sp, "F"),
                               ctypes.byref(st), _stream()), (FGI_ENOCONV,) if allow_noconv else ())
        return F, st.as_dict()

    def total_force_gradient(self, dims, act, U, phi=None, V=None, J=None, allow_noconv=False):
        """J = d/dt F(exp(t V) U) at t = 0 for the total force; V None: V = F(U)"""
        su, sp, se = self._shapes(dims)
        J = torch.empty(sp, dtype=torch.float64, device=U.device) if J is None else J
        st = fgi_stats()
        _check(lib().fgi_total_force_gradient(self.h, _geom(dims), ctypes.byref(act.c()),
                                              _ptr(U, torch.complex128, su, "U"), _ptr(phi, torch.complex128, se, "phi"),
                                              _ptr(V, torch.float64, sp, "V"), _ptr(J, torch.float64, sp, "J"),
                                              ctypes.byref(st), _stream()), (FGI_ENOCONV,) if allow_noconv else ())
        return J, st.as_dict()

    def hasen_heatbath(self, dims, act, U, eta2):
        su, _, se = self._shapes(dims)
        phi2 = torch.empty(se, dtype=torch.complex128, device=U.device)
        st = fgi_stats()
        _check(lib().fgi_hasen_heatbath(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                        _ptr(eta2, torch.complex128, se, "eta2"), _ptr(phi2, torch.complex128, se, "phi2"),
                                        ctypes.byref(st), _stream()))
        return phi2

    def hasen_action(self, dims, act, U, phi2):
        su, _, se = self._shapes(dims)
        S = ctypes.c_double()
        st = fgi_stats()
        _check(lib().fgi_hasen_action(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                      _ptr(phi2, torch.complex128, se, "phi2"), ctypes.byref(S), ctypes.byref(st),
                                      _stream()))
        return S.value

    def force_terms(self, dims, act, U, phi1, phi2, terms):
        su, sp, se = self._shapes(dims)
        F = torch.empty(sp, dtype=torch.float64, device=U.device)
        st = fgi_stats()
        _check(lib().fgi_force_terms(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                     _ptr(phi1, torch.complex128, se, "phi1"), _ptr(phi2, torch.complex128, se, "phi2"),
                                     int(terms), _ptr(F, torch.float64, sp, "F"), ctypes.byref(st), _stream()))
        return F, st.as_dict()

    def fermion_force(self, dims, act, U, X, F=None):
        su, sp, se = self._shapes(dims)
        F = torch.empty(sp, dtype=torch.float64, device=U.device) if F is None else F
        _check(lib().fgi_fermion_force(self.h, _geom(dims), ctypes.byref(act.c()),
                                       _ptr(U, torch.complex128, su, "U"), _ptr(X, torch.complex128, se, "X"),
                                       _ptr(F, torch.float64, sp, "F"), _stream()))
        return F

    # ---- Wilson operator / solver
    def dslash(self, dims, act, U, inp, out_parity, prec="fp64", out=None):
        su, _, se = self._shapes(dims)
        out = torch.empty(se, dtype=torch.complex128, device=U.device) if out is None else out
        _check(lib().fgi_dslash(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                _ptr(inp, torch.complex128, se, "in"), _ptr(out, torch.complex128, se, "out"),
                                int(out_parity), PREC[prec], _stream()))
        return out

    # t-decomposed hopping term (one GPU's share of a lattice split in t)
    def halo_bytes(self, dims, prec="fp64"):
        n = ctypes.c_size_t()
        _check(lib().fgi_halo_bytes(_geom(dims), PREC[prec], ctypes.byref(n)))
        return n.value

    def _halo_buf(self, t, n, name):
        if t.dtype != torch.uint8 or t.numel() != n or not t.is_contiguous():
            raise FgiError(FGI_EINVAL, "%s: halo buffer of the wrong size, dtype or stride" % name)
        return ctypes.c_void_p(t.data_ptr())

    def halo_pack(self, dims, act, U, inp, in_parity, sign_lo, sign_hi, to_lo, to_hi, prec="fp64"):
        su, _, se = self._shapes(dims)
        n = self.halo_bytes(dims, prec)
        _check(lib().fgi_halo_pack(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                   _ptr(inp, torch.complex128, se, "in"), int(in_parity), float(sign_lo),
                                   float(sign_hi), self._halo_buf(to_lo, n, "to_lo"), self._halo_buf(to_hi, n, "to_hi"),
                                   PREC[prec], _stream()))

    def dslash_halo(self, dims, act, U, inp, out_parity, from_lo, from_hi, split=True, prec="fp64", out=None):
        su, _, se = self._shapes(dims)
        n = self.halo_bytes(dims, prec)
        out = torch.empty(se, dtype=torch.complex128, device=U.device) if out is None else out
        _check(lib().fgi_dslash_halo(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                     _ptr(inp, torch.complex128, se, "in"), _ptr(out, torch.complex128, se, "out"),
                                     int(out_parity), self._halo_buf(from_lo, n, "from_lo"),
                                     self._halo_buf(from_hi, n, "from_hi"), int(bool(split)), PREC[prec], _stream()))
        return out

    def halo_time(self, dims, act, U, inp, reps=50):
        su, _, se = self._shapes(dims)
        t = fgi_halo_timing()
        _check(lib().fgi_halo_time(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                   _ptr(inp, torch.complex128, se, "in"), int(reps), ctypes.byref(t), _stream()))
        return t.as_dict()

    def mhat(self, dims, act, U, inp, dagger=False, out=None):
        su, _, se = self._shapes(dims)
        out = torch.empty(se, dtype=torch.complex128, device=U.device) if out is None else out
        _check(lib().fgi_mhat(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                              _ptr(inp, torch.complex128, se, "in"), _ptr(out, torch.complex128, se, "out"),
                              int(bool(dagger)), _stream()))
        return out

    def mhat_packed_noalloc(self, dims, kappa, U, inp, out, dagger=False):
        """fgi_mhat_packed_noalloc: Mhat (or Mhat^+) on packed fields (uint8
        device buffers from field_pack), writing the caller's out buffer; the
        library allocates nothing."""
        nl, ne = self.field_bytes(dims, "links"), self.field_bytes(dims, "even")
        for t, n, name in ((U, nl, "U"), (inp, ne, "in"), (out, ne, "out")):
            if t.dtype != torch.uint8 or t.numel() != n or not t.is_contiguous():
                raise FgiError(FGI_EINVAL, "%s: packed buffer of the wrong size, dtype or stride" % name)
        _check(lib().fgi_mhat_packed_noalloc(self.h, _geom(dims), float(kappa), ctypes.c_void_p(U.data_ptr()),
                                             ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                             int(bool(dagger)), _stream()))
        return out

    def cg_solve(self, dims, act, U, phi, X=None, allow_noconv=False):
        su, _, se = self._shapes(dims)
        X = torch.empty(se, dtype=torch.complex128, device=U.device) if X is None else X
        st = fgi_stats()
        rc = _check(lib().fgi_cg_solve(self.h, _geom(dims), ctypes.byref(act.c()),
                                       _ptr(U, torch.complex128, su, "U"), _ptr(phi, torch.complex128, se, "phi"),
                                       _ptr(X, torch.complex128, se, "X"), ctypes.byref(st), _stream()),
                    (FGI_ENOCONV,) if allow_noconv else ())
        d = st.as_dict()
        d["status"] = rc
        return X, d

    def pf_heatbath(self, dims, act, U, eta, phi=None):
        su, _, se = self._shapes(dims)
        phi = torch.empty(se, dtype=torch.complex128, device=U.device) if phi is None else phi
        _check(lib().fgi_pf_heatbath(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                     _ptr(eta, torch.complex128, se, "eta"), _ptr(phi, torch.complex128, se, "phi"),
                                     _stream()))
        return phi

    def pf_action(self, dims, act, U, phi):
        su, _, se = self._shapes(dims)
        S = ctypes.c_double()
        st = fgi_stats()
        _check(lib().fgi_pf_action(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                   _ptr(phi, torch.complex128, se, "phi"), ctypes.byref(S), ctypes.byref(st),
                                   _stream()))
        return S.value, st.as_dict()

    def poisson_brackets(self, dims, act, U, P, phi=None, h=1e-4):
        su, sp, se = self._shapes(dims)
        a, b = ctypes.c_double(), ctypes.c_double()
        st = fgi_stats()
        _check(lib().fgi_poisson_brackets(self.h, _geom(dims), ctypes.byref(act.c()),
                                          _ptr(U, torch.complex128, su, "U"), _ptr(P, torch.float64, sp, "P"),
                                          _ptr(phi, torch.complex128, se, "phi"), h, ctypes.byref(a),
                                          ctypes.byref(b), ctypes.byref(st), _stream()))
        return a.value, b.value

    BRACKETS4 = ("SST", "TST", "STSST", "STTST", "TTSST", "TTTST")

    def poisson_brackets4(self, dims, act, U, P, phi=None, h=1e-3):
        """fgi_poisson_brackets4: dict of SST, TST and the four dt^4 brackets of Table 1."""
        su, sp, se = self._shapes(dims)
        out = (ctypes.c_double * 6)()
        st = fgi_stats()
        _check(lib().fgi_poisson_brackets4(self.h, _geom(dims), ctypes.byref(act.c()),
                                           _ptr(U, torch.complex128, su, "U"), _ptr(P, torch.float64, sp, "P"),
                                           _ptr(phi, torch.complex128, se, "phi"), h, out, ctypes.byref(st),
                                           _stream()))
        return dict(zip(self.BRACKETS4, list(out)))

    # ---- trajectory
    def trajectory(self, dims, act, integ, tau, nsteps, U, P, eta1=None, eta2=None, pf_is_phi=False,
                   allow_noconv=False):
        """Updates U, P in place; returns (dH, stats)."""
        su, sp, se = self._shapes(dims)
        if isinstance(integ, str):
            integ = integrator_builtin(integ)
        dH = ctypes.c_double()
        st = fgi_stats()
        rc = _check(lib().fgi_trajectory(self.h, _geom(dims), ctypes.byref(act.c()), ctypes.byref(integ),
                                         float(tau), int(nsteps), _ptr(U, torch.complex128, su, "U"),
                                         _ptr(P, torch.float64, sp, "P"), _ptr(eta1, torch.complex128, se, "eta1"),
                                         _ptr(eta2, torch.complex128, se, "eta2"), int(bool(pf_is_phi)),
                                         ctypes.byref(dH), ctypes.byref(st), _stream()),
                    (FGI_ENOCONV,) if allow_noconv else ())
        d = st.as_dict()
        d["status"] = rc
        return dH.value, d

    # ---- internal layouts
    FIELD_KINDS = {"links": 0, "momenta": 1, "even": 2}

    def field_bytes(self, dims, kind):
        n = ctypes.c_size_t()
        _check(lib().fgi_field_bytes(_geom(dims), self.FIELD_KINDS[kind], ctypes.byref(n)))
        return n.value

    def _user_spec(self, dims, kind):
        su, sp, se = self._shapes(dims)
        return {"links": (su, torch.complex128), "momenta": (sp, torch.float64), "even": (se, torch.complex128)}[kind]

    def field_pack(self, dims, kind, user):
        """The internal layout of a user-layout field (a uint8 device buffer)."""
        shape, dtype = self._user_spec(dims, kind)
        out = torch.empty(self.field_bytes(dims, kind), dtype=torch.uint8, device=user.device)
        _check(lib().fgi_field_pack(self.h, _geom(dims), self.FIELD_KINDS[kind], _ptr(user, dtype, shape, kind),
                                    ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def field_unpack(self, dims, kind, internal):
        shape, dtype = self._user_spec(dims, kind)
        if internal.numel() != self.field_bytes(dims, kind) or internal.dtype != torch.uint8:
            raise FgiError(FGI_EINVAL, "internal buffer of the wrong size or dtype")
        out = torch.empty(shape, dtype=dtype, device=internal.device)
        _check(lib().fgi_field_unpack(self.h, _geom(dims), self.FIELD_KINDS[kind],
                                      ctypes.c_void_p(internal.data_ptr()), _ptr(out, dtype, shape, kind), _stream()))
        return out

    def trajectory_packed(self, dims, act, integ, tau, nsteps, U, P, eta1=None, eta2=None, pf_is_phi=False,
                          allow_noconv=False):
        """fgi_trajectory on internal-layout buffers (from field_pack); U, P updated in place."""
        if isinstance(integ, str):
            integ = integrator_builtin(integ)
        for t, k in ((U, "links"), (P, "momenta"), (eta1, "even"), (eta2, "even")):
            if t is not None and (t.dtype != torch.uint8 or t.numel() != self.field_bytes(dims, k)):
                raise FgiError(FGI_EINVAL, "internal %s buffer of the wrong size or dtype" % k)
        vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        dH = ctypes.c_double()
        st = fgi_stats()
        rc = _check(lib().fgi_trajectory_packed(self.h, _geom(dims), ctypes.byref(act.c()), ctypes.byref(integ),
                                                float(tau), int(nsteps), vp(U), vp(P), vp(eta1), vp(eta2),
                                                int(bool(pf_is_phi)), ctypes.byref(dH), ctypes.byref(st), _stream()),
                    (FGI_ENOCONV,) if allow_noconv else ())
        d = st.as_dict()
        d["status"] = rc
        return dH.value, d

    # ---- Markov chain on the device
    def refresh(self, dims, seed, traj, momenta=True, eta1=True, eta2=False):
        """Heatbath draws (P, eta1, eta2) of trajectory traj of the chain `seed` (None where not asked)."""
        su, sp, se = self._shapes(dims)
        P = torch.empty(sp, dtype=torch.float64, device="cuda") if momenta else None
        e1 = torch.empty(se, dtype=torch.complex128, device="cuda") if eta1 else None
        e2 = torch.empty(se, dtype=torch.complex128, device="cuda") if eta2 else None
        _check(lib().fgi_refresh(self.h, _geom(dims), int(seed), int(traj), _ptr(P, torch.float64, sp, "P"),
                                 _ptr(e1, torch.complex128, se, "eta1"), _ptr(e2, torch.complex128, se, "eta2"),
                                 _stream()))
        return P, e1, e2

    def hmc_run(self, dims, act, integ, tau, nsteps, U, seed, traj0, ntraj, metropolis=True, allow_noconv=False):
        """ntraj chain trajectories on U (updated in place); returns dH, accepted, plaquette lists and stats."""
        su, _, _ = self._shapes(dims)
        if isinstance(integ, str):
            integ = integrator_builtin(integ)
        n = max(int(ntraj), 1)
        dH, acc, plaq = (ctypes.c_double * n)(), (ctypes.c_int * n)(), (ctypes.c_double * n)()
        st = fgi_stats()
        rc = _check(lib().fgi_hmc_run(self.h, _geom(dims), ctypes.byref(act.c()), ctypes.byref(integ), float(tau),
                                      int(nsteps), _ptr(U, torch.complex128, su, "U"), int(seed), int(traj0),
                                      int(ntraj), int(bool(metropolis)), dH, acc, plaq, ctypes.byref(st), _stream()),
                    (FGI_ENOCONV,) if allow_noconv else ())
        d = st.as_dict()
        d["status"] = rc
        k = int(ntraj)
        return list(dH)[:k], [bool(a) for a in list(acc)[:k]], list(plaq)[:k], d

    def trajectory_batched(self, chains, act, integ, tau, nsteps, allow_noconv=False):
        """chains: list of dicts with dims, beta, kappa, U, P, eta (tensors on the
        device, U and P updated in place).  Returns (dH list, stats)."""
        n = len(chains)
        arr = (fgi_chain * n)()
        for i, ch in enumerate(chains):
            su, sp, se = self._shapes(ch["dims"])
            arr[i].dims = (ctypes.c_int * 4)(*[int(d) for d in ch["dims"]])
            arr[i].beta = float(ch["beta"])
            arr[i].kappa = float(ch.get("kappa", 0.0))
            arr[i].U = _ptr(ch["U"], torch.complex128, su, "U")
            arr[i].P = _ptr(ch["P"], torch.float64, sp, "P")
            arr[i].eta = _ptr(ch.get("eta"), torch.complex128, se, "eta")
        if isinstance(integ, str):
            integ = integrator_builtin(integ)
        dH = (ctypes.c_double * n)()
        st = fgi_stats()
        rc = _check(lib().fgi_trajectory_batched(self.h, n, ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(act.c()),
                                                 ctypes.byref(integ), float(tau), int(nsteps), dH, ctypes.byref(st),
                                                 _stream()), (FGI_ENOCONV,) if allow_noconv else ())
        d = st.as_dict()
        d["status"] = rc
        return list(dH), d

    def autotune_cg(self, dims, act, U, phi):
        """Time the CG schedules on this system, keep the fastest; returns the choices and timings."""
        su, _, se = self._shapes(dims)
        t = fgi_tuning()
        _check(lib().fgi_autotune_cg(self.h, _geom(dims), ctypes.byref(act.c()), _ptr(U, torch.complex128, su, "U"),
                                     _ptr(phi, torch.complex128, se, "phi"), ctypes.byref(t), _stream()))
        return t.as_dict()

    def autotune_batched(self, chains, act):
        """The autotuner on a batch of chains (dicts with dims, beta, kappa, U, P, eta as for trajectory_batched)."""
        n = len(chains)
        arr = (fgi_chain * n)()
        for i, ch in enumerate(chains):
            su, sp, se = self._shapes(ch["dims"])
            arr[i].dims = (ctypes.c_int * 4)(*[int(d) for d in ch["dims"]])
            arr[i].beta = float(ch["beta"])
            arr[i].kappa = float(ch.get("kappa", 0.0))
            arr[i].U = _ptr(ch["U"], torch.complex128, su, "U")
            arr[i].P = _ptr(ch["P"], torch.float64, sp, "P")
            arr[i].eta = _ptr(ch.get("eta"), torch.complex128, se, "eta")
        t = fgi_tuning()
        _check(lib().fgi_autotune_batched(self.h, n, ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(act.c()),
                                          ctypes.byref(t), _stream()))
        return t.as_dict()

    # ---- utilities
    def link_update(self, dims, h, P, U):
        su, sp, _ = self._shapes(dims)
        _check(lib().fgi_link_update(self.h, _geom(dims), float(h), _ptr(P, torch.float64, sp, "P"),
                                     _ptr(U, torch.complex128, su, "U"), _stream()))
        return U

    def reunitarize(self, dims, U):
        su, _, _ = self._shapes(dims)
        _check(lib().fgi_reunitarize(self.h, _geom(dims), _ptr(U, torch.complex128, su, "U"), _stream()))
        return U

    def exp_su3(self, p, h=1.0):
        n = p.shape[0]
        out = torch.empty((n, 3, 3), dtype=torch.complex128, device=p.device)
        _check(lib().fgi_exp_su3(self.h, int(n), _ptr(p, torch.float64, (n, 8), "p"), float(h),
                                 _ptr(out, torch.complex128, (n, 3, 3), "out"), _stream()))
        return out
