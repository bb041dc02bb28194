#!/usr/bin/env python3
"""Benchmark of the force-gradient HMC hot path on one MI355X.

Workload: Nf=2 Wilson fermions + Wilson gauge action on a 16^3 x 32 lattice,
beta = 5.6, kappa = 0.1575, even-odd preconditioned; links thermalised from a
seeded hot start by 20 FP64 HMC trajectories (Omelyan PQPQP, alpha = 0.1932,
Metropolis off for the first half); every measured trajectory starts from
that field with fresh seeded Gaussian momenta and pseudofermion noise.

One step = one trajectory (tau = 1) of the mixed-precision force-gradient
integrator (Table 1, last row, displacement form) at the step count n_FG at
which <dH^2> reaches the 80 % acceptance level; the FP64 leapfrog (PQP) leg is
timed the same way at its own matched step count and reported beside it.
All inputs (links, momenta, noise) are resident in HBM before timing starts.

Prints one JSON line (see the keys below).  --calibrate runs the step-size
sweep that fixes the matched step counts instead.
"""
import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s/trajectory at fixed <δH²> (FG vs leapfrog), 16^3x32 Nf=2; Dslash HBM GB/s"
HBM_PEAK_GBS = 8000.0
# target <dH^2> for 80 % acceptance: <P_acc> = erfc(sqrt(<dH>)/2), <dH^2> ~ 2 <dH>
DH2_TARGET = 0.257
# The legs of the matched-acceptance comparison: integrator, storage
# precision of the inner CG, link reconstruction of its sloppy links
LEGS = {"fg_mp16": ("FG", "mp16", 18), "fg_mp32": ("FG", "mp32", 12), "fg_fp64": ("FG", "fp64", 18),
        "pqpqp_fp64": ("PQPQP", "fp64", 18), "lf_fp64": ("PQP", "fp64", 18)}
# calibrated beside the timed legs for reference: FG-MP16 with 12-real links
CAL_ONLY = {"fg_mp16_r12": ("FG", "mp16", 12)}
# step counts swept by --calibrate (override with --cal-n)
CAL_N = {"fg_mp16": [15, 16, 17, 18, 20], "fg_mp16_r12": [15, 16, 17, 18, 19, 20, 22, 24],
         "fg_mp32": [15, 16, 17, 18, 19, 20, 22],
         "fg_fp64": [15, 16, 17, 18, 19], "pqpqp_fp64": [20, 22, 24, 28, 32, 36, 40, 44],
         "lf_fp64": [56, 64, 72, 76, 80]}
# n* per leg (the smallest swept n with <dH^2> <= DH2_TARGET) is read from
# this file, written from --calibrate runs; these apply when it is absent
CALIBRATION_FILE = os.path.join(ROOT, "profiles", "calibration_16x16x16x32.json")
N_STAR_FALLBACK = {"fg_mp16": 16, "fg_mp32": 16, "fg_fp64": 16, "pqpqp_fp64": 24, "lf_fp64": 80}
# compulsory bytes per output site of one bare Dslash (8 links + input + output spinor)
DSLASH_BYTES = {("mp16", 12): 8 * 24 + 2 * (48 + 4), ("mp16", 18): 8 * 36 + 2 * (48 + 4),
                ("mp32", 12): 8 * 48 + 2 * 96, ("mp32", 18): 8 * 72 + 2 * 96, ("fp64", 18): 8 * 144 + 2 * 192}
PREC_ID = {"fp64": 0, "mp32": 1, "mp16": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12, help="timed FG trajectories")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", default="16,16,16,32")
    ap.add_argument("--beta", type=float, default=5.6)
    ap.add_argument("--kappa", type=float, default=0.1575)
    ap.add_argument("--therm-pg", type=int, default=200, help="pure-gauge HMC trajectories from the hot start")
    ap.add_argument("--beta-pg", type=float, default=5.83, help="beta of the pure-gauge thermalisation phase")
    ap.add_argument("--therm", type=int, default=20, help="Nf=2 HMC trajectories after the pure-gauge phase")
    ap.add_argument("--therm-tau", type=float, default=2.0, help="trajectory length of the Nf=2 thermalisation")
    ap.add_argument("--therm-steps", type=int, default=32, help="FG steps per Nf=2 thermalisation trajectory")
    ap.add_argument("--therm-md-tol", type=float, default=1e-7, help="MD solve tolerance while thermalising")
    ap.add_argument("--n-fg", type=int, default=0, help="FG-MP16 step count (0: n* of the calibration)")
    ap.add_argument("--leg-traj", type=int, default=8,
                    help="trajectories of each comparison leg (FG-MP32, FG-FP64, PQPQP-FP64) at its n* (0: skip)")
    ap.add_argument("--lf-traj", type=int, default=12, help="trajectories of the FP64 leapfrog leg at its n*")
    ap.add_argument("--prec", default="mp16", choices=["fp64", "mp32", "mp16"])
    ap.add_argument("--recon", type=int, default=18, choices=[12, 18],
                    help="reals stored per sloppy link of the headline leg (16-bit or FP32)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--cg-batch", type=int, default=16)
    ap.add_argument("--cg-form", default="auto", choices=["auto", "0", "1"],
                    help="CG iteration form of the single-lattice solves: 0 classic (five launches), 1 "
                         "Chronopoulos-Gear (four), auto: the autotuner's choice per leg on full solves")
    ap.add_argument("--graphs", type=int, default=1, help="replay CG batches as HIP graphs (0: eager launches)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 32^3x64 Dslash roofline point")
    ap.add_argument("--no-batched", action="store_true", help="skip the 96-chain batched workload")
    ap.add_argument("--batched-steps", type=int, default=2, help="timed batched trajectories")
    ap.add_argument("--ensemble", default="2,8", metavar="K,...",
                    help="chain counts of the headline workload run together by the batched path ('' to skip)")
    ap.add_argument("--no-hasenbusch", action="store_true", help="skip the 32^3x64 Hasenbusch MD-step leg")
    ap.add_argument("--improved-steps", type=int, default=2,
                    help="pure-gauge FG trajectories per gauge action, Wilson and tree-level Symanzik (0: skip)")
    ap.add_argument("--fg-start", type=int, default=1, choices=[0, 1],
                    help="1: the displaced force's solve of an FG stage starts from the undisplaced solution")
    ap.add_argument("--exact-steps", type=int, default=2,
                    help="trajectories of the exact force-gradient form on the first timed inputs (0: skip)")
    ap.add_argument("--chain-steps", type=int, default=3, help="on-device Markov-chain trajectories (0: skip)")
    ap.add_argument("--dt4-steps", type=int, default=2,
                    help="exact-FG trajectories with the dt^4 brackets at both ends (0: skip)")
    ap.add_argument("--md-tol", type=float, default=1e-7,
                    help="force-solve tolerance of the looser-MD leg (0: skip; dH solves keep --tol)")
    ap.add_argument("--tune-alpha", type=int, default=4, metavar="K",
                    help="Omelyan alpha from Poisson brackets measured over 2K trajectories, two-fold "
                         "cross-validated (0: skip)")
    ap.add_argument("--tune-fg", type=int, default=5, metavar="K",
                    help="force-gradient family (lam, xi) from dt^2 and dt^4 brackets over 2K exact-FG "
                         "trajectories, two-fold cross-validated (0: skip)")
    ap.add_argument("--asym-factor", type=int, default=2,
                    help="the bracket legs (alpha tuning, dt^4 row, FG family tuning) run at this multiple of "
                         "their leg's n*: the shadow-Hamiltonian expansion describes dH only inside its asymptotic "
                         "range, and n* sits at the integrators' stability edge")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default CG schedule (block 256, XCD order, --cg-batch) instead of tuning per leg")
    ap.add_argument("--cpu-iters", type=int, default=12, help="oracle CG iterations timed for the CPU baseline")
    ap.add_argument("--calibrate", action="store_true", help="step-size sweep for the matched step counts")
    ap.add_argument("--cal-traj", type=int, default=32, help="trajectories per calibration point")
    ap.add_argument("--cal-legs", default=",".join(LEGS), help="comma-separated legs to calibrate")
    ap.add_argument("--cal-n", default="", help="step counts per leg, e.g. 'fg_mp16=18,20;lf_fp64=90'")
    ap.add_argument("--cal-out", default="", help="also write the calibration JSON to this file")
    ap.add_argument("--seed", type=int, default=0x09102950 + 2)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run one device copy of MIB MiB (a known-size kernel that calibrates "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


# fermion.hip up to this line holds the hopping-term kernels and their launchers;
# what follows (force gradients, the CG drivers) does not change the Dslash code
DSLASH_SOURCE_END = b"// ------------------------------------------------ force gradient (Section 4) ---"


def source_digest():
    """Digest of the Dslash kernel's sources (fgi_device.h and the kernel and
    launcher part of fermion.hip), recorded beside its counter measurements."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_0910_2950_amd", "csrc", "fermion.hip"), "rb") as fh:
        src = fh.read()
    cut = src.find(DSLASH_SOURCE_END)
    h.update(src if cut < 0 else src[:cut])
    with open(os.path.join(ROOT, "paper_0910_2950_amd", "csrc", "fgi_device.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_key, lattice="16x16x16x32"):
    """HBM bytes per launch of the profiled Dslash (kernel_key "prec/recon")
    from the committed rocprofv3 counter summary, or None when it is absent or
    the kernel source changed."""
    path = os.path.join(ROOT, "profiles", "dslash_hbm_traffic_%s_%s.txt" % (lattice, kernel_key.replace("/", "_")))
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest() or kv.get("kernel_key") != kernel_key:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Runner:
    def __init__(self, args):
        import torch

        from paper_0910_2950_amd import fgi, synth
        self.torch, self.fgi, self.synth = torch, fgi, synth
        self.args = args
        self.dims = tuple(int(x) for x in args.dims.split(","))
        self.dev = torch.device("cuda:0")
        self.ctx = fgi.Context(0)
        self.ctx.set_option("cg_batch", args.cg_batch)
        self.ctx.set_option("graphs", args.graphs)
        self.ctx.set_option("fg_start", args.fg_start)
        if args.cg_form != "auto":
            self.ctx.set_option("cg_form", int(args.cg_form))

    def action(self, prec, recon=18):
        return self.fgi.Action(beta=self.args.beta, kappa=self.args.kappa, cg_tol=self.args.tol,
                               cg_maxiter=50000, prec=prec, link_recon=recon)

    def to_dev(self, a):
        return self.torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)

    def thermalise(self):
        """Seeded hot start, then two phases of on-device HMC chains
        (fgi_hmc_run: momenta, noise and Metropolis uniforms drawn on the
        device, links reunitarised after every trajectory):
          1. --therm-pg pure-gauge trajectories at --beta-pg (FG, tau = 1,
             n = 10, no accept/reject): cheap, and they carry the plaquette
             from 0 to about the dynamical value (the Nf = 2 determinant acts
             at leading order as a shift of beta);
          2. --therm Nf = 2 trajectories at (beta, kappa) of the workload: FG,
             tau = --therm-tau, n = --therm-steps, MP16 solves (the MD solves at
             --therm-md-tol, the heatbath and energy solves at --tol) and the
             Metropolis test.  A chunk of 4 trajectories with more than two
             rejections raises n by a quarter before the next chunk (the
             field's stiffest fermion modes harden as it approaches
             equilibrium), so the run stays inside the integrator's stability
             range.
        Returns the links, the final plaquette and the per-trajectory history."""
        a = self.args
        synth = self.synth
        U0, _, _, _ = synth.hot_start(self.dims, a.seed, fermions=False)
        U = self.to_dev(U0)
        hist = []
        t0 = time.perf_counter()
        if a.therm_pg > 0:
            dH, acc, plaq, st = self.ctx.hmc_run(self.dims, self.fgi.Action(beta=a.beta_pg), "FG", 1.0, 10, U,
                                                 a.seed + 17, 0, a.therm_pg, metropolis=False)
            for k in range(a.therm_pg):
                hist.append(dict(phase="pure_gauge", beta=a.beta_pg, n=10, tau=1.0, dH=dH[k], acc=bool(acc[k]),
                                 plaq=plaq[k]))
            log("therm pure gauge beta=%.3f: %d trajectories, plaquette %.5f -> %.5f (%.1fs)" %
                (a.beta_pg, a.therm_pg, plaq[0], plaq[-1], time.perf_counter() - t0))
        act = dataclasses.replace(self.action("mp16", 12), cg_tol_md=a.therm_md_tol)
        n = a.therm_steps
        k = 0
        while k < a.therm:
            m = min(4, a.therm - k)
            t1 = time.perf_counter()
            dH, acc, plaq, st = self.ctx.hmc_run(self.dims, act, "FG", a.therm_tau, n, U, a.seed + 29, k, m)
            for j in range(m):
                hist.append(dict(phase="nf2", n=n, tau=a.therm_tau, dH=dH[j], acc=bool(acc[j]), plaq=plaq[j]))
                log("therm %2d n=%d dH=%+.4e acc=%d plaq=%.5f" % (k + j, n, dH[j], acc[j], plaq[j]))
            log("  chunk: %d CG iterations, %.1fs" % (st["cg_iters"], time.perf_counter() - t1))
            k += m
            if m - sum(acc) > m // 2:
                n = int(math.ceil(1.25 * n))
        plaq = hist[-1]["plaq"] if hist else float("nan")
        log("thermalisation %.1fs, plaquette %.5f" % (time.perf_counter() - t0, plaq))
        return U, plaq, hist

    def tune(self, U, prec, recon):
        """Autotune the CG schedule on the thermalised field for one precision
        (untimed); returns the choices, which apply() re-selects before a leg."""
        P, eta = self.synth.refresh(self.dims, self.args.seed + 700000)
        act = self.fgi.Action(beta=self.args.beta, kappa=self.args.kappa, cg_tol=self.args.tol, cg_maxiter=50000,
                              prec=prec, link_recon=recon)
        t = self.ctx.autotune_cg(self.dims, act, U, self.to_dev(eta))
        if self.args.cg_form != "auto":
            t["cg_form"] = int(self.args.cg_form)
        log("autotune %s: block %d, order %d, cg_batch %d, CG form %d (full solve %.2f / %.2f ms classic / "
            "Chronopoulos-Gear)" % (prec, t["dslash_block"], t["xcd_order"], t["cg_batch"], t["cg_form"],
                                    t["form_ms_per_solve"][0], t["form_ms_per_solve"][1]))
        return t

    def apply(self, t):
        if t is None:
            return
        self.ctx.set_option("dslash_block", t["dslash_block"])
        self.ctx.set_option("xcd_order", t["xcd_order"])
        self.ctx.set_option("cg_batch", t["cg_batch"])
        self.ctx.set_option("cg_form", t.get("cg_form", 0))

    def fresh_inputs(self, n, base):
        out = []
        for k in range(n):
            P, eta = self.synth.refresh(self.dims, base + k)
            out.append((self.to_dev(P), self.to_dev(eta)))
        return out

    def run_leg(self, U_therm, act, name, nsteps, inputs, profile=False):
        """Trajectories from U_therm with the given (P, eta) sets; returns per-trajectory records."""
        torch = self.torch
        integ = self.fgi.integrator_builtin(name, 0.1932) if isinstance(name, str) else name
        U = torch.empty_like(U_therm)
        P = torch.empty_like(inputs[0][0])
        if profile:
            self.ctx.set_option("profile_prec", PREC_ID[act.prec] if act.prec != "mp32" else 1)
            self.ctx.set_option("profile_reset", 1)
            self.ctx.set_option("profile", 1)
        recs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (P0, eta) in inputs:
            U.copy_(U_therm)
            P.copy_(P0)
            try:
                dH, st = self.ctx.trajectory(self.dims, act, integ, 1.0, nsteps, U, P, eta, allow_noconv=True)
            except self.fgi.FgiError as e:
                # a trajectory that left the integrator's stability range (a non-finite dH)
                # counts as rejected, with dH = +inf
                log("trajectory failed (%s): counted as dH = +inf" % e)
                dH, st = float("inf"), dict(solves=0, cg_iters=0, cg_iters_max=0, max_rel_resid=0.0,
                                            reliable_updates=0, force_evals=0, seconds=0.0, status=e.code)
            recs.append(dict(dH=dH, **st))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = None
        if profile:
            self.ctx.set_option("profile", 0)
            prof = self.ctx.get_profile()
        return recs, t1 - t0, prof


def tile_field(torch, U, dims, f=2):
    """U (4, V, 3, 3), x fastest, repeated f times along every axis: the same
    configuration on an f^4 times larger torus (still a valid SU(3) field)."""
    X, Y, Z, T = dims
    u = U.reshape(4, T, Z, Y, X, 3, 3).repeat(1, f, f, f, f, 1, 1)
    return u.reshape(4, -1, 3, 3).contiguous(), (f * X, f * Y, f * Z, f * T)


def dslash_roofline_large(R, U_therm, prec, recon):
    """The same bare-hop timing as the main roofline, on the thermalised field
    tiled to 32^3x64 (16 waves of sites per SIMD instead of one): 16 HIP-event
    timed launches after each of two CG solves of 32 full iterations."""
    torch, fgi = R.torch, R.fgi
    Ub, dims_b = tile_field(torch, U_therm, R.dims, 2)
    V = int(np.prod(dims_b))
    g = torch.Generator(device=R.dev)
    g.manual_seed(R.args.seed + 300000)
    phi = torch.randn((V // 2, 4, 3), dtype=torch.complex128, device=R.dev, generator=g)
    act = fgi.Action(beta=R.args.beta, kappa=R.args.kappa, cg_tol=1e-30, cg_maxiter=32, prec=prec, link_recon=recon)
    R.ctx.set_option("profile_prec", PREC_ID[prec] if prec != "mp32" else 1)
    R.ctx.set_option("profile", 1)
    # no inner stops (reliable updates) in these fixed-length solves, so every
    # CG launch does its full work (the profiled averages then describe the kernels)
    R.ctx.set_option("ru_delta", 1e-30)
    R.ctx.cg_solve(dims_b, act, Ub, phi, allow_noconv=True)
    R.ctx.set_option("profile_reset", 1)
    for _ in range(2):
        R.ctx.cg_solve(dims_b, act, Ub, phi, allow_noconv=True)
    ms, launches, sites = R.ctx.get_profile()
    R.ctx.set_option("profile", 0)
    R.ctx.set_option("ru_delta", 0.1)
    del Ub, phi
    torch.cuda.empty_cache()
    bps = DSLASH_BYTES[(prec, recon)]
    avg_s = ms / 1e3 / launches
    achieved = sites / launches * bps / avg_s / 1e9
    traffic = read_traffic("%s/%d" % (prec, recon), "x".join(map(str, dims_b)))
    return dict(lattice=list(dims_b), bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                traffic_GBs=round(traffic / avg_s / 1e9, 1) if traffic else None,
                avg_launch_us=round(avg_s * 1e6, 3), launches_timed=launches, kernel_key="%s/%d" % (prec, recon),
                algorithmic_bytes_per_launch=sites / launches * bps,
                kernel="bare even-odd Dslash hop t = D_oe g5 q (%s/%d), %d output sites per launch, on the "
                       "thermalised 16^3x32 field repeated 2x2x2x2" % (prec, recon, V // 2))


def halo_leg(R, U_therm, reps=50, ranks=8):
    """One GPU's share of the 32^3x64 lattice split over `ranks` GPUs in t: the
    local 32^3x(64/ranks) slab of the thermalised field repeated 2x2x2x2, its
    hopping term through face buffers (fgi_halo_time: face pack, interior
    launch, face launches, one launch over all sites, and the plain local hop),
    MP16 with FP16/12 and fixed-point 16-bit/18 links.  The face transfer itself (xGMI) is not
    part of a one-GPU run; its time at 153 GB/s per link is given beside."""
    torch, fgi = R.torch, R.fgi
    Ub, dims_b = tile_field(torch, U_therm, R.dims, 2)
    Lt = dims_b[3] // ranks
    loc = (dims_b[0], dims_b[1], dims_b[2], Lt)
    V = int(np.prod(loc))
    U = Ub[:, :V].contiguous()
    del Ub
    torch.cuda.empty_cache()
    g = torch.Generator(device=R.dev)
    g.manual_seed(R.args.seed + 450000)
    src = torch.randn((V // 2, 4, 3), dtype=torch.complex128, device=R.dev, generator=g)
    out = dict(local_lattice=list(loc), ranks=ranks, reps=reps)
    for recon in (12, 18):
        act = fgi.Action(beta=R.args.beta, kappa=R.args.kappa, prec="mp16", link_recon=recon)
        t = R.ctx.halo_time(loc, act, U, src, reps)
        t["xgmi_us_per_face_at_153GBs"] = round(t["halo_bytes"] / 153e9 * 1e6, 2)
        t["hop_bytes_algorithmic"] = (V // 2) * DSLASH_BYTES[("mp16", recon)]
        out["mp16/%d" % recon] = t
    del U, src
    torch.cuda.empty_cache()
    return out


def hasenbusch_leg(R, U_therm, prec):
    """The large-lattice workload: Nf=2 at kappa = 0.158 with Hasenbusch mass
    preconditioning (kappa' = 0.150) on three nested FG time scales (S_2
    outermost, S_1, then S_G with two sub-steps each), on the thermalised
    16^3x32 field repeated 2x2x2x2 to 32^3x64.  One outer MD step of length
    1/8, i.e. a trajectory call with tau = 1/8 and one step: it includes the
    Hasenbusch heatbath solve and the two final-action solves."""
    torch, fgi = R.torch, R.fgi
    Ub, dims_b = tile_field(torch, U_therm, R.dims, 2)
    V = int(np.prod(dims_b))
    g = torch.Generator(device=R.dev)
    g.manual_seed(R.args.seed + 400000)
    P = torch.randn((4, V, 8), dtype=torch.float64, device=R.dev, generator=g)
    eta1 = torch.randn((V // 2, 4, 3), dtype=torch.complex128, device=R.dev, generator=g)
    eta2 = torch.randn((V // 2, 4, 3), dtype=torch.complex128, device=R.dev, generator=g)
    FG = [("P", 1 / 6, 0.0), ("Q", 0.5, 0.0), ("G", 2 / 3, 1 / 72), ("Q", 0.5, 0.0), ("P", 1 / 6, 0.0)]
    integ = fgi.integrator_from_levels([(FG, fgi.TERM_HASEN, 1), (FG, fgi.TERM_FERMION, 2), (FG, fgi.TERM_GAUGE, 2)])
    act = fgi.Action(beta=R.args.beta, kappa=0.158, kappa_hasen=0.150, cg_tol=R.args.tol, cg_maxiter=100000,
                     prec=prec, link_recon=12 if prec != "fp64" else 18)
    R.ctx.set_option("profile_prec", PREC_ID[prec] if prec != "mp32" else 1)
    R.ctx.set_option("profile_reset", 1)
    R.ctx.set_option("profile", 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dH, st = R.ctx.trajectory(dims_b, act, integ, 0.125, 1, Ub, P, eta1, eta2)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    R.ctx.set_option("profile", 0)
    ms, launches, sites = R.ctx.get_profile()
    del Ub, P, eta1, eta2
    torch.cuda.empty_cache()
    bps = DSLASH_BYTES[(prec, 12 if prec != "fp64" else 18)]
    hop_s = ms / 1e3 / max(launches, 1)
    return dict(workload="Nf=2 32x32x32x64 beta=%.2f kappa=0.158, Hasenbusch kappa'=0.150, nested FG (S2 / S1 x2 / "
                         "SG x2), thermalised 16^3x32 field repeated 2x2x2x2; one outer MD step of 1/8 incl. "
                         "heatbath and final-action solves; %s CG tol %.0e" % (R.args.beta, prec, R.args.tol),
                s_per_outer_step=round(sec, 4), dH=dH, solves=st["solves"], cg_iters=st["cg_iters"],
                cg_iters_max=st["cg_iters_max"], max_rel_resid=st["max_rel_resid"],
                dslash_achieved_GBs=round(sites / max(launches, 1) * bps / hop_s / 1e9, 1) if launches else None,
                dslash_avg_launch_us=round(hop_s * 1e6, 3) if launches else None)


BATCH_SPEC = [((4, 4, 4, 4), 32), ((6, 6, 6, 6), 32), ((8, 8, 8, 8), 24), ((8, 8, 8, 16), 8)]


def batched_leg(R, prec, nsteps, steps, recon=12):
    """96 independent chains of uneven sizes (32x 4^4, 32x 6^4, 24x 8^4,
    8x 8^3x16), beta ~ U[5.5, 6.0], kappa ~ U[0.150, 0.157], each a seeded Haar
    start with Gaussian momenta and pseudofermion noise: FG trajectories of all
    chains in one batched call (one set of launches per MD sub-step) against
    the same trajectories run chain by chain."""
    torch, fgi, synth = R.torch, R.fgi, R.synth
    rng = synth.rng(R.args.seed + 500000)
    dims_list = [d for d, n in BATCH_SPEC for _ in range(n)]
    betas = rng.uniform(5.5, 6.0, len(dims_list))
    kappas = rng.uniform(0.150, 0.157, len(dims_list))
    host = []
    for k, dims in enumerate(dims_list):
        U0, P0, eta, _ = synth.hot_start(dims, R.args.seed + 600000 + k, fermions=True)
        host.append((R.to_dev(U0), R.to_dev(P0), R.to_dev(eta)))
    act = fgi.Action(beta=0.0, cg_tol=R.args.tol, cg_maxiter=50000, prec=prec, link_recon=recon if prec != "fp64" else 18)

    def fresh():
        return [dict(dims=d, beta=b, kappa=kp, U=U.clone(), P=P.clone(), eta=e)
                for d, b, kp, (U, P, e) in zip(dims_list, betas, kappas, host)]

    tuning = None
    if not R.args.no_autotune:
        tuning = R.ctx.autotune_batched(fresh(), act)
        log("autotune batched: block %d, order %d, cg_batch %d" % (tuning["dslash_block"], tuning["xcd_order"],
                                                                  tuning["cg_batch"]))
    R.ctx.trajectory_batched(fresh(), act, "FG", 1.0, nsteps)  # warmup (graph capture)
    times, iters = [], []
    for _ in range(steps):
        chains = fresh()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dH, st = R.ctx.trajectory_batched(chains, act, "FG", 1.0, nsteps)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        iters.append(st["cg_iters"])
    t_batch = float(np.mean(times))
    # the same trajectories chain by chain
    chains = fresh()
    integ = fgi.integrator_builtin("FG")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ch in chains:
        a1 = fgi.Action(beta=float(ch["beta"]), kappa=float(ch["kappa"]), cg_tol=R.args.tol, cg_maxiter=50000,
                        prec=prec, link_recon=act.link_recon)
        R.ctx.trajectory(ch["dims"], a1, integ, 1.0, nsteps, ch["U"], ch["P"], ch["eta"])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    return dict(workload="96 chains (32x 4^4, 32x 6^4, 24x 8^4, 8x 8^3x16), beta~U[5.5,6.0], kappa~U[0.150,0.157], "
                         "Haar starts; FG n=%d tau=1, %s/%d CG tol %.0e" % (nsteps, prec, act.link_recon, R.args.tol),
                chains=len(dims_list), s_per_batched_trajectory=round(t_batch, 5),
                chain_trajectories_per_s=round(len(dims_list) / t_batch, 2),
                s_chain_by_chain=round(t_seq, 4), speedup_vs_chain_by_chain=round(t_seq / t_batch, 2),
                cg_iters_per_batched_trajectory=float(np.mean(iters)), timed=steps, schedule=tuning)


def ensemble_leg(R, U_therm, act, nsteps, counts, ref_dH, steps=1):
    """K independent chains of the headline workload advanced together by the
    batched path (one set of launches per MD sub-step covers all K lattices):
    the FG trajectories of the headline leg's first K timed starts (its
    momenta and noise on the thermalised field), K chains at a time.  At
    16^3x32 every CG kernel of one chain fills the GPU with one wave per SIMD;
    K chains give each SIMD up to K waves (as many as the kernels' registers
    allow) and share each launch's fixed cost, so this measures how much
    throughput a single chain leaves unused.  dH of each chain is compared with the single
    chain run of the same start: the batched path gives each chain the bits
    of its single run, so the difference is zero."""
    torch, fgi = R.torch, R.fgi
    out = {}
    for K in counts:
        inputs = R.fresh_inputs(K, R.args.seed + 100000 + R.args.warmup)

        def fresh():
            return [dict(dims=R.dims, beta=R.args.beta, kappa=R.args.kappa, U=U_therm.clone(), P=P.clone(), eta=e)
                    for P, e in inputs]
        R.ctx.trajectory_batched(fresh(), act, "FG", 1.0, nsteps)  # warmup (graph capture)
        times, dHs = [], None
        for _ in range(steps):
            chains = fresh()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dHs, st = R.ctx.trajectory_batched(chains, act, "FG", 1.0, nsteps)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t = float(np.mean(times))
        m = min(K, len(ref_dH))
        out[str(K)] = dict(s_per_batched_trajectory=round(t, 4), trajectories_per_s=round(K / t, 3),
                           dH=dHs, max_abs_dH_diff_vs_single=float(np.max(np.abs(np.array(dHs[:m]) -
                                                                                  np.array(ref_dH[:m])))))
    return dict(workload="K chains of %s beta=%.2f kappa=%.4f from the thermalised field with the headline's first "
                         "K timed (momenta, noise); FG n=%d tau=1, %s/%d CG tol %.0e, batched path" %
                         ("x".join(map(str, R.dims)), R.args.beta, R.args.kappa, nsteps, act.prec, act.link_recon,
                          R.args.tol), timed=steps, chains=out)


def tune_alpha_leg(R, U_therm, k, n):
    """Section 3 tuning: {S,{S,T}} and {T,{S,T}} measured on the GPU at both ends
    of 2k PQPQP(0.1932) trajectories and the alpha minimising the predicted
    <dH^2> over all of them; checked by two-fold cross-validation: alpha tuned
    on each half of the starts is run on the other half, so the measured
    <dH^2> comes from trajectories the tuning never saw.  The starts follow a
    Metropolis chain from the thermalised links (each measured trajectory is
    the chain's next proposal), so the brackets sample an ensemble of gauge
    fields rather than fresh momenta on one field."""
    from paper_0910_2950_amd.tuning import predicted_dh2, tune_omelyan_alpha
    ctx, dims = R.ctx, R.dims
    act = R.action(R.args.prec, R.args.recon)
    inputs = R.fresh_inputs(2 * k, R.args.seed + 300000)
    dS, dT, dh0, links, acc = [], [], [], [], []
    t0 = time.perf_counter()
    metro = np.random.default_rng(R.args.seed + 300000 - 1)
    U_cur = U_therm.clone()
    for P0, eta in inputs:
        links.append(U_cur)
        phi = ctx.pf_heatbath(dims, act, U_cur, eta)
        s0, q0 = ctx.poisson_brackets(dims, act, U_cur, P0, phi, h=1e-4)
        U, P = U_cur.clone(), P0.clone()
        dH, _ = ctx.trajectory(dims, act, R.fgi.integrator_builtin("PQPQP", 0.1932), 1.0, n, U, P, eta)
        s1, q1 = ctx.poisson_brackets(dims, act, U, P, phi, h=1e-4)
        dS.append(s1 - s0)
        dT.append(q1 - q0)
        dh0.append(dH)
        log("  alpha tuning: start %d/%d, PQPQP(0.1932) dH %+.3e" % (len(dh0), 2 * k, dH))
        acc.append(bool(metro.random() < np.exp(-dH)))
        if acc[-1]:   # the starts follow a Metropolis chain: an ensemble, not one field
            ctx.reunitarize(dims, U)
            U_cur = U
    dS, dT = np.array(dS), np.array(dT)
    alpha = tune_omelyan_alpha(dS, dT)
    folds = (np.arange(k), np.arange(k, 2 * k))
    alphas, dh_cv, pred_cv = [], [0.0] * (2 * k), 0.0
    for fit, ev in ((0, 1), (1, 0)):
        a = tune_omelyan_alpha(dS[folds[fit]], dT[folds[fit]])
        alphas.append(a)
        pred_cv += predicted_dh2(a, dS[folds[ev]], dT[folds[ev]], 1.0 / n) / 2
        for i in folds[ev]:
            U, P = links[i].clone(), inputs[i][0].clone()
            dh_cv[i], _ = ctx.trajectory(dims, act, R.fgi.integrator_builtin("PQPQP", a), 1.0, n, U, P,
                                         inputs[i][1])
            log("  alpha tuning: start %d held out, alpha %.4f dH %+.3e" % (i + 1, a, dh_cv[i]))
    return dict(trajectories=2 * k, n=n, chain_accepted=acc, alpha_tuned=alpha, alpha_folds=alphas,
                predicted_dH2={"0.1932": predicted_dh2(0.1932, dS, dT, 1.0 / n),
                               "tuned": predicted_dh2(alpha, dS, dT, 1.0 / n), "cross_validated": pred_cv},
                measured_dH2={"0.1932": float(np.mean(np.square(dh0))),
                              "cross_validated": float(np.mean(np.square(dh_cv)))},
                dH={"0.1932": dh0, "cross_validated": dh_cv}, seconds=time.perf_counter() - t0)


def fg_row(b):
    """Table 1, last row: H~ = H - dt^4/155520 (36 STSST + 72 STTST + 126 TTSST
    + 54 TTTST) for the exact force-gradient integrator, so dH = dt^4 times the
    change of this combination over the trajectory (+ O(dt^6))."""
    return (36 * b["STSST"] + 72 * b["STTST"] + 126 * b["TTSST"] + 54 * b["TTTST"]) / 155520.0


def dt4_leg(R, U_therm, act, n, inputs):
    """Table 1's dt^4 row on the thermalised field: the four dt^4 brackets
    (fgi_poisson_brackets4, step 1e-3) at both ends of exact-FG trajectories
    (n steps, tau = 1) from the given starts, the predicted dH beside the
    measured one, and the displacement form's dH from the same start."""
    torch, ctx, dims = R.torch, R.ctx, R.dims
    act_ex = dataclasses.replace(act, fg_exact=True)
    out = []
    t0 = time.perf_counter()
    for P0, eta in inputs:
        phi = ctx.pf_heatbath(dims, act, U_therm, eta)
        b0 = ctx.poisson_brackets4(dims, act, U_therm, P0, phi, h=1e-3)
        U, P = U_therm.clone(), P0.clone()
        dH, _ = ctx.trajectory(dims, act_ex, "FG", 1.0, n, U, P, phi, pf_is_phi=True)
        b1 = ctx.poisson_brackets4(dims, act, U, P, phi, h=1e-3)
        U, P = U_therm.clone(), P0.clone()
        dHd, _ = ctx.trajectory(dims, act, "FG", 1.0, n, U, P, phi, pf_is_phi=True)
        pred = (fg_row(b1) - fg_row(b0)) / n ** 4
        out.append(dict(dH_exact=dH, dH_predicted=pred, dH_displacement=dHd,
                        brackets_start=b0, brackets_end=b1))
    return dict(n=n, trajectories=len(out), records=out, seconds=time.perf_counter() - t0,
                note="predicted = dt^4 Delta(36 STSST + 72 STTST + 126 TTSST + 54 TTTST)/155520 (Table 1, last row)")


def fg_family_leg(R, U_therm, act, n, k):
    """The conclusions' next step for the fourth-order integrators: the family
    P(lam) Q(1/2) G(1 - 2 lam, xi) Q(1/2) P(lam) with the exact G stage (the FG
    integrator at (1/6, 1/72)) has a shadow Hamiltonian known to dt^4 in closed
    form (tuning.fg_family_coeffs), so with the six brackets measured at both
    ends of 2k exact-FG trajectories (n steps, tau = 1) the member minimising
    the predicted <dH^2> at dt = 1/n follows.  Checked by two-fold
    cross-validation: the member tuned on each half of the starts is run on
    the other half (same cost per step as FG) and compared with FG there.  The
    starts follow a Metropolis chain from the thermalised links, as in the
    alpha tuning."""
    from paper_0910_2950_amd import tuning
    ctx, dims = R.ctx, R.dims
    act_ex = dataclasses.replace(act, fg_exact=True)
    terms = R.fgi.TERM_GAUGE | R.fgi.TERM_FERMION

    def member(lam, xi):
        return R.fgi.integrator_from_levels([(tuning.fg_family_stages(lam, xi), terms, 1)])

    def run(integ, U0, P0, phi):
        U, P = U0.clone(), P0.clone()
        dH, _ = ctx.trajectory(dims, act_ex, integ, 1.0, n, U, P, phi, pf_is_phi=True)
        return dH, U, P

    t0 = time.perf_counter()
    fg = member(1.0 / 6.0, 1.0 / 72.0)
    keys = tuning.FG_KEYS2 + tuning.FG_KEYS4
    dB = {key: [] for key in keys}
    starts = R.fresh_inputs(2 * k, R.args.seed + 400000)
    metro = np.random.default_rng(R.args.seed + 400000 - 1)
    U_cur = U_therm.clone()
    links, phis, dh_fg, acc = [], [], [], []
    for P0, eta in starts:
        links.append(U_cur)
        phis.append(ctx.pf_heatbath(dims, act, U_cur, eta))
        b0 = ctx.poisson_brackets4(dims, act, U_cur, P0, phis[-1], h=1e-3)
        dH, U, P = run(fg, U_cur, P0, phis[-1])
        b1 = ctx.poisson_brackets4(dims, act, U, P, phis[-1], h=1e-3)
        for key in keys:
            dB[key].append(b1[key] - b0[key])
        dh_fg.append(dH)
        log("  FG family tuning: start %d/%d, FG dH %+.3e" % (len(dh_fg), 2 * k, dH))
        acc.append(bool(metro.random() < np.exp(-dH)))
        if acc[-1]:   # the starts follow a Metropolis chain: an ensemble, not one field
            ctx.reunitarize(dims, U)
            U_cur = U
    dB = {key: np.array(v) for key, v in dB.items()}
    dt = 1.0 / n
    lam, xi = tuning.tune_fg_family(dB, dt)
    folds = (np.arange(k), np.arange(k, 2 * k))
    fits, dh_cv, pred_cv = [], [0.0] * (2 * k), [0.0] * (2 * k)
    for fit, ev in ((0, 1), (1, 0)):
        lf, xf = tuning.tune_fg_family({key: v[folds[fit]] for key, v in dB.items()}, dt)
        fits.append((lf, xf))
        pe = tuning.predicted_dh_fg_family(lf, xf, {key: v[folds[ev]] for key, v in dB.items()}, dt)
        integ = member(lf, xf)
        for j, i in enumerate(folds[ev]):
            pred_cv[i] = float(pe[j])
            dh_cv[i] = run(integ, links[i], starts[i][0], phis[i])[0]
            log("  FG family tuning: start %d held out, dH %+.3e (predicted %+.3e)" % (i + 1, dh_cv[i], pred_cv[i]))

    def ms(v):
        return float(np.mean(np.square(v)))
    return dict(trajectories=2 * k, n=n, chain_accepted=acc, lam=lam, xi=xi, fold_fits=fits,
                predicted_dH2={"FG": ms(tuning.predicted_dh_fg_family(1.0 / 6.0, 1.0 / 72.0, dB, dt)),
                               "tuned": ms(tuning.predicted_dh_fg_family(lam, xi, dB, dt)),
                               "cross_validated": ms(pred_cv)},
                measured_dH2={"FG": ms(dh_fg), "cross_validated": ms(dh_cv)},
                dH={"FG": dh_fg, "cross_validated": dh_cv, "cross_validated_predicted": pred_cv},
                bracket_changes={key: [float(x) for x in v] for key, v in dB.items()},
                seconds=time.perf_counter() - t0)


def chain_leg(R, U_therm, act, n, ntraj, seed=0x5EED):
    """The on-device Markov chain (fgi_hmc_run): ntraj FG trajectories from the
    thermalised links with momenta, noise and the Metropolis uniform drawn on
    the device from (seed, trajectory index), accept/reject and
    reunitarisation, against the per-trajectory cost of the timed leg (whose
    inputs were resident before timing)."""
    torch = R.torch
    U = U_therm.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dH, acc, plaq, st = R.ctx.hmc_run(R.dims, act, "FG", 1.0, n, U, seed, 0, ntraj)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    return dict(trajectories=ntraj, n=n, s_per_traj=sec / ntraj, dH=dH, accepted=acc, plaquette=plaq,
                solves_per_traj=st["solves"] / ntraj, cg_iters_per_traj=st["cg_iters"] / ntraj)


# SU(3) products per link of the rectangle force: per nu != mu three pairs of
# five-link staples sharing their first factor (two four-link remainders of 3
# products each, summed, then 1 product with the shared factor) and U A; 198
# flops per 3x3 complex product (27 complex multiply-adds)
RECT_FORCE_FLOPS_PER_LINK = (3 * 3 * 7 + 1) * 198
FP64_PEAK_TFLOPS = 78.6


def improved_gauge_leg(R, U_therm, inputs, n, c1=-1.0 / 12.0):
    """The tree-level Symanzik gauge action (plaquettes at 1 - 8 c1, rectangles
    at c1) beside the Wilson action: pure-gauge FG trajectories (n steps, tau =
    1) from the thermalised links with the timed momenta, timed for both
    actions (no fermions, so the difference is the rectangle kernels' share of
    a trajectory; the field is in equilibrium for the Wilson action only, so
    the Symanzik dH is a cost probe, not an acceptance), and the rectangle force
    kernel alone: the total gauge force with and without the rectangles, HIP
    events on the library's stream around 20 calls each (packing and the
    plaquette kernel are common to both)."""
    torch = R.torch
    integ = R.fgi.integrator_builtin("FG", 0.1932)
    U = torch.empty_like(U_therm)
    P = torch.empty_like(inputs[0][0])
    out = dict(c1=c1, n=n, trajectories=len(inputs), kappa=0.0)
    for key, cc in (("wilson", 0.0), ("symanzik", c1)):
        act = R.fgi.Action(beta=R.args.beta, c1=cc)
        dHs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (P0, _) in inputs:
            U.copy_(U_therm)
            P.copy_(P0)
            dH, st = R.ctx.trajectory(R.dims, act, integ, 1.0, n, U, P)
            dHs.append(dH)
        torch.cuda.synchronize()
        out[key] = dict(s_per_traj=(time.perf_counter() - t0) / len(inputs), dH=dHs, force_evals=st["force_evals"])
    F = torch.empty((4, int(np.prod(R.dims)), 8), dtype=torch.float64, device=R.dev)
    ms = {}
    for key, cc in (("wilson", 0.0), ("symanzik", c1)):
        a = R.fgi.Action(beta=R.args.beta, c1=cc)
        R.ctx.force(R.dims, a, U_therm, F=F)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            R.ctx.force(R.dims, a, U_therm, F=F)
        e1.record()
        torch.cuda.synchronize()
        ms[key] = e0.elapsed_time(e1) / 20
    t_rect = (ms["symanzik"] - ms["wilson"]) * 1e-3
    links = 4 * int(np.prod(R.dims))
    tf = RECT_FORCE_FLOPS_PER_LINK * links / t_rect / 1e12 if t_rect > 0 else None
    out.update(gauge_force_call_ms=dict(wilson=round(ms["wilson"], 4), symanzik=round(ms["symanzik"], 4)),
               rect_force_kernel=dict(bound="alu", us=round(t_rect * 1e6, 2), flops_per_link=RECT_FORCE_FLOPS_PER_LINK,
                                      achieved_TFLOPs=round(tf, 2) if tf else None, peak_TFLOPs=FP64_PEAK_TFLOPS,
                                      frac=round(tf / FP64_PEAK_TFLOPS, 4) if tf else None))
    return out


def stout_leg(R, U_therm, rho=0.1, n=2, reps=20):
    """Cost of stout smearing at the benchmark lattice: fgi_stout_smear and
    fgi_stout_force at n levels against the same calls at zero levels (which
    only pack and unpack), HIP events on the library's stream; the difference
    per level is the smearing kernel, and the adjoint kernels plus a
    re-smearing for the force.  Per force evaluation with smeared fermions the
    library runs n smearing levels and n adjoint levels."""
    torch = R.torch
    V = int(np.prod(R.dims))
    Us = torch.empty_like(U_therm)
    Fs = torch.randn((4, V, 8), dtype=torch.float64, device=R.dev)
    F = torch.empty_like(Fs)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    ms = {}
    for k in (0, n):
        ms["smear", k] = timed(lambda: R.ctx.stout_smear(R.dims, rho, k, U_therm, Us))
        ms["force", k] = timed(lambda: R.ctx.stout_force(R.dims, rho, k, U_therm, Fs, F))
    smear_us = (ms["smear", n] - ms["smear", 0]) * 1e3 / n
    back_us = (ms["force", n] - ms["force", 0]) * 1e3 / n - smear_us
    return dict(rho=rho, n=n, smear_us_per_level=round(smear_us, 2), adjoint_us_per_level=round(back_us, 2),
                per_force_evaluation_ms=round(n * (smear_us + back_us) / 1e3, 4),
                call_ms={"smear_n0": round(ms["smear", 0], 4), "smear_n": round(ms["smear", n], 4),
                         "force_n0": round(ms["force", 0], 4), "force_n": round(ms["force", n], 4)})


def clover_leg(R, U_therm, inputs, n, kappa=0.135, csw=1.0, reps=10):
    """The clover-improved fermion operator (FP64; csw = 1, kappa = 0.135:
    kappa csw < 1/6 keeps A(x) positive on any field, and the clover operator
    stays below its critical kappa on the thermalised beta = 5.6 field, which
    at csw = 1 lies under the Wilson value of the timed leg) beside the Wilson
    operator at the same kappa: one FG trajectory (n steps, tau = 1) of each
    from the thermalised links with the first timed momenta and noise (FP64
    solves at the timed tolerance), and fgi_mhat with and without the clover
    term (HIP events around reps calls: pack, clover blocks, two hops and the
    site-local A_ee, A_oo^-1 products); the clover trajectory again with the
    mixed-precision solver (FP32 inner CG, FP64 defect correction)."""
    torch = R.torch
    integ = R.fgi.integrator_builtin("FG", 0.1932)
    U = torch.empty_like(U_therm)
    P = torch.empty_like(inputs[0][0])
    P0, eta = inputs[0]
    out = dict(kappa=kappa, csw=csw, n=n)
    for key, cc, prec in (("wilson", 0.0, "fp64"), ("clover", csw, "fp64"), ("clover_mp32", csw, "mp32")):
        act = R.fgi.Action(beta=R.args.beta, kappa=kappa, csw=cc, cg_tol=R.args.tol, prec=prec)
        U.copy_(U_therm)
        P.copy_(P0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dH, st = R.ctx.trajectory(R.dims, act, integ, 1.0, n, U, P, eta)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[key] = dict(s_per_traj=sec, dH=dH, solves=st["solves"], cg_iters=st["cg_iters"],
                        ms_per_cg_iter=round(sec * 1e3 / max(1, st["cg_iters"]), 4))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        R.ctx.mhat(R.dims, act, U_therm, eta)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            R.ctx.mhat(R.dims, act, U_therm, eta)
        e1.record()
        torch.cuda.synchronize()
        out[key]["mhat_call_ms"] = round(e0.elapsed_time(e1) / reps, 4)
    return out


def summarise(recs):
    """Per-leg statistics over independent trajectories from the same start
    field: <dH>, <dH^2>, acceptance <min(1, e^-dH)> and the Creutz mean
    <e^-dH>, each with its standard error over the trajectories, and the
    solver counts."""
    dh = np.array([r["dH"] for r in recs])
    n = len(dh)
    se = (lambda v: float(np.std(v, ddof=1) / math.sqrt(n))) if n > 1 else (lambda v: None)
    acc = np.minimum(1.0, np.exp(-np.minimum(dh, 700.0)))
    emd = np.exp(-np.minimum(dh, 700.0))
    return dict(trajectories=n, mean_dH=float(dh.mean()), mean_dH2=float((dh ** 2).mean()), mean_dH2_err=se(dh ** 2),
                acceptance=float(acc.mean()), acceptance_err=se(acc),
                exp_minus_dH=float(emd.mean()), exp_minus_dH_err=se(emd),
                solves_per_traj=float(np.mean([r["solves"] for r in recs])),
                cg_iters_per_traj=float(np.mean([r["cg_iters"] for r in recs])),
                cg_iters_max=int(max(r["cg_iters_max"] for r in recs)),
                max_rel_resid=float(max(r["max_rel_resid"] for r in recs)),
                reliable_updates_per_traj=float(np.mean([r["reliable_updates"] for r in recs])),
                force_evals_per_traj=float(np.mean([r["force_evals"] for r in recs])))


def n_star(leg):
    """n* of a leg from the committed calibration (or the fallback)."""
    try:
        with open(CALIBRATION_FILE) as fh:
            v = json.load(fh)["legs"][leg]["n_star"]
        if v:
            return int(v), "calibration"
    except (OSError, KeyError, ValueError, TypeError):
        pass
    return N_STAR_FALLBACK[leg], "fallback"


# Compulsory bytes per unit of work (each input read once, each output written
# once), for the whole-trajectory roofline: one CG iteration per even site for
# each inner precision (four hops plus the vectors of k_cg_p, M_CGQ and M_CGX),
# one reliable update per even site (the FP64 residual phi - Mhat^+ Mhat X:
# four FP64 hops plus its vectors, and the FP32 accumulator fold, conversion
# and clear), one force evaluation (fermion force per site plus its four FP64
# hops per even site, gauge force per link) and one link update per link.
def cg_iteration_bytes(prec, recon):
    """Compulsory bytes per even site of one CG iteration: two bare hops (H
    each); M_CGQ = a hop whose output is q, plus p in (H + vec); M_CGX = a hop
    that stores nothing (H - vec) plus q, p in and x, r in and out; k_cg_p = r
    in, p in and out.  4 H + 4 vec + 5 vx: MP16/12 1872 B, MP32/12 3168 B,
    FP64/18 7872 B."""
    hop = DSLASH_BYTES[(prec, recon)]
    if prec == "fp64":
        vec, vx = 192, 192
    elif prec == "mp32":
        vec, vx = 96, 96
    else:
        vec, vx = 52, 96
    hops = 2 * hop
    cgq = hop + vec
    cgx = (hop - vec) + 2 * vec + 4 * vx
    cgp = vx + 2 * vec
    return hops + cgq + cgx + cgp


RU_BYTES = 4 * DSLASH_BYTES[("fp64", 18)] + 3 * 192 + (96 + 2 * 192) + (192 + 96) + 96
FERMION_FORCE_SITE_BYTES, FP64_HOP_BYTES = 1472, DSLASH_BYTES[("fp64", 18)]
GAUGE_FORCE_LINK_BYTES, LINK_UPDATE_BYTES = 272, 352


def trajectory_roofline(summary, dims, prec, recon, link_updates, fermions, seconds):
    """t_roof = compulsory bytes of the trajectory (from its own counters) / 8 TB/s,
    and its ratio to the measured time."""
    V = int(np.prod(dims))
    Vh = V // 2
    it = summary["cg_iters_per_traj"] * Vh * cg_iteration_bytes(prec, recon)
    ru = summary["reliable_updates_per_traj"] * Vh * RU_BYTES
    nf = summary["force_evals_per_traj"]
    force = nf * 4 * V * GAUGE_FORCE_LINK_BYTES
    if fermions:
        force += nf * (V * FERMION_FORCE_SITE_BYTES + 4 * Vh * FP64_HOP_BYTES)
    upd = link_updates * 4 * V * (LINK_UPDATE_BYTES + (24 if prec == "mp16" else 48 if prec == "mp32" else 0))
    total = it + ru + force + upd
    t_roof = total / (HBM_PEAK_GBS * 1e9)
    return dict(t_roof_ms=round(t_roof * 1e3, 2), t_measured_ms=round(seconds * 1e3, 2),
                frac=round(t_roof / seconds, 4), bytes=dict(cg_iterations=it, reliable_updates=ru,
                                                             force_evaluations=force, link_updates=upd,
                                                             total=total),
                cg_iteration_bytes_per_even_site=cg_iteration_bytes(prec, recon))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def whole_trajectories(args):
    """The oracle's whole trajectories on the host for the two small
    workloads, beside the same trajectories on the GPU:
      4^4 pure gauge, beta = 6.0: PQP, PQPQP(0.1932) and FG at dtau in
          {1/4, 1/8, 1/16, 1/32}, tau = 1 (twelve trajectories, one Haar start);
      8^4 Nf = 2, beta = 5.6, kappa = 0.155: FG at n = 10, tau = 1, CG 1e-10,
          from a Haar start (FP64 on both sides)."""
    import torch

    from oracle import oracle as orc
    from paper_0910_2950_amd import fgi, synth
    orc.lib()
    ctx = fgi.Context(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    out = {}
    dims = (4, 4, 4, 4)
    U0, P0, _, _ = synth.hot_start(dims, synth.SEED_BASE, fermions=False)
    runs = [(nm, n) for nm in ("PQP", "PQPQP", "FG") for n in (4, 8, 16, 32)]
    t = time.perf_counter()
    for nm, n in runs:
        orc.trajectory(dims, 6.0, orc.table(nm), 1.0, n, U0, P0)
    t_cpu = (time.perf_counter() - t) / len(runs)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for nm, n in runs:
        ctx.trajectory(dims, fgi.Action(beta=6.0), nm, 1.0, n, dev(U0), dev(P0))
    torch.cuda.synchronize()
    t_gpu = (time.perf_counter() - t) / len(runs)
    out["4x4x4x4_pure_gauge"] = dict(s_per_traj=t_cpu, gpu_s_per_traj=t_gpu, trajectories=len(runs),
                                     runs="PQP, PQPQP(0.1932), FG x dtau 1/4..1/32, tau=1, beta=6.0")
    dims = (8, 8, 8, 8)
    U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 1, fermions=True)
    t = time.perf_counter()
    orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 10, U0, P0, kappa=0.155, eta=eta, tol=1e-10)
    t_cpu = time.perf_counter() - t
    act = fgi.Action(beta=5.6, kappa=0.155, cg_tol=1e-10)
    ctx.trajectory(dims, act, "FG", 1.0, 10, dev(U0), dev(P0), dev(eta))
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.trajectory(dims, act, "FG", 1.0, 10, dev(U0), dev(P0), dev(eta))
    torch.cuda.synchronize()
    out["8x8x8x8_nf2"] = dict(s_per_traj=t_cpu, gpu_s_per_traj=time.perf_counter() - t, trajectories=1,
                              runs="FG n=10, tau=1, beta=5.6, kappa=0.155, FP64 CG 1e-10")
    ctx.close()
    # the 96-chain batch: the first chain of each size class (the batched leg's own
    # seeded starts and couplings), one FG n=8 trajectory each, scaled by the class counts
    rng = synth.rng(args.seed + 500000)
    dims_list = [d for d, n in BATCH_SPEC for _ in range(n)]
    betas = rng.uniform(5.5, 6.0, len(dims_list))
    kappas = rng.uniform(0.150, 0.157, len(dims_list))
    est, parts, k0 = 0.0, {}, 0
    for d, n in BATCH_SPEC:
        U0, P0, eta, _ = synth.hot_start(d, args.seed + 600000 + k0, fermions=True)
        t = time.perf_counter()
        orc.trajectory(d, float(betas[k0]), orc.table("FG"), 1.0, 8, U0, P0, kappa=float(kappas[k0]), eta=eta,
                       tol=args.tol)
        dt = time.perf_counter() - t
        parts["x".join(map(str, d))] = round(dt, 4)
        est += n * dt
        k0 += n
    out["96_chain_batch"] = dict(s_per_batched_trajectory=est, extrapolated=True, sample_s_per_class=parts,
                                 runs="one FG n=8 trajectory (tau=1, FP64 CG %.0e) of the first chain of each size "
                                      "class, times the class counts (32, 32, 24, 8)" % args.tol)
    return out


def cpu_baseline(args, dims, lf, fg, n_fg):
    """The oracle as it stands on the host cores.  For the headline workload
    a bounded sample -- oracle CG iterations, one gauge force, one fermion
    force, one link update and one heatbath at 16^3x32 on a synthetic
    hot-start field -- scaled to one FG trajectory with the GPU run's counts
    (FP64 CG iterations per solve from the FP64 leapfrog leg, the FG solve
    and force counts); extrapolated, and labelled so.  For the 4^4 and 8^4
    workloads the oracle's whole trajectories (whole_trajectories)."""
    from oracle import oracle as orc
    from paper_0910_2950_amd import synth
    U, _, eta, _ = synth.hot_start(dims, args.seed + 77, fermions=True)
    P = synth.gaussian_momenta(synth.rng(args.seed + 78), dims)
    orc.lib()
    t = time.perf_counter()
    phi = orc.pf_heatbath(dims, args.kappa, U, eta)
    t_heat = time.perf_counter() - t
    t = time.perf_counter()
    orc.cg(dims, args.kappa, U, phi, tol=1e-30, maxiter=args.cpu_iters)
    t_it = (time.perf_counter() - t) / args.cpu_iters
    t = time.perf_counter()
    orc.gauge_force(dims, args.beta, U)
    t_gf = time.perf_counter() - t
    t = time.perf_counter()
    orc.fermion_force(dims, args.kappa, U, phi)
    t_ff = time.perf_counter() - t
    t = time.perf_counter()
    orc.link_update(dims, 0.1, P, U)
    t_lu = time.perf_counter() - t
    iters_per_solve = lf["cg_iters_per_traj"] / lf["solves_per_traj"] if lf else \
        fg["cg_iters_per_traj"] / fg["solves_per_traj"]
    iters = iters_per_solve * fg["solves_per_traj"]
    nf, nl = fg["force_evals_per_traj"], 2 * n_fg
    est = iters * t_it + nf * (t_gf + t_ff) + nl * t_lu + t_heat
    sample = ("extrapolated: oracle at %s on a hot-start field, %d CG iterations (%.3f s each), 1 gauge force "
              "(%.2f s), 1 fermion force (%.2f s), 1 link update (%.2f s), 1 heatbath (%.2f s); scaled to one FG "
              "trajectory at n=%d with the GPU run's counts (%.0f FP64 CG iterations, %.0f force evaluations, %d "
              "link updates)" % ("x".join(map(str, dims)), args.cpu_iters, t_it, t_gf, t_ff, t_lu, t_heat, n_fg,
                                 iters, nf, nl))
    return dict(value=est, unit="s/trajectory", cores=orc.threads(), cpu_model=cpu_model(), kind="oracle",
                sample=sample, configs=whole_trajectories(args))


def calibrate(args):
    """Step-size sweep on the thermalised field: for every leg and step count,
    --cal-traj trajectories (tau = 1) from the same field with fresh seeded
    (P, eta), <dH^2> with its standard error; n* = the smallest swept n whose
    <dH^2> is at most DH2_TARGET, and the power-law fit of <dH^2> against dtau
    over the points below 10."""
    R = Runner(args)
    U, plaq, hist = R.thermalise()
    ns = dict(CAL_N)
    for part in filter(None, args.cal_n.split(";")):
        k, v = part.split("=")
        ns[k.strip()] = [int(x) for x in v.split(",")]
    out = {}
    for leg in filter(None, args.cal_legs.split(",")):
        name, prec, recon = {**LEGS, **CAL_ONLY}[leg]
        R.apply(None if args.no_autotune else R.tune(U, prec, recon))
        act = R.action(prec, recon)
        pts = []
        for n in ns[leg]:
            inputs = R.fresh_inputs(args.cal_traj, args.seed + 500000 + 1000 * n)
            recs, sec, _ = R.run_leg(U, act, name, n, inputs)
            st = summarise(recs)
            st.update(n=n, s_per_traj=sec / len(recs), dH=[r["dH"] for r in recs])
            pts.append(st)
            log("cal %-10s n=%3d <dH^2>=%.4e +- %.1e acc=%.3f <e^-dH>=%.3f s/traj=%.3f solves=%.0f iters=%.0f" %
                (leg, n, st["mean_dH2"], st["mean_dH2_err"] or 0, st["acceptance"], st["exp_minus_dH"],
                 st["s_per_traj"], st["solves_per_traj"], st["cg_iters_per_traj"]))
        fit_pts = [p for p in pts if p["mean_dH2"] < 10.0]
        q = n_fit = None
        if len(fit_pts) >= 2:
            x = np.log(1.0 / np.array([p["n"] for p in fit_pts]))
            y = np.log(np.array([max(p["mean_dH2"], 1e-30) for p in fit_pts]))
            q, c = np.polyfit(x, y, 1)
            n_fit = float(math.exp((c - math.log(DH2_TARGET)) / q))
        # n*: the smallest swept n from which on every swept point meets the target
        ok = [p["n"] for p in pts if all(r["mean_dH2"] <= DH2_TARGET for r in pts if r["n"] >= p["n"])]
        out[leg] = dict(integrator=name, prec=prec, link_recon=recon, points=pts, slope=q, n_fit=n_fit,
                        n_star=min(ok) if ok else None)
        log("fit %s: <dH^2> ~ dt^%s  n_fit=%s n*=%s" % (leg, q, n_fit, out[leg]["n_star"]))
        res = calibration_record(args, R, out, plaq, hist)
        if args.cal_out:  # after every leg, so a cut-off sweep keeps its finished legs
            with open(args.cal_out, "w") as fh:
                json.dump(res, fh)
    print(json.dumps(calibration_record(args, R, out, plaq, hist)))


def calibration_record(args, R, out, plaq, hist):
    return dict(legs=out, plaquette=plaq, dims=list(R.dims), beta=args.beta, kappa=args.kappa, cg_tol=args.tol,
               target_dH2=DH2_TARGET, trajectories_per_point=args.cal_traj,
               thermalisation=dict(pure_gauge=args.therm_pg, beta_pg=args.beta_pg, nf2=args.therm,
                                   tau=args.therm_tau, steps=args.therm_steps,
                                   plaquette_history=[round(h["plaq"], 6) for h in hist if h["phase"] == "nf2"]),
               command="python bench.py " + " ".join(sys.argv[1:]))


def leg_record(R, U, leg, n, inputs, schedule):
    """One comparison leg at its step count n over the given starts: the
    per-leg statistics, seconds per trajectory and the whole-trajectory
    roofline."""
    name, prec, recon = LEGS[leg]
    R.apply(schedule)
    recs, sec, _ = R.run_leg(U, R.action(prec, recon), name, n, inputs)
    st = summarise(recs)
    st.update(n=n, s_per_traj=sec / len(recs), dH=[r["dH"] for r in recs], schedule=schedule)
    links = {"FG": 2 * n, "PQPQP": 2 * n, "PQP": n}[name]
    st["trajectory_roofline"] = trajectory_roofline(st, R.dims, prec, recon, links, True, st["s_per_traj"])
    log("%-10s n=%3d: %.4f s/traj  <dH^2>=%.4e +- %.1e acc=%.3f <e^-dH>=%.3f +- %.3f solves=%.1f iters=%.0f" %
        (leg, n, st["s_per_traj"], st["mean_dH2"], st["mean_dH2_err"] or 0, st["acceptance"], st["exp_minus_dH"],
         st["exp_minus_dH_err"] or 0, st["solves_per_traj"], st["cg_iters_per_traj"]))
    return st


def dslash_sample(R, U, inputs, n, prec, recon):
    """The Dslash roofline sample, outside the timed region: FG trajectories
    of the headline leg with the live hop profile on (after every solve, 16
    back-to-back launches of the CG's bare hop t = D_oe g5 q on the solve's
    stream, bracketed by HIP events)."""
    _, _, prof = R.run_leg(U, R.action(prec, recon), "FG", n, inputs, profile=True)
    return prof


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (--gpus %d requested)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calibrate:
        calibrate(args)
        return
    R = Runner(args)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        x = R.torch.ones(n, dtype=R.torch.float32, device=R.dev)
        y = R.torch.empty_like(x)
        y.copy_(x)
        R.torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (4 * n, 4 * n))
        del x, y
    t_setup = time.perf_counter()
    U, plaq, therm_hist = R.thermalise()
    nstar = {leg: n_star(leg) for leg in LEGS}
    n_fg = args.n_fg or nstar["fg_mp16"][0]
    recon_fg = args.recon if args.prec != "fp64" else 18
    act_fg = R.action(args.prec, recon_fg)
    inputs = R.fresh_inputs(args.warmup + args.steps, args.seed + 100000)
    log("setup (thermalisation + inputs) %.1fs; n* %s" % (time.perf_counter() - t_setup,
                                                          {k: v[0] for k, v in nstar.items()}))
    sched = {}
    if not args.no_autotune:
        for prec, recon in sorted({(args.prec, recon_fg)} | {(LEGS[k][1], LEGS[k][2]) for k in LEGS}):
            sched[prec, recon] = R.tune(U, prec, recon)
    tune_fg = sched.get((args.prec, recon_fg))
    R.apply(tune_fg)
    # warmup (untimed), then the headline: K FG trajectories, profiling off
    if args.warmup:
        R.run_leg(U, act_fg, "FG", n_fg, inputs[:args.warmup])
    recs, sec, _ = R.run_leg(U, act_fg, "FG", n_fg, inputs[args.warmup:])
    fg = summarise(recs)
    fg.update(n=n_fg, n_source=nstar["fg_mp16"][1] if not args.n_fg else "--n-fg", schedule=tune_fg,
              dH=[r["dH"] for r in recs])
    s_per_traj = sec / args.steps
    fg["s_per_traj"] = s_per_traj
    fg["trajectory_roofline"] = trajectory_roofline(fg, R.dims, args.prec, recon_fg, 2 * n_fg, True, s_per_traj)
    log("FG-%s n=%d: %.4f s/traj  <dH^2>=%.4e +- %.1e acc=%.3f <e^-dH>=%.3f solves=%.1f iters=%.0f" %
        (args.prec, n_fg, s_per_traj, fg["mean_dH2"], fg["mean_dH2_err"] or 0, fg["acceptance"],
         fg["exp_minus_dH"], fg["solves_per_traj"], fg["cg_iters_per_traj"]))
    log("FG trajectory roofline: %.1f ms of compulsory HBM traffic at 8 TB/s against %.1f ms measured (%.1f%%)" %
        (fg["trajectory_roofline"]["t_roof_ms"], s_per_traj * 1e3, 100 * fg["trajectory_roofline"]["frac"]))

    # the other legs at their own n*, on the first timed starts
    legs = {}
    k_leg = min(args.leg_traj, args.steps)
    for leg in ("fg_mp32", "fg_fp64", "pqpqp_fp64"):
        if k_leg > 0:
            _, prec, recon = LEGS[leg]
            legs[leg] = leg_record(R, U, leg, nstar[leg][0], inputs[args.warmup:args.warmup + k_leg],
                                   sched.get((prec, recon)))
            legs[leg]["n_source"] = nstar[leg][1]
    lf = None
    lf_inputs = []
    if args.lf_traj > 0:
        lf_inputs = inputs[args.warmup:args.warmup + min(args.lf_traj, args.steps)]
        lf_inputs += R.fresh_inputs(args.lf_traj - len(lf_inputs), args.seed + 200000)
        lf = leg_record(R, U, "lf_fp64", nstar["lf_fp64"][0], lf_inputs, sched.get(("fp64", 18)))
        lf["n_source"] = nstar["lf_fp64"][1]
        legs["lf_fp64"] = lf

    # exact G stage (Section 4 force gradient) on the first timed starts
    exact = None
    if args.exact_steps > 0:
        R.apply(tune_fg)
        k = min(args.exact_steps, args.steps)
        act_ex = dataclasses.replace(act_fg, fg_exact=True)
        recs_ex, sec_ex, _ = R.run_leg(U, act_ex, "FG", n_fg, inputs[args.warmup:args.warmup + k])
        exact = summarise(recs_ex)
        exact.update(n=n_fg, s_per_traj=sec_ex / k, dH=[r["dH"] for r in recs_ex],
                     dH_displacement_same_start=[r["dH"] for r in recs[:k]])
        log("FG-%s exact form n=%d: %.4f s/traj solves=%.1f iters=%.0f dH=%s (displacement %s)" %
            (args.prec, n_fg, exact["s_per_traj"], exact["solves_per_traj"], exact["cg_iters_per_traj"],
             ["%+.3e" % d for d in exact["dH"]], ["%+.3e" % d for d in exact["dH_displacement_same_start"]]))

    dt4 = None
    if args.dt4_steps > 0:
        R.apply(tune_fg)
        n4 = args.asym_factor * n_fg
        dt4 = dt4_leg(R, U, act_fg, n4, inputs[args.warmup:args.warmup + min(args.dt4_steps, args.steps)])
        for rec in dt4["records"]:
            log("dt^4 row at n=%d: exact-FG dH %+.4e, Table 1 prediction %+.4e; displacement-form dH %+.4e" %
                (n4, rec["dH_exact"], rec["dH_predicted"], rec["dH_displacement"]))

    # roofline of the dominant kernel, the bare sloppy Dslash hop inside CG,
    # from a separate profiled pass over the first timed starts
    R.apply(tune_fg)
    k_prof = min(2, args.steps)
    ms, launches, sites = dslash_sample(R, U, inputs[args.warmup:args.warmup + k_prof], n_fg, args.prec, recon_fg)
    V = int(np.prod(R.dims))
    bps = DSLASH_BYTES[(args.prec, recon_fg)]
    key = "%s/%d" % (args.prec, recon_fg)
    roof = None
    if launches:
        avg_s = ms / 1e3 / launches
        bytes_per_launch = sites / launches * bps
        achieved = bytes_per_launch / avg_s / 1e9
        traffic = read_traffic(key)
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    traffic_GBs=round(traffic / avg_s / 1e9, 1) if traffic else None,
                    kernel="bare even-odd Dslash hop t = D_oe g5 q of the CG (%s storage), %d output sites "
                           "per launch; HIP events around 16 back-to-back launches after every solve of %d "
                           "untimed FG trajectories" % (key, V // 2, k_prof),
                    algorithmic_bytes_per_launch=bytes_per_launch, avg_launch_us=round(avg_s * 1e6, 3),
                    launches_timed=launches)

    large = large_other = None
    if not args.no_large:
        # the 32^3x64 workload keeps 12-real FP16 links (the faster format there,
        # where the hop streams its links from HBM); the other format beside it
        recon_l = 12 if args.prec == "mp16" else recon_fg
        large = dslash_roofline_large(R, U, args.prec, recon_l)
        if args.prec == "mp16":
            large_other = dslash_roofline_large(R, U, args.prec, 18)
        for lg in filter(None, (large, large_other)):
            log("Dslash %s on %s: %.1f GB/s (%.1f%% of HBM peak), %.2f us per launch" %
                (lg["kernel_key"], "x".join(map(str, lg["lattice"])), lg["achieved"], 100 * lg["frac"],
                 lg["avg_launch_us"]))
    halo = None
    if not args.no_large:
        halo = halo_leg(R, U)
        for k in ("mp16/12", "mp16/18"):
            t = halo[k]
            log("t-split share %s %s: pack %.2f us, interior %.2f us, faces %.2f us (one launch %.2f us; local hop "
                "%.2f us); %d-byte faces, %.2f us each over one xGMI link" %
                ("x".join(map(str, halo["local_lattice"])), k, t["pack_us"], t["interior_us"], t["faces_us"],
                 t["all_us"], t["local_us"], t["halo_bytes"], t["xgmi_us_per_face_at_153GBs"]))
    hasen = None
    if not args.no_hasenbusch:
        hasen = hasenbusch_leg(R, U, args.prec)
        log("Hasenbusch 32^3x64: %.2f s per outer step, %d solves, %d CG iterations (max %d per solve), dH=%+.3e, "
            "Dslash %.1f GB/s" % (hasen["s_per_outer_step"], hasen["solves"], hasen["cg_iters"],
                                  hasen["cg_iters_max"], hasen["dH"], hasen["dslash_achieved_GBs"] or 0))
    alpha_leg = None
    if args.tune_alpha > 0:
        R.apply(tune_fg)
        alpha_leg = tune_alpha_leg(R, U, args.tune_alpha, args.asym_factor * nstar["pqpqp_fp64"][0])
        a = alpha_leg
        log("alpha tuning (PQPQP n=%d, %d trajectories): alpha %.4f (halves %.4f, %.4f), predicted <dH^2> %.3e -> "
            "%.3e; cross-validated: predicted %.3e, measured %.3e -> %.3e" %
            (a["n"], a["trajectories"], a["alpha_tuned"], a["alpha_folds"][0], a["alpha_folds"][1],
             a["predicted_dH2"]["0.1932"], a["predicted_dH2"]["tuned"], a["predicted_dH2"]["cross_validated"],
             a["measured_dH2"]["0.1932"], a["measured_dH2"]["cross_validated"]))
    family_leg = None
    if args.tune_fg > 0:
        R.apply(tune_fg)
        n_fam = args.asym_factor * n_fg
        family_leg = fg_family_leg(R, U, act_fg, n_fam, args.tune_fg)
        f = family_leg
        log("FG family tuning (exact G, n=%d, %d trajectories): (lam, xi) = (%.4f, %.5f), halves (%.4f, %.5f) and "
            "(%.4f, %.5f); predicted <dH^2> FG %.3e -> %.3e; cross-validated: predicted %.3e, measured FG %.3e -> "
            "%.3e" % (n_fam, f["trajectories"], f["lam"], f["xi"], f["fold_fits"][0][0], f["fold_fits"][0][1],
                      f["fold_fits"][1][0], f["fold_fits"][1][1], f["predicted_dH2"]["FG"], f["predicted_dH2"]["tuned"],
                      f["predicted_dH2"]["cross_validated"], f["measured_dH2"]["FG"],
                      f["measured_dH2"]["cross_validated"]))
    md_leg = None
    if args.md_tol > 0:
        # the first timed starts again, the solves inside force evaluations at --md-tol
        R.apply(tune_fg)
        k = min(k_leg or 4, args.steps)
        act_md = dataclasses.replace(act_fg, cg_tol_md=args.md_tol)
        recs_md, sec_md, _ = R.run_leg(U, act_md, "FG", n_fg, inputs[args.warmup:args.warmup + k])
        md_leg = summarise(recs_md)
        same = fg["dH"][:k]
        md_leg.update(cg_tol_md=args.md_tol, n=n_fg, s_per_traj=sec_md / k,
                      dH=[r["dH"] for r in recs_md], dH_single_tolerance_same_start=same,
                      speedup_vs_value=round(s_per_traj / (sec_md / k), 3))
        if lf is not None:
            kl = min(4, len(lf_inputs))
            R.apply(sched.get(("fp64", 18)))
            recs_lmd, sec_lmd, _ = R.run_leg(U, dataclasses.replace(R.action("fp64"), cg_tol_md=args.md_tol),
                                             "PQP", lf["n"], lf_inputs[:kl])
            lmd = summarise(recs_lmd)
            lmd.update(n=lf["n"], s_per_traj=sec_lmd / kl)
            md_leg["lf_fp64"] = lmd
            md_leg["speedup_vs_lf_fp64"] = round(lmd["s_per_traj"] / md_leg["s_per_traj"], 3)
        log("FG-%s n=%d with MD solves at %.0e: %.4f s/traj on %d starts (single tolerance %.4f), iters=%.0f" %
            (args.prec, n_fg, args.md_tol, md_leg["s_per_traj"], k, s_per_traj, md_leg["cg_iters_per_traj"]))
    chain = None
    if args.chain_steps > 0:
        R.apply(tune_fg)
        chain = chain_leg(R, U, act_fg, n_fg, args.chain_steps)
        log("on-device chain (fgi_hmc_run) FG-%s n=%d: %.4f s/traj (timed leg %.4f), accepted %s, dH %s" %
            (args.prec, n_fg, chain["s_per_traj"], s_per_traj, chain["accepted"],
             ["%+.3e" % d for d in chain["dH"]]))
    improved = clover = stout = None
    if args.improved_steps > 0:
        k = min(args.improved_steps, args.steps)
        improved = improved_gauge_leg(R, U, inputs[args.warmup:args.warmup + k], n_fg)
        log("pure-gauge FG n=%d: Wilson %.4f s/traj, tree-level Symanzik %.4f s/traj; gauge force call "
            "%.3f ms -> %.3f ms, rectangle kernel %.1f us = %.1f TFLOP/s FP64" %
            (n_fg, improved["wilson"]["s_per_traj"], improved["symanzik"]["s_per_traj"],
             improved["gauge_force_call_ms"]["wilson"], improved["gauge_force_call_ms"]["symanzik"],
             improved["rect_force_kernel"]["us"], improved["rect_force_kernel"]["achieved_TFLOPs"] or 0))
        clover = clover_leg(R, U, inputs[args.warmup:args.warmup + 1], n_fg)
        log("clover FG n=%d at kappa %.3f, csw %.2f: FP64 %.3f s/traj (%d CG iterations), MP32 %.3f s/traj; "
            "Wilson FP64 at the same kappa %.3f s/traj; mhat call %.3f -> %.3f ms" %
            (n_fg, clover["kappa"], clover["csw"], clover["clover"]["s_per_traj"], clover["clover"]["cg_iters"],
             clover["clover_mp32"]["s_per_traj"], clover["wilson"]["s_per_traj"],
             clover["wilson"]["mhat_call_ms"], clover["clover"]["mhat_call_ms"]))
        stout = stout_leg(R, U)
        log("stout smearing (rho %.2f, %d levels): %.1f us per level, adjoint %.1f us per level, %.3f ms per "
            "force evaluation" % (stout["rho"], stout["n"], stout["smear_us_per_level"],
                                  stout["adjoint_us_per_level"], stout["per_force_evaluation_ms"]))
    batched = None
    if not args.no_batched:
        try:
            batched = batched_leg(R, args.prec, 8, args.batched_steps)
            log("batched 96 chains: %.4f s per trajectory of all chains (%.1f chain-trajectories/s), chain by "
                "chain %.3f s, speedup %.1fx" % (batched["s_per_batched_trajectory"],
                                                 batched["chain_trajectories_per_s"], batched["s_chain_by_chain"],
                                                 batched["speedup_vs_chain_by_chain"]))
        except R.fgi.FgiError as e:
            batched = dict(error=str(e))
            log("batched 96 chains: %s" % e)
    ensemble = None
    if args.ensemble:
        R.apply(tune_fg)
        counts = [int(k) for k in args.ensemble.split(",")]
        try:
            ensemble = ensemble_leg(R, U, act_fg, n_fg, counts, fg["dH"])
            ensemble["single_chain_s_per_traj"] = round(s_per_traj, 4)
            for K, e in ensemble["chains"].items():
                e["throughput_vs_single_chain"] = round(e["trajectories_per_s"] * s_per_traj, 3)
                log("%s chains of %s batched: %.4f s per trajectory of all chains, %.3f trajectories/s (%.2fx one "
                    "chain), max |dH - dH single| %.1e" % (K, "x".join(map(str, R.dims)), e["s_per_batched_trajectory"],
                                                           e["trajectories_per_s"], e["throughput_vs_single_chain"],
                                                           e["max_abs_dH_diff_vs_single"]))
        except R.fgi.FgiError as e:
            ensemble = dict(error=str(e))
            log("ensemble: %s" % e)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, R.dims, lf, fg, n_fg)
        log("cpu baseline %.1f s/traj (extrapolated) on %d threads; whole oracle trajectories: %s; 96 chains %.1f s "
            "per batched trajectory (extrapolated)" %
            (cpu["value"], cpu["cores"], {k: round(v["s_per_traj"], 3) for k, v in cpu["configs"].items()
                                          if "s_per_traj" in v},
             cpu["configs"]["96_chain_batch"]["s_per_batched_trajectory"]))

    speedup = None
    if lf is not None:
        speedup = dict(value=round(lf["s_per_traj"] / s_per_traj, 3),
                       lf_fp64=dict(n=lf["n"], s_per_traj=lf["s_per_traj"], mean_dH2=lf["mean_dH2"],
                                    mean_dH2_err=lf["mean_dH2_err"]),
                       fg=dict(n=n_fg, s_per_traj=s_per_traj, mean_dH2=fg["mean_dH2"],
                               mean_dH2_err=fg["mean_dH2_err"]),
                       note="both legs at their own n*: the smallest step count whose <dH^2> in the committed "
                            "calibration (32 trajectories per point) is at most %.3f (80%% acceptance)" % DH2_TARGET)
    therm = dict(pure_gauge=args.therm_pg, beta_pg=args.beta_pg, nf2=args.therm, tau=args.therm_tau,
                 n_final=therm_hist[-1]["n"] if therm_hist else None,
                 plaquette_history=[round(h["plaq"], 6) for h in therm_hist if h["phase"] == "nf2"],
                 accepted=[h["acc"] for h in therm_hist if h["phase"] == "nf2"])
    out = dict(metric=METRIC, value=round(s_per_traj, 5), unit="s/trajectory", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(s_per_traj * 1e3, 3), higher_is_better=False,
               scaling="weak", vs_baseline=None, dtype={"fp64": "f64"}.get(args.prec, "f32"),
               precision={"mp16": "f32 arithmetic on f16 storage (per-site scale), f64 reliable updates, "
                                  "Hamiltonian and dH", "mp32": "f32 arithmetic and storage, f64 reliable updates, "
                                  "Hamiltonian and dH", "fp64": "f64 throughout"}[args.prec], data="synthetic",
               config=dict(workload="Nf=2 Wilson %s beta=%.2f kappa=%.4f, thermalised from a seeded hot start "
                                    "(%d pure-gauge trajectories at beta %.2f, then %d Nf=2 HMC trajectories); FG "
                                    "(%s, displacement form%s) at its calibrated n*=%d, tau=1, CG tol %.0e" %
                                    ("x".join(map(str, R.dims)), args.beta, args.kappa, args.therm_pg, args.beta_pg,
                                     args.therm, args.prec, ", displaced solve started from the undisplaced "
                                     "solution" if args.fg_start else "", n_fg, args.tol),
                           lattice=list(R.dims), integrator="FG", n_steps=n_fg, plaquette=round(plaq, 6)),
               fg=fg, legs=legs, speedup_vs_lf_fp64=speedup, fg_exact=exact, dt4_brackets=dt4, thermalisation=therm,
               roofline=roof, roofline_32x32x32x64=large, roofline_32x32x32x64_other_links=large_other,
               halo_32x32x32x8=halo,
               hasenbusch_32x32x32x64=hasen, batched=batched, ensemble=ensemble,
               alpha_tuning=alpha_leg, fg_family_tuning=family_leg, md_tolerance=md_leg, chain=chain, improved_gauge=improved, clover=clover,
               stout=stout, cpu_baseline=cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
