"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle is the parity authority, so an out-of-bounds read or an undefined
operation in it would make every parity test unsound.  This builds a second
copy of oracle/fgi_oracle.c with -fsanitize=address,undefined (host code
only; nothing here touches a GPU) and drives the heavy paths on small
lattices in a child process with the sanitizer runtime preloaded: FG, PQPQP
and Campostrini trajectories with Nf = 2 fermions (displacement and exact FG),
the improved gauge action with stout smearing, the clover operator, the
nested Hasenbusch driver, the dt^2 and dt^4 brackets and the on-device
chain's counterpart.  Any sanitizer report aborts the child with a non-zero
status.  Skipped when gcc's sanitizer runtimes are missing.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fgi_oracle.c")


def _runtime(name):
    try:
        p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


DRIVER = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, {root!r})
    from oracle import oracle as orc
    from paper_0910_2950_amd import synth
    orc._LIB = {lib!r}
    orc.lib()
    for dims in ((2, 2, 2, 2), (4, 4, 2, 2)):
        U0, P0, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 7, fermions=True)
        for name in ("FG", "PQPQP", "CAMPOSTRINI"):
            r = orc.trajectory(dims, 5.6, orc.table(name), 1.0, 3, U0, P0, kappa=0.155, eta=eta, tol=1e-12)
            assert r[4] == 0 and np.isfinite(r[2]), (dims, name, r[4])
        r = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 2, U0, P0, kappa=0.155, eta=eta, tol=1e-12,
                           fg_exact=True)
        assert r[4] == 0 and np.isfinite(r[2])
        r = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 2, U0, P0, kappa=0.155, eta=eta, tol=1e-12,
                           c1=-1.0 / 12.0, stout_rho=0.1, stout_n=2)
        assert r[4] == 0 and np.isfinite(r[2])
        r = orc.trajectory(dims, 5.6, orc.table("FG"), 1.0, 2, U0, P0, kappa=0.13, eta=eta, tol=1e-12, csw=1.0)
        assert r[4] == 0 and np.isfinite(r[2])
        fg = orc.table("FG")
        r = orc.trajectory_nested(dims, 5.6, [(fg, 4, 1), (fg, 2, 2), (fg, 1, 2)], 1.0, 2, U0, P0, kappa=0.155,
                                  kappa2=0.15, eta1=eta, eta2=eta, tol=1e-12)
        assert r[4] == 0 and np.isfinite(r[2])
        phi = orc.pf_heatbath(dims, 0.155, U0, eta)
        b4 = orc.brackets4(dims, 5.6, U0, P0, kappa=0.155, phi=phi, tol=1e-12)
        assert all(np.isfinite(v) for v in b4.values())
        r = orc.hmc_run(dims, 5.6, fg, 1.0, 3, U0, 11, 0, 2, kappa=0.155, fermions=True, tol=1e-12)
        assert r[4] == 0
    print("sanitized oracle ok", flush=True)
""")


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None or _runtime("libubsan.so") is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    cmd = ["gcc", "-std=gnu99", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", lib, SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([sys.executable, "-c", DRIVER.format(root=ROOT, lib=lib)], env=env, capture_output=True,
                       text=True, timeout=600)
    assert p.returncode == 0 and "sanitized oracle ok" in p.stdout, (p.returncode, p.stdout[-2000:],
                                                                      p.stderr[-4000:])
