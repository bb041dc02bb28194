"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/fgi.h declares, validates arguments before touching
a device, and its built-in Table 1 stage tables agree with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0910_2950_amd import fgi
from oracle.oracle import table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fgi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fgi_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    assert "fgi_trajectory" in syms and "fgi_force" in syms and len(syms) >= 20


def test_library_exports_every_declared_symbol():
    lib = fgi.lib()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    # the binding declares a signature for each of them
    assert set(declared_symbols()) == set(fgi.SIGNATURES), set(declared_symbols()) ^ set(fgi.SIGNATURES)


def test_struct_layouts_match_c_sizes():
    # sizes fixed by include/fgi.h (LP64): stage 24, level 16 + 16*24, integrator 8 + 4*level
    assert ctypes.sizeof(fgi.fgi_stage) == 24
    assert ctypes.sizeof(fgi.fgi_level) == 16 + 16 * 24
    assert ctypes.sizeof(fgi.fgi_integrator) == 8 + 4 * ctypes.sizeof(fgi.fgi_level)
    assert fgi.fgi_action.c1.offset == 48
    assert fgi.fgi_action.stout_rho.offset == 56 and fgi.fgi_action.stout_n.offset == 64
    assert fgi.fgi_action.cg_tol_md.offset == 72 and fgi.fgi_action.csw.offset == 80
    assert ctypes.sizeof(fgi.fgi_action) == 88
    # fgi_chain: int dims[4], int pad, double beta, double kappa, 3 pointers
    assert ctypes.sizeof(fgi.fgi_chain) == 64 and fgi.fgi_chain.beta.offset == 24
    # fgi_tuning: 4 ints, 6 + 5 + 2 doubles
    assert ctypes.sizeof(fgi.fgi_tuning) == 16 + 13 * 8 and fgi.fgi_tuning.sched_us_per_iter.offset == 16
    assert fgi.fgi_tuning.cg_form.offset == 12 and fgi.fgi_tuning.form_ms_per_solve.offset == 16 + 11 * 8


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """sizeof and offsetof as gcc lays the header's structs out, against ctypes"""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    structs = {"fgi_action": fgi.fgi_action, "fgi_stage": fgi.fgi_stage, "fgi_level": fgi.fgi_level,
               "fgi_integrator": fgi.fgi_integrator, "fgi_stats": fgi.fgi_stats, "fgi_chain": fgi.fgi_chain,
               "fgi_tuning": fgi.fgi_tuning}
    lines = []
    for name, cls in structs.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (name, name))
        for f in cls._fields_:
            if f[0] != "pad":
                lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f[0], name, f[0]))
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"fgi.h\"\nint main(void) {\n"
                   + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    for line in filter(None, out):
        name, field, val = line.split()
        cls = structs[name]
        got = ctypes.sizeof(cls) if field == "sizeof" else getattr(cls, field).offset
        assert got == int(val), (name, field, got, val)


@pytest.mark.parametrize("name", ["PQP", "QPQ", "PQPQP", "CAMPOSTRINI", "FG"])
def test_builtin_tables_match_oracle(name):
    I = fgi.integrator_builtin(name, 0.1932)
    assert I.nlevels == 1
    L = I.lev[0]
    got = [(chr(L.st[k].kind), L.st[k].w, L.st[k].xi) for k in range(L.nstages)]
    ref = table(name, 0.1932)
    assert len(got) == len(ref)
    for (k1, w1, x1), (k2, w2, x2) in zip(got, ref):
        assert k1 == k2 and abs(w1 - w2) < 1e-15 and abs(x1 - x2) < 1e-15


def test_campostrini_weights_sum_to_one():
    L = fgi.integrator_builtin("CAMPOSTRINI").lev[0]
    q = sum(L.st[k].w for k in range(L.nstages) if chr(L.st[k].kind) == "Q")
    p = sum(L.st[k].w for k in range(L.nstages) if chr(L.st[k].kind) == "P")
    assert abs(q - 1) < 1e-15 and abs(p - 1) < 1e-15


def test_builtin_rejects_bad_arguments():
    with pytest.raises(fgi.FgiError) as e:
        fgi.integrator_builtin(17)
    assert e.value.code == fgi.FGI_EINVAL
    with pytest.raises(fgi.FgiError):
        fgi.integrator_builtin("PQPQP", 0.7)


def test_null_context_is_rejected_without_device_work():
    lib = fgi.lib()
    S = ctypes.c_double()
    rc = lib.fgi_gauge_action(None, fgi._geom((4, 4, 4, 4)), 6.0, None, ctypes.byref(S), None)
    assert rc == fgi.FGI_EINVAL
    assert b"context" in lib.fgi_last_error()


def test_create_without_device_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = fgi.lib().fgi_create(ctypes.byref(h), 0)
    assert rc in (fgi.FGI_EHIP, fgi.FGI_EINVAL)
    assert fgi.lib().fgi_last_error() != b""
