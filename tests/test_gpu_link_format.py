"""GPU: what the 16-bit fixed-point storage of the 18 link reals (MP16,
link_recon = 18) is for.  Rounding the sloppy links is a fixed change of the
operator the inner CG inverts, and it costs iterations; rounding the vectors
is undone by the reliable updates and costs none.  FP16 links (the 12-real
format) round the entries near 1 to 4.9e-4 relative, the fixed point of the
18-real format to 1.5e-5 absolute.

On a pure-gauge thermalised 8^4 field (beta = 5.83) at kappa = 0.158 the
MP16 solve with fixed-point links needs no more iterations than with FP16
links and stays within 12 % of the FP64 solve (an FP64 emulation of the
three inner precisions on such a field gives FP64-like vectors 253, FP16
links 304, fixed-point links 275 iterations), and every solve meets the
1e-10 true residual.
"""
import numpy as np
import pytest
import torch

from paper_0910_2950_amd import synth
from paper_0910_2950_amd.fgi import Action, Context

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
DIMS = (8, 8, 8, 8)
KAPPA = 0.158


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def test_fixed_point_links_save_iterations(ctx):
    U = torch.from_numpy(synth.haar_su3(synth.rng(400), 4 * synth.volume(DIMS)).reshape(4, -1, 3, 3)).to(DEV)
    ctx.hmc_run(DIMS, Action(beta=5.83), "FG", 1.0, 10, U, 401, 0, 150, metropolis=False)
    ctx.reunitarize(DIMS, U)
    eta = torch.from_numpy(synth.gaussian_noise(synth.rng(402), DIMS)).to(DEV)
    phi = ctx.pf_heatbath(DIMS, Action(beta=5.6, kappa=KAPPA), U, eta)
    iters = {}
    for prec, recon in (("fp64", 18), ("mp32", 18), ("mp16", 12), ("mp16", 18)):
        act = Action(beta=5.6, kappa=KAPPA, cg_tol=1e-10, cg_maxiter=20000, prec=prec, link_recon=recon)
        _, st = ctx.cg_solve(DIMS, act, U, phi)
        iters[prec, recon] = st["cg_iters"]
        print(prec, recon, "iterations", st["cg_iters"], "true residual", st["max_rel_resid"], flush=True)
        assert st["max_rel_resid"] <= 1e-10
    assert iters["mp16", 18] <= iters["mp16", 12]
    assert iters["mp16", 18] <= 1.12 * iters["fp64", 18]
    assert iters["mp32", 18] <= 1.03 * iters["fp64", 18]
