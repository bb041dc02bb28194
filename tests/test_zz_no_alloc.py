"""The allocation-free Schur operator fgi_mhat_packed_noalloc (for callers
that cannot allocate device memory) against fgi_mhat, the entry point whose
kernels it shares: bitwise equal on packed copies of the same fields, over two
calls in a row with the second on a smaller lattice (the fixed scratch array
keeps the first call's contents), and against the oracle's Mhat; sizes above
the fixed maximum and overlapping in/out buffers are refused before any
launch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_0910_2950_amd import fgi, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = fgi.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_noalloc_mhat_equals_mhat(ctx, orc):
    kappa = 0.155
    act = fgi.Action(beta=5.6, kappa=kappa)
    # second call smaller than the first; 16^3 x 64 sits at the scratch maximum
    cases = [((8, 8, 8, 16), False), ((6, 4, 4, 6), True), ((16, 16, 16, 64), False), ((4, 4, 4, 4), True)]
    for k, (dims, dagger) in enumerate(cases):
        print("noalloc mhat dims=%s dagger=%d" % (dims, dagger), flush=True)
        U0, _, eta, _ = synth.hot_start(dims, synth.SEED_BASE + 900 + k, fermions=True)
        U, e = dev(U0), dev(eta)
        ref = ctx.mhat(dims, act, U, e, dagger=dagger)
        Up = ctx.field_pack(dims, "links", U)
        ep = ctx.field_pack(dims, "even", e)
        out = torch.empty_like(ep)
        ctx.mhat_packed_noalloc(dims, kappa, Up, ep, out, dagger=dagger)
        res = ctx.field_unpack(dims, "even", out)
        torch.cuda.synchronize()
        assert torch.equal(res, ref), dims
        if int(np.prod(dims)) <= 4096:
            o = orc.mhat(dims, kappa, U0, eta, dagger=dagger)
            r = res.cpu().numpy()
            assert np.max(np.abs(r - o)) / np.max(np.abs(o)) < 1e-13


def test_noalloc_mhat_refuses_before_launch(ctx):
    L = fgi.lib()
    small = (4, 4, 4, 4)
    Up = torch.zeros(ctx.field_bytes(small, "links"), dtype=torch.uint8, device=DEV)
    ep = torch.zeros(ctx.field_bytes(small, "even"), dtype=torch.uint8, device=DEV)
    out = torch.full_like(ep, 7)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    # V/2 = 16^3 x 66 / 2 = 135168 > FGI_NOALLOC_MAX_VH: refused on the host
    rc = L.fgi_mhat_packed_noalloc(ctx.h, fgi._geom((16, 16, 16, 66)), 0.15, p(Up), p(ep), p(out), 0, None)
    assert rc == fgi.FGI_EINVAL and "FGI_NOALLOC_MAX_VH" in fgi.lib().fgi_last_error().decode()
    rc = L.fgi_mhat_packed_noalloc(ctx.h, fgi._geom(small), 0.15, p(Up), p(ep), p(ep), 0, None)
    assert rc == fgi.FGI_EINVAL
    rc = L.fgi_mhat_packed_noalloc(ctx.h, fgi._geom(small), float("nan"), p(Up), p(ep), p(out), 0, None)
    assert rc == fgi.FGI_EINVAL
    torch.cuda.synchronize()
    assert bool((out == 7).all())
