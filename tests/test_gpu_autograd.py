"""GPU tests of the autograd view of S_G (row a11): value, backward = -F,
double backward along F = minus the force gradient, and along a random
direction = the chart Hessian, all against the CPU oracle and central finite
differences (h = 1e-5, FP64) on 4^4 lattices, for the Wilson action and the
Iwasaki improved action (c1 = -0.331)."""
import numpy as np
import pytest
import scipy.linalg
import torch

from paper_0910_2950_amd import synth
from paper_0910_2950_amd.autograd import gauge_action
from paper_0910_2950_amd.fgi import Context

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
T = 0.5j * synth.gell_mann()


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def alg(p):
    return np.einsum("...a,aij->...ij", p, T)


def comps(X):
    """components x_a = -2 Tr(T^a X)"""
    return np.real(-2 * np.einsum("aij,...ji->...a", T, X))


@pytest.fixture(scope="module")
def setup():
    dims = (4, 4, 4, 4)
    U0 = synth.haar_su3(synth.rng(0x09102950 + 4), 4 * synth.volume(dims)).reshape(4, -1, 3, 3)
    return dims, 5.8, U0


@pytest.mark.parametrize("c1", [0.0, -0.331])
def test_value_and_gradient(ctx, orc, setup, c1):
    dims, beta, U0 = setup
    omega = torch.zeros((4, synth.volume(dims), 8), dtype=torch.float64, device=DEV, requires_grad=True)
    S = gauge_action(ctx, dims, beta, torch.from_numpy(U0).to(DEV), omega, c1)
    assert abs(S.item() - orc.gauge_action(dims, beta, U0, c1)) < 1e-12 * abs(S.item())
    (g,) = torch.autograd.grad(S, omega)
    F = orc.gauge_force(dims, beta, U0, c1)
    assert np.max(np.abs(g.cpu().numpy() + F)) < 1e-12 * np.max(np.abs(F))
    # central finite differences of S_G(exp(h T^a) U0) on a few links
    h = 1e-5
    for (mu, i, a) in [(0, 0, 0), (3, 255, 7), (2, 100, 4)]:
        Up, Um = U0.copy(), U0.copy()
        Up[mu, i] = scipy.linalg.expm(h * T[a]) @ U0[mu, i]
        Um[mu, i] = scipy.linalg.expm(-h * T[a]) @ U0[mu, i]
        fd = (orc.gauge_action(dims, beta, Up, c1) - orc.gauge_action(dims, beta, Um, c1)) / (2 * h)
        assert abs(fd - g[mu, i, a].item()) < 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("c1", [0.0, -0.331])
def test_double_backward_along_force_is_force_gradient(ctx, orc, setup, c1):
    dims, beta, U0 = setup
    Ud = torch.from_numpy(U0).to(DEV)
    omega = torch.zeros((4, synth.volume(dims), 8), dtype=torch.float64, device=DEV, requires_grad=True)
    S = gauge_action(ctx, dims, beta, Ud, omega, c1)
    (g,) = torch.autograd.grad(S, omega, create_graph=True)
    F = orc.gauge_force(dims, beta, U0, c1)
    (hv,) = torch.autograd.grad(g, omega, grad_outputs=torch.from_numpy(F).to(DEV))
    JF = orc.gauge_force_tangent(dims, beta, U0, F, c1)
    assert np.max(np.abs(hv.cpu().numpy() + JF)) < 1e-12 * np.max(np.abs(JF))


@pytest.mark.parametrize("c1", [0.0, -0.331])
def test_double_backward_random_direction_vs_finite_difference(ctx, orc, setup, c1):
    """H v = d/dh grad_chart(h v) at h = 0 with grad_chart(w) = dexp_{-w}(-F(exp(w) U0))
    = -F(U_h) + [h v, F(U_h)]/2 + O(h^2), evaluated with the oracle's force."""
    dims, beta, U0 = setup
    v = synth.rng(5).standard_normal((4, synth.volume(dims), 8))
    omega = torch.zeros_like(torch.from_numpy(v)).to(DEV).requires_grad_(True)
    S = gauge_action(ctx, dims, beta, torch.from_numpy(U0).to(DEV), omega, c1)
    (g,) = torch.autograd.grad(S, omega, create_graph=True)
    (hv,) = torch.autograd.grad(g, omega, grad_outputs=torch.from_numpy(v).to(DEV), retain_graph=True)
    h = 1e-5

    def chart_grad(t):
        Ut = orc.link_update(dims, t, v, U0)
        Ft = orc.gauge_force(dims, beta, Ut, c1)
        V, Fm = alg(t * v), alg(Ft)
        return -Ft + 0.5 * comps(V @ Fm - Fm @ V)

    fd = (chart_grad(h) - chart_grad(-h)) / (2 * h)
    assert np.max(np.abs(hv.cpu().numpy() - fd)) < 1e-6 * np.max(np.abs(fd))
    # the Hessian is symmetric: <w, H v> = <v, H w>
    w = synth.rng(6).standard_normal(v.shape)
    (hw,) = torch.autograd.grad(g, omega, grad_outputs=torch.from_numpy(w).to(DEV), retain_graph=True)
    a = float(np.sum(w * hv.cpu().numpy()))
    b = float(np.sum(v * hw.cpu().numpy()))
    assert abs(a - b) < 1e-10 * abs(a)


def test_nonzero_omega_rejected(ctx, setup):
    dims, beta, U0 = setup
    omega = torch.ones((4, synth.volume(dims), 8), dtype=torch.float64, device=DEV, requires_grad=True)
    with pytest.raises(ValueError):
        gauge_action(ctx, dims, beta, torch.from_numpy(U0).to(DEV), omega)
