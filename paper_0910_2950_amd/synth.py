"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

This module holds only random-number generation of inputs; none of the
method's arithmetic lives here.  Everything runs on the host with numpy's
PCG64 generator, in a fixed draw order, so both sides read identical arrays:

  links     U  complex128 (4, V, 3, 3): Haar-random SU(3), mu-major, lexicographic sites
  momenta   P  float64    (4, V, 8):    Gaussian, unit variance per su(3) component
  noise     eta complex128 (V/2, 4, 3): Re, Im ~ N(0, 1/2) per even site, spin, colour
                                        (P(eta) ~ exp(-eta^+ eta))
  uniforms  u  float64     Metropolis accept/reject draws

Site order: i = x + Lx (y + Ly (z + Lz t)); even sites (x+y+z+t even) are
stored in lexicographic order.
"""
import numpy as np

SEED_BASE = 0x09102950


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def volume(dims):
    return int(np.prod(dims))


def haar_su3(gen, n):
    """n Haar-distributed SU(3) matrices: QR of a complex Gaussian matrix with
    the phases of R's diagonal moved into Q (Mezzadri's recipe), then divided by
    the principal cube root of the determinant."""
    z = (gen.standard_normal((n, 3, 3)) + 1j * gen.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return np.ascontiguousarray(q)


def unit_links(dims):
    V = volume(dims)
    U = np.zeros((4, V, 3, 3), np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def gaussian_momenta(gen, dims):
    return gen.standard_normal((4, volume(dims), 8))


def gaussian_noise(gen, dims):
    Vh = volume(dims) // 2
    return (gen.standard_normal((Vh, 4, 3)) + 1j * gen.standard_normal((Vh, 4, 3))) / np.sqrt(2.0)


def hot_start(dims, seed, fermions=True, n_uniform=0):
    """(U, P, eta, u) drawn in the fixed order U, P, eta, uniforms."""
    g = rng(seed)
    V = volume(dims)
    U = haar_su3(g, 4 * V).reshape(4, V, 3, 3)
    P = gaussian_momenta(g, dims)
    eta = gaussian_noise(g, dims) if fermions else None
    u = g.random(n_uniform) if n_uniform else None
    return U, P, eta, u


def refresh(dims, seed, fermions=True):
    """Fresh momenta and noise for a trajectory starting from given links."""
    g = rng(seed)
    P = gaussian_momenta(g, dims)
    eta = gaussian_noise(g, dims) if fermions else None
    return P, eta


def near_unit_links(dims, seed, eps):
    """Links exp(eps * X) with random su(3) X: a smooth field for tests that need
    small forces (e.g. perturbative checks).  Uses only the Gell-Mann basis."""
    g = rng(seed)
    V = volume(dims)
    a = g.standard_normal((4 * V, 8)) * eps
    lam = gell_mann()
    X = 0.5j * np.einsum("na,aij->nij", a, lam)
    w, v = np.linalg.eigh(-1j * X)
    E = np.einsum("nij,nj,nkj->nik", v, np.exp(1j * w), v.conj())
    return E.reshape(4, V, 3, 3)


def gell_mann():
    lam = np.zeros((8, 3, 3), np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam
