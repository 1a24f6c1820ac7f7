"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module holds no arithmetic of the HMC method itself: no Dirac
operator, no exponential, no Gram-Schmidt reunitarisation, no Philox.  It
only draws seeded numpy random numbers and shapes them into the canonical
field layouts (lexicographic site i = x + Lx*(y + Ly*(z + Lz*t))):

* gauge links  complex128 (V, 4, 3, 3)
* spinors      complex128 (V, 4, 3)
* momenta      complex128 (V, 4, 3, 3), traceless Hermitian

SU(3) matrices come from the QR decomposition of a complex Gaussian matrix
with the phases of R's diagonal moved into Q (Mezzadri, Notices AMS 54
(2007) 592) followed by division by a cube root of the determinant; "near
identity" links apply the same QR step to 1 + eps*G.
"""
from __future__ import annotations

import numpy as np


def volume(L):
    return int(np.prod(L))


def rng(seed):
    return np.random.default_rng(seed)


def _qr_unitary(m):
    q, r = np.linalg.qr(m)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    return q * ph[..., None, :]


def _to_special(u):
    det = np.linalg.det(u)
    return u / (det ** (1.0 / 3.0))[..., None, None]


def random_su3(g, n):
    """n Haar-random SU(3) matrices, shape (n, 3, 3)."""
    z = (g.standard_normal((n, 3, 3)) + 1j * g.standard_normal((n, 3, 3))) / np.sqrt(2)
    return _to_special(_qr_unitary(z))


def near_identity_su3(g, n, eps):
    z = (g.standard_normal((n, 3, 3)) + 1j * g.standard_normal((n, 3, 3))) / np.sqrt(2)
    return _to_special(_qr_unitary(np.eye(3) + eps * z))


def gauge_field(seed, L, eps=None):
    """Random SU(3) links; Haar if eps is None, else near the identity."""
    g = rng(seed)
    n = volume(L) * 4
    u = random_su3(g, n) if eps is None else near_identity_su3(g, n, eps)
    return np.ascontiguousarray(u.reshape(volume(L), 4, 3, 3))


def gauge_transform(seed, L):
    """One Haar SU(3) matrix per site, shape (V, 3, 3)."""
    return np.ascontiguousarray(random_su3(rng(seed), volume(L)))


def spinor(seed, L, parity_mask=None, parity=None):
    """Complex Gaussian spinor; zero on the sites where parity_mask != parity."""
    g = rng(seed)
    V = volume(L)
    s = (g.standard_normal((V, 4, 3)) + 1j * g.standard_normal((V, 4, 3))) / np.sqrt(2)
    if parity_mask is not None:
        s[np.asarray(parity_mask, dtype=int) != parity] = 0
    return np.ascontiguousarray(s)


def integer_spinor(seed, L, lo=-8, hi=8):
    """Spinor with small integer components (exact sums in any order)."""
    g = rng(seed)
    V = volume(L)
    s = g.integers(lo, hi, (V, 4, 3)) + 1j * g.integers(lo, hi, (V, 4, 3))
    return np.ascontiguousarray(s.astype(np.complex128))


def hermitian_traceless(seed, L, scale=1.0):
    """Random traceless Hermitian 3x3 per link, shape (V, 4, 3, 3)."""
    g = rng(seed)
    n = volume(L) * 4
    a = g.standard_normal((n, 3, 3)) + 1j * g.standard_normal((n, 3, 3))
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[:, None, None] * np.eye(3)
    return np.ascontiguousarray((scale * h).reshape(volume(L), 4, 3, 3))


def site_coords(L):
    """(V, 4) int array of (x, y, z, t) in lexicographic order."""
    t, z, y, x = np.meshgrid(*(np.arange(n) for n in L[::-1]), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)
