"""Seeded random inputs: initial temperatures, rotations, log-uniform
eigenvalues, Gaussian random fields and sensor picks.

Every generator takes an explicit ``numpy.random.Generator`` (PCG64) so that
the oracle and the GPU path see bit-identical inputs.
"""
from __future__ import annotations

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform(gen, lo, hi, n):
    return gen.uniform(lo, hi, size=n).astype(np.float64)


def haar_rotations(gen, n):
    """n random rotations, Haar distributed: QR of a Gaussian matrix with the
    signs of R's diagonal folded into Q, then det fixed to +1."""
    a = gen.standard_normal(size=(n, 3, 3))
    q, r = np.linalg.qr(a)
    d = np.sign(np.diagonal(r, axis1=1, axis2=2))
    d[d == 0] = 1.0
    q = q * d[:, None, :]
    det = np.linalg.det(q)
    q[:, :, 2] *= np.sign(det)[:, None]
    return q


def log_uniform(gen, lo, hi, shape):
    return np.exp(gen.uniform(np.log(lo), np.log(hi), size=shape))


def spd_tensors(gen, n, lam_lo, lam_hi):
    """Per-element symmetric positive definite tensors R diag(lam) R^T, packed
    as 6 rows (xx, yy, zz, xy, yz, xz) of length n."""
    rot = haar_rotations(gen, n)
    lam = log_uniform(gen, lam_lo, lam_hi, (n, 3))
    d = np.einsum("nij,nj,nkj->nik", rot, lam, rot)
    return np.stack([d[:, 0, 0], d[:, 1, 1], d[:, 2, 2],
                     d[:, 0, 1], d[:, 1, 2], d[:, 0, 2]]).copy()


def gaussian_random_field(gen, shape, corr_cells, mean=0.0, sigma=1.0):
    """Periodic Gaussian random field with squared-exponential correlation
    exp(-r^2 / (2 l^2)), l = corr_cells grid cells, made by filtering white
    noise in Fourier space, then shifted/scaled to the exact sample mean 0 and
    variance 1 before ``mean + sigma * field``.  Returned flattened with the
    first axis slowest (C order)."""
    noise = gen.standard_normal(size=shape)
    ks = np.meshgrid(*[np.fft.fftfreq(n) * 2.0 * np.pi for n in shape], indexing="ij")
    k2 = sum(k * k for k in ks)
    filt = np.exp(-0.25 * (corr_cells ** 2) * k2)
    field = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    field = (field - field.mean()) / field.std()
    return (mean + sigma * field).ravel()


def pick(gen, n, k):
    """k distinct ids out of range(n), sorted."""
    return np.sort(gen.choice(n, size=k, replace=False)).astype(np.int32)
