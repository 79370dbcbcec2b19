"""CPU oracle for the PC1 projection step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never imports it, and it
imports nothing from there.

What it computes (the one-band representation I that the KNN filter reads):
the PCA of Sec. II.C.2 has four steps -- (i) subtract each band's average to
centre the image, (ii) covariance matrix, (iii) eigenvectors (Jacobi), (iv)
project the image onto the eigenvectors and keep the first component.  Steps
(ii) and (iii) need real image cubes and run on the host in the paper (Sec.
III.A.2.c, III.B.2.c); they stay outside this library, so the band averages and
the first eigenvector are inputs here.  The GPU implementations centre the
cube (Sec. III.A.2.a, III.B.2.a) and compute the projection as one
matrix-vector product (Sec. III.A.2.d, III.B.2.d); the desktop version does
both in double precision, so this oracle does too.  The KNN filter reads a
"normalized" I (Sec. II.C.3, Eq. 1); the paper does not say how.  Reading:
min-max normalisation to [0, 1] over the frame, and all zeros when I is
constant.  One rounding to binary32 at the end.

Pinned by ``tests/test_pc1_oracle_pins.py`` (exact rational evaluation on tiny
cubes, a rank-one cube whose projection is known, sign and scale invariances,
the constant image).
"""
from __future__ import annotations

import numpy as np


def centre(cube, mean):
    """Step (i) with the band averages given: Xc[p][b] = X[p][b] - mean[b] in binary64."""
    x = np.asarray(cube, dtype=np.float32)
    mu = np.asarray(mean, dtype=np.float64)
    if x.ndim != 2 or mu.shape != (x.shape[1],):
        raise ValueError("cube must be [pixels, bands] and mean [bands]")
    return x.astype(np.float64) - mu[None, :]


def project(xc, vec):
    """Step (iv): I[p] = sum_b Xc[p][b] * v[b], a matrix-vector product in binary64."""
    v = np.asarray(vec, dtype=np.float64)
    if v.shape != (xc.shape[1],):
        raise ValueError("vec must have one entry per band")
    return xc @ v


def normalise(values):
    """Min-max normalisation to [0, 1] over the frame (0 everywhere for a constant I)."""
    lo, hi = float(values.min()), float(values.max())
    if not hi > lo:
        return np.zeros_like(values)
    return (values - lo) / (hi - lo)


def pc1(cube, mean, vec, normalize: bool = True) -> np.ndarray:
    """The one-band representation I of a [pixels, bands] cube, binary32 [pixels]."""
    values = project(centre(cube, mean), vec)
    if normalize:
        values = normalise(values)
    return values.astype(np.float32)
