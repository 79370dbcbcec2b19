"""Pins for the PC1 projection oracle (CPU): each check fixes the result by
something other than the oracle's own code -- exact rational arithmetic, a
cube whose projection is known in closed form, invariances of the definition,
and the degenerate constant image."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import pc1_oracle as po


def ulp32(x: float) -> float:
    return float(np.spacing(np.float32(abs(x))))


def exact_pc1(cube, mean, vec, normalize=True):
    """The definition in exact rational arithmetic (every binary32/binary64
    input is an exact rational), pure-Python loops: tiny cubes only."""
    npix, nb = cube.shape
    vals = []
    for p in range(npix):
        s = Fraction(0)
        for b in range(nb):
            s += (Fraction(float(cube[p, b])) - Fraction(float(mean[b]))) * Fraction(float(vec[b]))
        vals.append(s)
    if normalize:
        lo, hi = min(vals), max(vals)
        vals = [Fraction(0) if hi == lo else (v - lo) / (hi - lo) for v in vals]
    return vals


@pytest.mark.parametrize("seed,npix,nb", [(1, 12, 5), (2, 7, 16), (3, 20, 3), (4, 1, 9)])
@pytest.mark.parametrize("normalize", [True, False])
def test_matches_exact_rational_evaluation(seed, npix, nb, normalize):
    rng = np.random.default_rng(seed)
    cube = rng.random((npix, nb), dtype=np.float32)
    mean = rng.random(nb) * 0.8
    vec = rng.standard_normal(nb)
    got = po.pc1(cube, mean, vec, normalize)
    ref = exact_pc1(cube, mean, vec, normalize)
    for g, r in zip(got, ref):
        # binary64 evaluation rounded once to binary32: within half an ulp,
        # up to the binary64 rounding of the sum
        assert abs(Fraction(float(g)) - r) <= Fraction(ulp32(float(r))) * Fraction(1, 2) * Fraction(1000001, 1000000) \
            + Fraction(1, 2**60), (g, float(r))


def test_rank_one_cube_projects_to_its_coefficients():
    """X[p] = mean + a_p * u with u . u = 1 and v = u: I[p] = a_p exactly
    (dyadic values, so every step is exact)."""
    u = np.array([0.5, -0.5, 0.5, 0.5, 0.0, 0.0])
    mean = np.array([0.25, 0.5, 0.125, 0.75, 0.5, 0.375])
    a = np.array([0.0, 0.25, -0.5, 0.75, 0.125, -0.25, 1.0, 0.5])
    cube = (mean[None, :] + a[:, None] * u[None, :]).astype(np.float32)
    assert np.array_equal(cube.astype(np.float64), mean[None, :] + a[:, None] * u[None, :])
    raw = po.pc1(cube, mean, u, normalize=False)
    assert np.array_equal(raw, a.astype(np.float32))
    norm = po.pc1(cube, mean, u, normalize=True)
    assert np.array_equal(norm, ((a - a.min()) / (a.max() - a.min())).astype(np.float32))
    assert norm[np.argmin(a)] == 0.0 and norm[np.argmax(a)] == 1.0


def test_sign_of_the_eigenvector_mirrors_the_normalised_band():
    rng = np.random.default_rng(5)
    cube = rng.random((300, 10), dtype=np.float32)
    mean = rng.random(10)
    vec = rng.standard_normal(10)
    pos = po.pc1(cube, mean, vec).astype(np.float64)
    neg = po.pc1(cube, mean, -vec).astype(np.float64)
    assert np.max(np.abs(pos + neg - 1.0)) <= 2 * 2.0**-24
    assert pos.min() == 0.0 and pos.max() == 1.0


def test_scaling_the_eigenvector_by_a_power_of_two_changes_nothing():
    rng = np.random.default_rng(6)
    cube = rng.random((200, 7), dtype=np.float32)
    mean = rng.random(7)
    vec = rng.standard_normal(7)
    assert np.array_equal(po.pc1(cube, mean, vec), po.pc1(cube, mean, 4.0 * vec))


def test_band_averages_only_shift_the_raw_projection():
    """Centering subtracts mean . v from every pixel: the raw projections for
    two mean vectors differ by a constant, the normalised ones not at all."""
    rng = np.random.default_rng(7)
    cube = rng.random((150, 8), dtype=np.float32)
    vec = rng.standard_normal(8)
    m1, m2 = rng.random(8), rng.random(8)
    r1 = po.pc1(cube, m1, vec, normalize=False).astype(np.float64)
    r2 = po.pc1(cube, m2, vec, normalize=False).astype(np.float64)
    shift = float((m2 - m1) @ vec)
    assert np.max(np.abs((r1 - r2) - shift)) <= 4 * 2.0**-23 * max(1.0, np.max(np.abs(r1)))
    n1, n2 = po.pc1(cube, m1, vec), po.pc1(cube, m2, vec)
    assert np.max(np.abs(n1.astype(np.float64) - n2)) <= 2 * 2.0**-24


def test_constant_image_normalises_to_zero():
    cube = np.full((50, 4), 0.3, np.float32)
    out = po.pc1(cube, np.zeros(4), np.array([0.5, 0.5, 0.5, 0.5]))
    assert np.array_equal(out, np.zeros(50, np.float32))


def test_rejects_mismatched_shapes():
    with pytest.raises(ValueError):
        po.pc1(np.zeros((3, 4), np.float32), np.zeros(3), np.zeros(4))
    with pytest.raises(ValueError):
        po.pc1(np.zeros((3, 4), np.float32), np.zeros(4), np.zeros(5))
