"""Seeded synthetic inputs for the KNN filtering stage.

The paper's hyperspectral images (Table 1) and trained SVM models are not
available, so these generators stand in for them with the same shapes and a
similar structure: a normalised one-band image I (the first principal component)
and per-pixel class-probability maps P (the SVM output, pixels x classes).

This module holds input preparation only -- random draws, region layouts and a
softmax that turns logits into probability rows -- and none of the filter's own
arithmetic.  It is shared by the tests, the benchmark and the serving harness;
the oracle never imports it.

All generators use ``numpy.random.default_rng(seed)`` (PCG64) and return
C-contiguous float32 arrays ``pc1`` (H, W) and ``prob`` (H, W, C).  The softmax
is evaluated in float64 and cast once.

* ``g_unif``  -- I ~ U[0, 1), logits ~ N(0, 1).
* ``g_brain`` -- brain-like frames (four classes: tumour, healthy, blood,
  background; Sec. II.A): six Voronoi regions with smooth levels plus
  N(0, 0.02) noise; logits favour the region's class.
* ``g_cube`` / ``g_svm_model`` -- a hyperspectral cube with its PCA inputs,
  and a one-vs-one SVM model, for the two steps before the filter.
* ``g_derma`` -- dermatology-like frames (Sec. II.A, 50 x 50 snapshot sensor and
  1000 x 1000 fused images): an elliptical lesion on skin, two levels plus
  N(0, 0.02) noise; logits favour class 0 inside, class 1 outside.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

NUM_CLASSES = 4


def _softmax_f32(logits: np.ndarray) -> np.ndarray:
    z = logits.astype(np.float64)
    z = z - z.max(axis=-1, keepdims=True)
    ez = np.exp(z)
    return np.ascontiguousarray((ez / ez.sum(axis=-1, keepdims=True)).astype(np.float32))


def g_unif(H: int, W: int, seed: int, C: int = NUM_CLASSES):
    rng = np.random.default_rng(seed)
    pc1 = rng.random((H, W), dtype=np.float32)
    logits = rng.standard_normal((H, W, C), dtype=np.float32)
    return np.ascontiguousarray(pc1), _softmax_f32(logits)


def _gaussian_blur_reflect(img: np.ndarray, sigma: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter

    return gaussian_filter(img, sigma=sigma, mode="reflect")


def g_brain(H: int, W: int, seed: int, C: int = NUM_CLASSES, sites: int = 6):
    rng = np.random.default_rng(seed)
    sy = rng.uniform(0.0, H, size=sites)
    sx = rng.uniform(0.0, W, size=sites)
    mu = rng.uniform(0.15, 0.85, size=sites)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    d2 = (yy[None] - sy[:, None, None]) ** 2 + (xx[None] - sx[:, None, None]) ** 2
    label = np.argmin(d2, axis=0)  # ties go to the lower site index
    level = _gaussian_blur_reflect(mu[label], 2.0)
    pc1 = (level + rng.normal(0.0, 0.02, size=(H, W))).astype(np.float32)
    means = np.zeros((sites, C), np.float64)
    means[np.arange(sites), np.arange(sites) % C] = 2.0
    logits = means[label] + rng.standard_normal((H, W, C))
    return np.ascontiguousarray(pc1), _softmax_f32(logits)


def g_derma(H: int, W: int, seed: int, C: int = NUM_CLASSES):
    rng = np.random.default_rng(seed)
    cy = H / 2.0 + rng.uniform(-0.15, 0.15) * H
    cx = W / 2.0 + rng.uniform(-0.15, 0.15) * W
    ay = rng.uniform(0.2, 0.35) * H
    ax = rng.uniform(0.2, 0.35) * W
    th = rng.uniform(0.0, np.pi)
    mu_in = rng.uniform(0.2, 0.4)
    mu_out = rng.uniform(0.6, 0.8)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    u = (xx - cx) * np.cos(th) + (yy - cy) * np.sin(th)
    v = -(xx - cx) * np.sin(th) + (yy - cy) * np.cos(th)
    rho = np.sqrt((u / ax) ** 2 + (v / ay) ** 2)
    # signed distance to the ellipse edge, in pixels (approximate), and a
    # logistic ramp one pixel wide
    sd = (rho - 1.0) * min(ax, ay)
    w_in = 1.0 / (1.0 + np.exp(np.clip(sd, -60, 60)))
    level = w_in * mu_in + (1.0 - w_in) * mu_out
    pc1 = (level + rng.normal(0.0, 0.02, size=(H, W))).astype(np.float32)
    inside = w_in >= 0.5
    means = np.zeros((H, W, C), np.float64)
    means[inside, 0] = 2.0
    means[~inside, 1 % C] = 2.0
    logits = means + rng.standard_normal((H, W, C))
    return np.ascontiguousarray(pc1), _softmax_f32(logits)


GENERATORS = {"unif": g_unif, "brain": g_brain, "derma": g_derma}


def g_cube(H: int, W: int, B: int, seed: int, kind: str = "brain"):
    """A hyperspectral cube for the PC1 projection step, with the band
    averages and the first eigenvector it is given (the covariance and Jacobi
    steps are not part of the library).

    Regions as in ``g_brain`` (six Voronoi cells) or ``g_derma`` (lesion and
    skin); every region has a smooth reflectance spectrum in [0, 1] (a base
    curve plus two Gaussian bumps over the bands), scaled by a smooth
    illumination field, plus N(0, 0.01) noise.  ``mean`` is the base curve and
    ``vec`` the unit direction from the base curve to the first region's
    spectrum -- generator parameters, not statistics of the cube.

    Returns ``cube`` float32 [H*W, B] (pixel-major, bands contiguous),
    ``mean`` and ``vec`` float64 [B].
    """
    rng = np.random.default_rng(seed)
    bands = np.linspace(0.0, 1.0, B)
    base = 0.35 + 0.15 * np.sin(2.0 * np.pi * (bands * rng.uniform(0.6, 1.4) + rng.uniform(0, 1)))
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    if kind == "brain":
        sites = 6
        sy = rng.uniform(0.0, H, size=sites)
        sx = rng.uniform(0.0, W, size=sites)
        d2 = (yy[None] - sy[:, None, None]) ** 2 + (xx[None] - sx[:, None, None]) ** 2
        label = np.argmin(d2, axis=0)
    elif kind == "derma":
        sites = 2
        cy, cx = H / 2.0 + rng.uniform(-0.15, 0.15) * H, W / 2.0 + rng.uniform(-0.15, 0.15) * W
        ay, ax = rng.uniform(0.2, 0.35) * H, rng.uniform(0.2, 0.35) * W
        label = (((yy - cy) / ay) ** 2 + ((xx - cx) / ax) ** 2 > 1.0).astype(np.int64)
    else:
        raise ValueError(f"unknown cube kind {kind!r}")
    spectra = np.empty((sites, B))
    for k in range(sites):
        bump = np.zeros(B)
        for _ in range(2):
            c, w, a = rng.uniform(0.1, 0.9), rng.uniform(0.05, 0.2), rng.uniform(-0.25, 0.25)
            bump += a * np.exp(-0.5 * ((bands - c) / w) ** 2)
        spectra[k] = np.clip(base + bump, 0.0, 1.0)
    illum = 1.0 + 0.1 * np.sin(yy / max(H, 1) * rng.uniform(2, 6) + rng.uniform(0, 6)) \
        * np.cos(xx / max(W, 1) * rng.uniform(2, 6))
    cube = spectra[label] * illum[..., None] + rng.normal(0.0, 0.01, size=(H, W, B))
    direction = spectra[0] - base
    vec = direction / np.sqrt(np.sum(direction * direction))
    return (np.ascontiguousarray(cube.reshape(H * W, B).astype(np.float32)),
            np.ascontiguousarray(base), np.ascontiguousarray(vec))


def g_svm_model(C: int, B: int, seed: int):
    """A synthetic one-vs-one SVM model for the probability stage (the
    paper's trained models are not available): for every class pair (i, j),
    i < j, in lexicographic order, a hyperplane w ~ N(0, 1) * 40 / sqrt(B)
    (binary64), an offset that centres it on a flat 0.35 reflectance plus
    N(0, 0.5), and sigmoid parameters A ~ U[-2.5, -0.5], B ~ U[-0.3, 0.3].
    On ``g_cube`` cubes the decision values span a few units, so the binary
    probabilities cover (0, 1) and the coupling runs several sweeps.

    Returns ``w`` float64 [M, B], ``bias``, ``A``, ``B`` float64 [M],
    M = C (C - 1) / 2.
    """
    rng = np.random.default_rng(seed)
    M = C * (C - 1) // 2
    w = rng.normal(0.0, 1.0, (M, B)) * (40.0 / np.sqrt(B))
    bias = -0.35 * w.sum(axis=1) + rng.normal(0.0, 0.5, M)
    A = rng.uniform(-2.5, -0.5, M)
    Bp = rng.uniform(-0.3, 0.3, M)
    return (np.ascontiguousarray(w), np.ascontiguousarray(bias), np.ascontiguousarray(A),
            np.ascontiguousarray(Bp))


@dataclass(frozen=True)
class FrameSpec:
    """One frame of a workload: generator, shape, seed and filter parameters."""

    gen: str
    H: int
    W: int
    seed: int
    K: int
    R: int
    lam: float = 0.01
    C: int = NUM_CLASSES

    def make(self):
        return GENERATORS[self.gen](self.H, self.W, self.seed, self.C)

    @property
    def pixels(self) -> int:
        return self.H * self.W

    def pairs(self) -> int:
        """Candidate pairs evaluated by an exhaustive windowed scan."""
        tot = 0
        for r in range(self.H):
            rows = min(self.H - 1, r + self.R) - max(0, r - self.R) + 1
            tot += rows
        return tot * self.W * self.W


@dataclass
class Workload:
    name: str
    frames: list = field(default_factory=list)

    @property
    def pixels(self) -> int:
        return sum(f.pixels for f in self.frames)

    def pairs(self) -> int:
        return sum(f.pairs() for f in self.frames)


def config0() -> Workload:
    """One 64 x 64 uniform frame, K = 8, window +-4 rows, lambda = 0.01, seed 0."""
    return Workload("plain-64x64-unif-K8-R4", [FrameSpec("unif", 64, 64, 0, K=8, R=4)])


def config1() -> Workload:
    """One brain-like frame, width 480 x height 380, K = 40, +-14 rows, lambda 0.01."""
    return Workload("plain-brain-W480xH380-K40-R14",
                    [FrameSpec("brain", 380, 480, 0, K=40, R=14)])


def config2(n: int = 64) -> Workload:
    """64 brain-like frames with H, W uniform in [50, 1000], K = 40, +-14 rows."""
    sizes = np.random.default_rng(0).integers(50, 1001, size=(n, 2))
    return Workload("batch-64-uneven-brain-K40-R14",
                    [FrameSpec("brain", int(h), int(w), 1000 + i, K=40, R=14)
                     for i, (h, w) in enumerate(sizes)])


def config3(n: int = 1024) -> Workload:
    """1024 dermatology-like 50 x 50 frames, K = 16, +-7 rows."""
    return Workload("batch-1024-derma-50x50-K16-R7",
                    [FrameSpec("derma", 50, 50, 2000 + i, K=16, R=7) for i in range(n)])


SERVE_CLASSES = {
    "S": dict(gen="derma", H=50, W=50, K=16, R=7),
    "M": dict(gen="brain", H=380, W=480, K=40, R=14),
    "L": dict(gen="derma", H=1000, W=1000, K=40, R=14),
}


def serve_stream(n: int = 2000, rate_hz: float = 200.0, seed: int = 5,
                 probs=(0.70, 0.25, 0.05)):
    """Poisson arrivals with a 70/25/5 % mix of S/M/L frames.

    Returns a list of (arrival_seconds, class_name, FrameSpec).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    t = np.cumsum(gaps) - gaps[0]
    cls = rng.choice(np.array(list(SERVE_CLASSES.keys())), size=n, p=list(probs))
    out = []
    for i in range(n):
        c = str(cls[i])
        p = SERVE_CLASSES[c]
        out.append((float(t[i]), c, FrameSpec(p["gen"], p["H"], p["W"], 10000 + i,
                                              K=p["K"], R=p["R"])))
    return out
