"""CPU oracle for the SVM probability stage -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never imports it, and it
imports nothing from there.

What it computes (the probability maps P that the KNN filter averages): the
classification stage of the one-vs-one SVM of Sec. II.C.1, pixel by pixel, in
three steps (Sec. II.C.1; Sec. III.A.1 and III.B.1 for the GPU versions):

(i)   decision values: the distance of every pixel spectrum to every binary
      hyperplane, one matrix product of the image with the hyperplane matrix
      (Sec. III.A.1, III.B.1): f[p][m] = sum_b w[m][b] * x[p][b] + bias[m];
(ii)  binary probabilities: a sigmoid of the decision value (the adapted
      sigmoid of the SVM reference the paper cites, i.e. Platt's form),
      r = 1 / (1 + exp(A[m] * f + B[m])) for the first class of the pair and
      1 - r for the second;
(iii) multiclass probabilities by pairwise coupling (the method of Wu, Lin and
      Weng the paper cites as [30], their second method): minimise p^T Q p over
      the probability simplex with Q[t][t] = sum_{s != t} r[s][t]^2 and
      Q[t][j] = -r[j][t] * r[t][j], by the fixed-point sweep
      p[t] <- (p^T Q p - sum_{j != t} Q[t][j] p[j]) / Q[t][t], each update
      followed by renormalising p to sum 1, starting from the uniform p.

Readings where the paper is silent (each stated again where it is used):
* the training (hyperplanes, bias, sigmoid parameters) is offline and not in
  the paper; the model is an input.  Hyperplane m covers the class pair
  (i, j), i < j, in lexicographic order (0,1), (0,2), ..., (0,C-1), (1,2), ...;
  a positive decision value favours class i when A[m] < 0;
* binary probabilities are clamped to [1e-7, 1 - 1e-7] so that Q[t][t] > 0;
* the iteration stops when max_t |(Q p)[t] - p^T Q p| < 0.005 / C (the
  optimality condition of the coupling problem, within a tolerance) or after
  100 sweeps -- the paper names a threshold and a maximum without values;
* every step is evaluated in binary64 (the image is binary32, the model
  binary64), and the probabilities are rounded once to binary32 at the end,
  class fastest -- the layout the filter reads.

Pinned by ``tests/test_svm_oracle_pins.py``: exact rational decision values on
tiny cubes, the sigmoid's special values, consistent pairwise probabilities
(r[i][j] = p[i] / (p[i] + p[j])) whose p is the coupling's exact fixed point,
the two-class closed form, a brute-force minimisation of p^T Q p on the
simplex, and class relabelling.
"""
from __future__ import annotations

import numpy as np

CLAMP = 1e-7
MAX_SWEEPS = 100


def pairs(C: int):
    """The class pair of every hyperplane, in order: (0,1), (0,2), ..., (C-2,C-1)."""
    return [(i, j) for i in range(C) for j in range(i + 1, C)]


def decision(cube, w, bias) -> np.ndarray:
    """Step (i): f[p][m] = sum_b w[m][b] * x[p][b] + bias[m] in binary64, [P, M]."""
    x = np.asarray(cube, dtype=np.float32).astype(np.float64)
    wm = np.asarray(w, dtype=np.float64)
    b = np.asarray(bias, dtype=np.float64)
    if x.ndim != 2 or wm.ndim != 2 or wm.shape[1] != x.shape[1] or b.shape != (wm.shape[0],):
        raise ValueError("cube [P, B], w [M, B], bias [M]")
    return x @ wm.T + b[None, :]


def binary_prob(f, A, B) -> np.ndarray:
    """Step (ii): r = 1 / (1 + exp(A f + B)) per hyperplane, clamped to
    [1e-7, 1 - 1e-7]; the probability of the pair's first class."""
    z = np.asarray(f, dtype=np.float64) * np.asarray(A, np.float64)[None, :] \
        + np.asarray(B, np.float64)[None, :]
    with np.errstate(over="ignore"):
        r = 1.0 / (1.0 + np.exp(z))
    return np.clip(r, CLAMP, 1.0 - CLAMP)


def pairwise_matrix(r, C: int) -> np.ndarray:
    """R[p][i][j] = r_ij, the probability of class i within the pair {i, j}:
    r for i < j, 1 - r for i > j; the diagonal is unused (0)."""
    P = r.shape[0]
    R = np.zeros((P, C, C))
    for m, (i, j) in enumerate(pairs(C)):
        R[:, i, j] = r[:, m]
        R[:, j, i] = 1.0 - r[:, m]
    return R


def coupling_matrix(R) -> np.ndarray:
    """Q[t][t] = sum_{s != t} r_st^2, Q[t][j] = -r_jt r_tj (j != t)."""
    P, C, _ = R.shape
    Q = np.empty_like(R)
    for t in range(C):
        for j in range(C):
            if j == t:
                Q[:, t, t] = sum(R[:, s, t] ** 2 for s in range(C) if s != t)
            else:
                Q[:, t, j] = -R[:, j, t] * R[:, t, j]
    return Q


def couple(R, max_sweeps: int = MAX_SWEEPS, p0=None, eps=None):
    """Step (iii) for every pixel at once (each pixel iterates on its own and
    stops on its own).  ``eps`` defaults to 0.005 / C (tests pass a tighter
    one to compare with a direct minimisation).  Returns (p [P, C] binary64,
    sweeps done [P])."""
    P, C, _ = R.shape
    Q = coupling_matrix(R)
    eps = 0.005 / C if eps is None else eps
    p = np.full((P, C), 1.0 / C) if p0 is None else np.array(p0, dtype=np.float64)
    sweeps = np.zeros(P, dtype=np.int64)
    for _ in range(max_sweeps):
        Qp = np.einsum("ptj,pj->pt", Q, p)
        pQp = np.einsum("pt,pt->p", p, Qp)
        active = np.max(np.abs(Qp - pQp[:, None]), axis=1) >= eps
        if not active.any():
            break
        sweeps += active
        for t in range(C):
            pQp = np.einsum("pt,ptj,pj->p", p, Q, p)
            off = sum(Q[:, t, j] * p[:, j] for j in range(C) if j != t)
            new_t = (pQp - off) / Q[:, t, t]
            q = p.copy()
            q[:, t] = new_t
            q = q / q.sum(axis=1, keepdims=True)
            p = np.where(active[:, None], q, p)
    return p, sweeps


def svm_prob(cube, w, bias, A, B, C: int) -> np.ndarray:
    """Probability maps of a [P, bands] cube, binary32 [P, C] (class fastest)."""
    M = C * (C - 1) // 2
    if np.asarray(w).shape[0] != M:
        raise ValueError(f"{C} classes need {M} hyperplanes")
    r = binary_prob(decision(cube, w, bias), A, B)
    p, _ = couple(pairwise_matrix(r, C))
    return p.astype(np.float32)
