"""Pins for the SVM probability oracle (CPU): exact rational decision values,
the sigmoid's special values, the orientation of the pairwise matrix, the
coupling's exact fixed point for consistent pairwise probabilities, the
two-class closed form, a direct minimisation of the coupling objective on the
simplex, and class relabelling."""
from fractions import Fraction

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import svm_oracle as so


def consistent_r(p):
    """r_ij = p_i / (p_i + p_j): pairwise probabilities that agree exactly with p."""
    C = len(p)
    R = np.zeros((1, C, C))
    for i in range(C):
        for j in range(C):
            if i != j:
                R[0, i, j] = p[i] / (p[i] + p[j])
    return R


def test_pairs_are_lexicographic():
    assert so.pairs(4) == [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    assert so.pairs(2) == [(0, 1)]


def test_decision_matches_exact_rational_arithmetic():
    rng = np.random.default_rng(3)
    P, B, M = 5, 7, 3
    x = rng.uniform(0, 1, (P, B)).astype(np.float32)
    w = rng.normal(0, 1, (M, B))
    bias = rng.normal(0, 1, M)
    f = so.decision(x, w, bias)
    for p in range(P):
        for m in range(M):
            exact = sum(Fraction(float(w[m, b])) * Fraction(float(x[p, b])) for b in range(B)) \
                + Fraction(float(bias[m]))
            mag = sum(abs(float(w[m, b]) * float(x[p, b])) for b in range(B)) + abs(bias[m])
            assert abs(f[p, m] - float(exact)) <= (B + 2) * 2.0 ** -53 * mag


def test_sigmoid_special_values():
    A = np.array([-2.0, -1.0, 3.0])
    B = np.array([0.0, np.log(3.0), 0.0])
    f = np.array([[0.0, 0.0, 0.0]])
    r = so.binary_prob(f, A, B)
    assert r[0, 0] == 0.5                       # A f + B = 0
    assert abs(r[0, 1] - 0.25) < 1e-15          # exp(ln 3) = 3
    big = so.binary_prob(np.array([[1e4, -1e4, 1e4]]), A, np.zeros(3))
    assert big[0, 0] == 1.0 - so.CLAMP and big[0, 1] == so.CLAMP and big[0, 2] == so.CLAMP
    # decreasing in A f + B
    zs = np.linspace(-5, 5, 11)[:, None]
    rr = so.binary_prob(zs, np.array([1.0]), np.array([0.0]))[:, 0]
    assert np.all(np.diff(rr) < 0)


def test_pairwise_matrix_orientation():
    r = np.array([[0.9, 0.2, 0.6]])  # pairs (0,1), (0,2), (1,2)
    R = so.pairwise_matrix(r, 3)[0]
    assert R[0, 1] == 0.9 and R[1, 0] == pytest.approx(0.1)
    assert R[0, 2] == 0.2 and R[2, 0] == pytest.approx(0.8)
    assert R[1, 2] == 0.6 and R[2, 1] == pytest.approx(0.4)


@pytest.mark.parametrize("C", [2, 3, 4])
def test_consistent_probabilities_are_the_fixed_point(C):
    rng = np.random.default_rng(10 + C)
    p = rng.dirichlet(np.ones(C))
    R = consistent_r(p)
    Q = so.coupling_matrix(R)[0]
    Qp = Q @ p
    # (Q p)_t is the same for every t and equals p^T Q p = 0
    assert np.max(np.abs(Qp)) < 1e-15 and abs(p @ Qp) < 1e-15
    got, sweeps = so.couple(R, p0=p[None, :])
    assert sweeps[0] == 0 and np.array_equal(got[0], p)
    got, sweeps = so.couple(R, eps=1e-13, max_sweeps=5000)
    assert np.max(np.abs(got[0] - p)) < 1e-10
    got, sweeps = so.couple(R)
    assert 0 < sweeps[0] <= so.MAX_SWEEPS and np.argmax(got[0]) == np.argmax(p)
    assert np.max(np.abs(got[0] - p)) < 0.02


@pytest.mark.parametrize("r", [0.5, 0.8, 0.03, so.CLAMP])
def test_two_classes_closed_form(r):
    """With two classes the coupling returns (r, 1 - r)."""
    R = so.pairwise_matrix(np.array([[r]]), 2)
    got, _ = so.couple(R, eps=1e-14, max_sweeps=5000)
    assert np.max(np.abs(got[0] - [r, 1 - r])) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_coupling_minimises_the_objective(seed):
    """Inconsistent random pairwise probabilities: the fixed point equals the
    minimiser of p^T Q p on the simplex found by a general-purpose solver."""
    C = 4
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.02, 0.98, (1, C * (C - 1) // 2))
    R = so.pairwise_matrix(r, C)
    Q = so.coupling_matrix(R)[0]
    res = minimize(lambda q: q @ Q @ q, np.full(C, 1.0 / C), method="SLSQP",
                   bounds=[(0, 1)] * C, constraints=[{"type": "eq", "fun": lambda q: q.sum() - 1}],
                   options={"ftol": 1e-15, "maxiter": 1000})
    got, _ = so.couple(R, eps=1e-13, max_sweeps=5000)
    assert np.max(np.abs(got[0] - res.x)) < 1e-5
    # the default stopping rule stays close to it
    dflt, _ = so.couple(R)
    assert np.max(np.abs(dflt[0] - res.x)) < 0.02


def test_relabelling_classes_permutes_the_output():
    """Renaming the classes by a permutation renames the probabilities: a pair
    whose order flips takes the complementary sigmoid (A, B negated)."""
    C, nb = 4, 6
    rng = np.random.default_rng(21)
    x = rng.uniform(0, 1, (9, nb)).astype(np.float32)
    w = rng.normal(0, 2, (6, nb)).astype(np.float32)
    bias, A, B = rng.normal(0, 1, 6), -rng.uniform(1, 3, 6), rng.normal(0, 0.3, 6)
    perm = [2, 0, 3, 1]  # old class k is new class perm[k]
    idx = {pr: m for m, pr in enumerate(so.pairs(C))}
    w2, bias2, A2, B2 = np.empty_like(w), np.empty(6), np.empty(6), np.empty(6)
    for m, (i, j) in enumerate(so.pairs(C)):
        a, b = perm[i], perm[j]
        n = idx[(min(a, b), max(a, b))]
        sgn = 1.0 if a < b else -1.0
        w2[n], bias2[n], A2[n], B2[n] = w[m], bias[m], sgn * A[m], sgn * B[m]
    def probs(w_, b_, A_, B_):
        R = so.pairwise_matrix(so.binary_prob(so.decision(x, w_, b_), A_, B_), C)
        return so.couple(R, eps=1e-13, max_sweeps=5000)[0]
    p1 = probs(w, bias, A, B)
    p2 = probs(w2, bias2, A2, B2)
    assert np.max(np.abs(p2[:, perm] - p1)) < 1e-9


def test_svm_prob_shapes_and_simplex():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (50, 16)).astype(np.float32)
    w = rng.normal(0, 1, (6, 16)).astype(np.float32)
    out = so.svm_prob(x, w, rng.normal(0, 1, 6), -np.ones(6), np.zeros(6), 4)
    assert out.dtype == np.float32 and out.shape == (50, 4)
    assert np.all(out > 0) and np.allclose(out.sum(axis=1), 1.0, atol=1e-6)
    with pytest.raises(ValueError):
        so.svm_prob(x, w[:5], np.zeros(5), np.ones(5), np.zeros(5), 4)
