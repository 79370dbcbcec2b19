"""Pins of the oracles against worked examples derived by hand with exact
rationals (``tests/golden/derive.py`` writes them; it calls neither the oracle
nor the library).

* ``eq1_lambda001.txt``: Eq. 1 (Sec. II.C.3) at lambda = 0.01, every binary32
  rounding of the evaluation order written out.  The cases were chosen so that
  each plausible alternative order gives other bits: the fused multiply-adds
  nested the other way, the spectral or column term hoisted instead of the row
  term, no fused operations, one rounding of the exact sum, lambda applied to
  the coordinate difference, lambda * x fused into the subtraction, lambda
  taken as the binary64 0.01, and lambda^2 factored out of the spatial terms.
* ``coupling_3class.txt``: the pairwise coupling of Sec. II.C.1 sweep by
  sweep, so the stopping threshold (0.005 / C) and the sweep count are fixed:
  with 0.005 instead the coupling stops one sweep earlier, 2.6e-3 away.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import svm_oracle as so

GOLDEN = os.path.dirname(os.path.abspath(__file__)) + "/golden"


def read_eq1():
    cases = []
    for line in open(os.path.join(GOLDEN, "eq1_lambda001.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, tail = line.split(":")
        r, c, iq, i, j, ip = head.split()
        d_hex, bits = tail.split()
        cases.append((int(r), int(c), float.fromhex(iq), int(i), int(j), float.fromhex(ip),
                      float.fromhex(d_hex), int(bits, 16)))
    return cases


EQ1 = read_eq1()


def eq1_frame(case, H=40, W=480):
    """A frame where the case's candidate is the query's nearest other pixel:
    every other pixel has I = 10 (its spectral term alone exceeds 80)."""
    r, c, iq, i, j, ip, _, _ = case
    pc1 = np.full((H, W), 10.0, np.float32)
    pc1[r, c] = np.float32(iq)
    pc1[i, j] = np.float32(ip)
    prob = np.full((H, W, 2), 0.5, np.float32)
    return pc1, prob


def test_eq1_golden_covers_the_frame():
    assert len(EQ1) == 7
    for r, c, iq, i, j, ip, d, bits in EQ1:
        assert np.float32(iq) == iq and np.float32(ip) == ip
        assert np.float32(d).view(np.uint32) == bits
        assert abs(r - i) <= 3 and 0 <= min(r, i, c, j) and max(r, i) < 40 and max(c, j) < 480


@pytest.mark.parametrize("case", EQ1, ids=lambda c: f"q{c[0]}_{c[1]}-p{c[3]}_{c[4]}")
def test_eq1_lambda001_hand_derived(case):
    r, c, iq, i, j, ip, d, bits = case
    W = 480
    pc1, prob = eq1_frame(case)
    q, p = r * W + c, i * W + j
    _, _, nbr, dist = oracle.knn_pixels(pc1, prob, 2, 3, 0.01, [q, p])
    assert nbr[0].tolist() == [q, p] and nbr[1].tolist() == [p, q]
    assert dist[0].view(np.uint32)[1] == bits, f"{dist[0][1].hex()} != {d.hex()}"
    assert dist[1].view(np.uint32)[1] == bits  # the distance is symmetric bitwise


def read_coupling():
    rows = []
    for line in open(os.path.join(GOLDEN, "coupling_3class.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, tail = line.split("|")
        r = [float(eval(x)) for x in head.split()]  # small fractions such as 3/5
        t = tail.split()
        rows.append((tuple(r), t[0], int(t[1]), np.array([float(x) for x in t[2:]])))
    return rows


COUPLING = read_coupling()


@pytest.mark.parametrize("row", COUPLING, ids=lambda x: f"{x[0]}-{x[1]}")
def test_coupling_stop_rule_hand_derived(row):
    r, eps_label, sweeps, p_want = row
    R = so.pairwise_matrix(np.array([r]), 3)
    if eps_label == "0.005/3":
        p, s = so.couple(R)                  # the default rule
    else:
        p, s = so.couple(R, eps=0.005)
    assert int(s[0]) == sweeps
    assert np.max(np.abs(p[0] - p_want)) <= 1e-12


def test_coupling_thresholds_are_distinguishable():
    by = {}
    for r, eps_label, sweeps, p in COUPLING:
        by.setdefault(r, {})[eps_label] = (sweeps, p)
    for r, d in by.items():
        (s1, p1), (s2, p2) = d["0.005/3"], d["0.005"]
        assert s1 == s2 + 1 and np.max(np.abs(p1 - p2)) > 1e-3


def sigmoid_model_for(r):
    """A zero-weight 3-class model whose binary probabilities are r: with
    f = bias = 0, 1 / (1 + exp(B)) = r for B = ln((1 - r) / r)."""
    M, bands = 3, 4
    w = np.zeros((M, bands))
    bias = np.zeros(M)
    A = -np.ones(M)
    B = np.array([math.log((1.0 - x) / x) for x in r])
    return w, bias, A, B


def test_svm_prob_uses_the_default_stop_rule():
    """The whole SVM stage (decision values, sigmoid, coupling) on such a model
    returns the hand-derived 0.005 / C fixed point, rounded to binary32."""
    for r, eps_label, _, p_want in COUPLING:
        if eps_label != "0.005/3":
            continue
        x = np.random.default_rng(0).uniform(0, 1, (5, 4)).astype(np.float32)
        out = so.svm_prob(x, *sigmoid_model_for(r), 3)
        assert np.max(np.abs(out.astype(np.float64) - p_want[None, :])) <= 1e-7


def test_sweep_cap_never_binds_for_clamped_probabilities():
    """The 100-sweep cap is a guard: for binary probabilities inside the clamp
    the 0.005 / C rule stops within a handful of sweeps (random, extreme and
    cyclic inputs for 3 to 8 classes), so the cap's value never reaches the
    outputs."""
    rng = np.random.default_rng(2)
    worst = 0
    for C in (3, 4, 6, 8):
        M = C * (C - 1) // 2
        rs = [rng.uniform(0, 1, (400, M)),
              np.where(rng.random((400, M)) < 0.5, 10 ** rng.uniform(-7, 0, (400, M)),
                       1 - 10 ** rng.uniform(-7, 0, (400, M))),
              rng.choice([so.CLAMP, 1 - so.CLAMP, 0.5, 1e-3, 1 - 1e-3], (400, M))]
        for r in rs:
            r = np.clip(r, so.CLAMP, 1 - so.CLAMP)
            _, s = so.couple(so.pairwise_matrix(r, C))
            worst = max(worst, int(s.max()))
    assert worst <= 10 < so.MAX_SWEEPS
