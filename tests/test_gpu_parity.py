"""GPU parity: the HIP path against the CPU oracle, through the C-ABI.

Bar: neighbour indices, neighbour distances and the class map bit-exact; the
filtered probabilities within 1e-6 absolute (bit-exact is expected and is
reported).  Small frames are compared at every pixel; the full-size brain-like
frame (W 480 x H 380, K = 40, +-14 rows) at every pixel too.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_10631_amd import _lib, inputs
from paper_2404_10631_amd.frames import DeviceFrame, current_stream

pytestmark = pytest.mark.gpu

PROB_TOL = 1e-6

SHAPES = [(1, 8), (1, 16), (2, 4), (2, 8), (4, 4)]
EXH8 = dict(search=0, tile_rows=2, tile_cols=8, waves=2)
PRU8 = dict(search=1, tile_rows=2, tile_cols=8, waves=2)
# the two 8-query shapes (1 x 8 is the context's default)
PRU24 = dict(search=1, tile_rows=2, tile_cols=4, waves=1)
PRU18 = dict(search=1, tile_rows=1, tile_cols=8, waves=1)
TIE_PLANS = (EXH8, PRU8, PRU24, PRU18)
ALL_PLANS = [dict(search=s, tile_rows=r, tile_cols=c, waves=w)
             for s in (0, 1) for (r, c) in SHAPES for w in (1, 2, 4)]


def plan_id(p):
    return f"s{p['search']}t{p['tile_rows']}x{p['tile_cols']}w{p['waves']}"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "no GPU visible"
    c = _lib.knnf_create(0)
    yield c
    _lib.knnf_destroy(c)


def run_gpu(ctx, pc1, prob, K, R, lam, plan, with_nbr=True):
    import torch

    df = DeviceFrame(pc1, prob, K, R, lam, with_nbr=with_nbr)
    df.clear_outputs()
    _lib.knnf_filter(ctx, df.as_c(), plan, current_stream())
    torch.cuda.synchronize()
    return df.results()


def assert_parity(gpu, ref, label=""):
    go, gc, gn, gd = gpu
    ro, rc, rn, rd = ref
    if rn is not None:
        bad = np.argwhere(np.any(gn != rn, axis=-1))
        assert bad.size == 0, f"{label}: nbr differs at {bad[:5].tolist()} (of {len(bad)})"
        assert np.array_equal(gd.view(np.uint32), rd.view(np.uint32)), f"{label}: dist differs"
    assert np.array_equal(gc, rc), f"{label}: class differs at {np.argwhere(gc != rc)[:5].tolist()}"
    err = float(np.max(np.abs(go.astype(np.float64) - ro.astype(np.float64)))) if go.size else 0.0
    assert err <= PROB_TOL, f"{label}: prob max abs err {err}"
    return err


CASES = [
    # label, generator, H, W, K, R, lam
    ("one-pixel", "unif", 1, 1, 1, 0, 0.01),
    ("one-row-wide", "unif", 1, 70, 5, 0, 0.01),
    ("K-whole-frame", "unif", 3, 5, 15, 2, 0.01),
    ("K64-R0", "unif", 5, 200, 64, 0, 0.01),
    ("R-beyond-H", "brain", 17, 130, 40, 14, 0.01),
    ("one-column", "unif", 100, 1, 6, 5, 0.01),
    ("ragged-brain", "brain", 33, 129, 16, 7, 0.01),
    ("derma-50", "derma", 50, 50, 16, 7, 0.01),
    ("lambda-one", "unif", 25, 90, 12, 4, 1.0),
    ("tall-narrow", "brain", 150, 37, 40, 14, 0.01),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
@pytest.mark.parametrize("plan", [EXH8, PRU8, dict(search=1, tile_rows=4, tile_cols=4, waves=4),
                                  dict(search=0, tile_rows=1, tile_cols=16, waves=1),
                                  dict(search=1, tile_rows=1, tile_cols=8, waves=1)],
                         ids=plan_id)
def test_small_frames_bit_exact(ctx, case, plan):
    label, gen, H, W, K, R, lam = case
    pc1, prob = inputs.GENERATORS[gen](H, W, 31)
    say(f"case {label} H={H} W={W} K={K} R={R} lam={lam} plan={plan}")
    ref = oracle.knn_filter(pc1, prob, K, R, lam)
    assert_parity(run_gpu(ctx, pc1, prob, K, R, lam, plan), ref, label)


@pytest.mark.parametrize("plan", ALL_PLANS, ids=plan_id)
def test_config0_all_plans(ctx, plan):
    """One 64 x 64 uniform frame, K = 8, +-4 rows, lambda = 0.01, seed 0."""
    spec = inputs.config0().frames[0]
    pc1, prob = spec.make()
    say(f"config0 plan={plan}")
    ref = oracle.knn_filter(pc1, prob, spec.K, spec.R, spec.lam)
    assert_parity(run_gpu(ctx, pc1, prob, spec.K, spec.R, spec.lam, plan), ref, "config0")


def test_ties_constant_band_lambda_zero(ctx):
    """Every distance equal: the order is decided by the linear index alone."""
    H, W, K, R = 20, 70, 10, 3
    pc1 = np.full((H, W), 0.5, np.float32)
    _, prob = inputs.g_unif(H, W, 4)
    ref = oracle.knn_filter(pc1, prob, K, R, 0.0)
    for plan in TIE_PLANS:
        say(f"constant band lambda 0 plan={plan}")
        assert_parity(run_gpu(ctx, pc1, prob, K, R, 0.0, plan), ref, "const-l0")


def test_ties_dyadic(ctx):
    rng = np.random.default_rng(9)
    H, W, K, R = 31, 45, 24, 5
    pc1 = (rng.integers(0, 5, size=(H, W)) / 4.0).astype(np.float32)
    _, prob = inputs.g_unif(H, W, 5)
    ref = oracle.knn_filter(pc1, prob, K, R, 0.25)
    for plan in TIE_PLANS:
        say(f"dyadic ties plan={plan}")
        assert_parity(run_gpu(ctx, pc1, prob, K, R, 0.25, plan), ref, "dyadic")


def test_near_ties_low_bits(ctx):
    """Distances that differ only in their last mantissa bits: a fifth of the
    pixels sit near 0, the rest near 1 (offsets below 1e-5), lambda = 0, and K
    reaches into the near-1 group, whose order is decided by those bits."""
    rng = np.random.default_rng(21)
    H, W, K, R = 24, 40, 60, 2
    low = rng.random((H, W)) < 0.2
    pc1 = (np.where(low, 0.0, 1.0) + rng.random((H, W)) * 1e-5).astype(np.float32)
    _, prob = inputs.g_unif(H, W, 6)
    ref = oracle.knn_filter(pc1, prob, K, R, 0.0)
    for plan in TIE_PLANS:
        say(f"near ties plan={plan}")
        assert_parity(run_gpu(ctx, pc1, prob, K, R, 0.0, plan), ref, "near-ties")


@pytest.mark.parametrize("C", [1, 3, 16])
def test_class_counts(ctx, C):
    H, W, K, R = 19, 77, 12, 3
    pc1, prob = inputs.g_brain(H, W, 8, C=C)
    say(f"classes C={C}")
    ref = oracle.knn_filter(pc1, prob, K, R, 0.01)
    assert_parity(run_gpu(ctx, pc1, prob, K, R, 0.01, PRU8), ref, f"C{C}")


def test_without_neighbour_outputs(ctx):
    pc1, prob = inputs.g_brain(40, 90, 2)
    ref = oracle.knn_filter(pc1, prob, 20, 6, 0.01, with_nbr=False)
    say("no nbr outputs")
    assert_parity(run_gpu(ctx, pc1, prob, 20, 6, 0.01, EXH8, with_nbr=False), ref, "no-nbr")


@pytest.fixture(scope="module")
def config1_oracle():
    """The oracle over every pixel of the brain-like W 480 x H 380 frame
    (K = 40, +-14 rows): about 2.5e9 window distances, seconds on the host."""
    spec = inputs.config1().frames[0]
    pc1, prob = spec.make()
    say("config1: oracle over every pixel")
    return spec, pc1, prob, oracle.knn_filter(pc1, prob, spec.K, spec.R, spec.lam)


@pytest.mark.parametrize("plan", [EXH8, PRU8, PRU18], ids=["exhaustive", "pruned", "pruned-1x8"])
def test_config1_full_size_every_pixel(ctx, config1_oracle, plan):
    """Brain-like frame W 480 x H 380, K = 40, +-14 rows: every pixel against
    the oracle (neighbours, distances, classes bit-exact), plus the
    properties every pixel must have."""
    spec, pc1, prob, ref = config1_oracle
    say(f"config1 full size plan={plan}")
    go, gc, gn, gd = run_gpu(ctx, pc1, prob, spec.K, spec.R, spec.lam, plan)
    assert_parity((go, gc, gn, gd), ref, "config1")
    H, W = spec.H, spec.W
    lin = np.arange(H * W).reshape(H, W)
    assert np.array_equal(gn[..., 0], lin)
    assert np.all(gd[..., 0] == 0)
    assert np.all(np.diff(gd, axis=-1) >= 0)
    assert np.max(np.abs(go.astype(np.float64).sum(-1) - 1.0)) <= 1e-5
    rows = gn // W
    assert np.all(np.abs(rows - lin[..., None] // W) <= spec.R)


def test_exhaustive_equals_pruned_and_deterministic(ctx):
    spec = inputs.config1().frames[0]
    pc1, prob = spec.make()
    say("config1 exhaustive vs pruned vs repeat")
    a = run_gpu(ctx, pc1, prob, spec.K, spec.R, spec.lam, EXH8)
    b = run_gpu(ctx, pc1, prob, spec.K, spec.R, spec.lam, PRU8)
    c = run_gpu(ctx, pc1, prob, spec.K, spec.R, spec.lam, PRU8)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(y, z)


def test_batch_matches_single_frames_and_oracle(ctx):
    import torch

    specs = [inputs.FrameSpec("brain", 70, 130, 1, K=40, R=14),
             inputs.FrameSpec("derma", 50, 50, 2, K=16, R=7),
             inputs.FrameSpec("unif", 9, 300, 3, K=8, R=4),
             inputs.FrameSpec("derma", 50, 50, 4, K=16, R=7),
             inputs.FrameSpec("brain", 130, 61, 5, K=40, R=14),
             inputs.FrameSpec("unif", 1, 1, 6, K=1, R=0),
             inputs.FrameSpec("brain", 64, 64, 7, K=24, R=3, lam=0.05)]
    shapes = (EXH8, PRU8, dict(search=1, tile_rows=1, tile_cols=16, waves=1))
    for plan in [dict(p, launch=launch) for p in shapes for launch in (1, 2)]:
        say(f"batch of {len(specs)} plan={plan}")
        data = [s.make() for s in specs]
        batch = [DeviceFrame(p, q, s.K, s.R, s.lam) for s, (p, q) in zip(specs, data)]
        for df in batch:
            df.clear_outputs()
        _lib.knnf_filter_batch(ctx, [df.as_c() for df in batch], plan, current_stream())
        torch.cuda.synchronize()
        for s, (p, q), df in zip(specs, data, batch):
            got = df.results()
            single = run_gpu(ctx, p, q, s.K, s.R, s.lam, plan)
            for x, y in zip(got, single):
                assert np.array_equal(x, y)
            assert_parity(got, oracle.knn_filter(p, q, s.K, s.R, s.lam), f"batch {s}")


def test_batch_table_size_boundary(ctx):
    """Tables of up to 39 work items reach the device as a kernel argument,
    larger ones through a copy: batches of 38..41 small frames of different
    shapes, both launch modes, each frame bitwise equal to its own launch."""
    import torch

    rng = np.random.default_rng(21)
    for n in (38, 39, 40, 41):
        specs = [inputs.FrameSpec("unif", int(rng.integers(3, 20)), int(rng.integers(8, 40)), 100 + k,
                                  K=int(rng.integers(1, 9)), R=int(rng.integers(1, 4)))
                 for k in range(n)]
        data = [s.make() for s in specs]
        singles = [run_gpu(ctx, p, q, s.K, s.R, s.lam, PRU18) for s, (p, q) in zip(specs, data)]
        for launch in (1, 2):
            plan = dict(PRU18, launch=launch)
            say(f"batch of {n} frames, launch mode {launch}")
            batch = [DeviceFrame(p, q, s.K, s.R, s.lam) for s, (p, q) in zip(specs, data)]
            for df in batch:
                df.clear_outputs()
            _lib.knnf_filter_batch(ctx, [df.as_c() for df in batch], plan, current_stream())
            torch.cuda.synchronize()
            for k, df in enumerate(batch):
                for x, y in zip(df.results(), singles[k]):
                    assert np.array_equal(x, y), f"batch of {n}, frame {k}, launch {launch}"
        for k in (0, n - 1):
            s, (p, q) = specs[k], data[k]
            assert_parity(singles[k], oracle.knn_filter(p, q, s.K, s.R, s.lam), f"frame {k}")


def test_invalid_frame_is_rejected_before_launch(ctx):
    pc1, prob = inputs.g_unif(4, 4, 0)
    df = DeviceFrame(pc1, prob, 9, 0, 0.01)  # K = 9 > window of 4
    with pytest.raises(_lib.KnnfError) as ei:
        _lib.knnf_filter(ctx, df.as_c(), None, current_stream())
    assert ei.value.status == _lib.KNNF_EINVAL
    with pytest.raises(_lib.KnnfError):
        _lib.knnf_filter_batch(ctx, [df.as_c()], None, current_stream())


def test_single_hip_runtime_loaded(ctx):
    maps = open("/proc/self/maps").read()
    libs = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(libs) == 1, libs
    assert any("libknnf.so" in line for line in maps.splitlines())


def test_work_counters(ctx):
    """Exhaustive search evaluates every window pair (plus 64 pass-A block
    slots per pixel); the pruned search evaluates fewer and gives the same
    outputs."""
    import torch

    spec = inputs.FrameSpec("brain", 96, 150, 3, K=40, R=14)
    pc1, prob = spec.make()
    df = DeviceFrame(pc1, prob, spec.K, spec.R, spec.lam)
    _lib.knnf_stats_enable(ctx, True)
    try:
        _lib.knnf_stats_read(ctx, reset=True)
        _lib.knnf_filter(ctx, df.as_c(), EXH8, current_stream())
        pe, te = _lib.knnf_stats_read(ctx, reset=True)
        _lib.knnf_filter(ctx, df.as_c(), PRU8, current_stream())
        pp, tp = _lib.knnf_stats_read(ctx, reset=True)
    finally:
        _lib.knnf_stats_enable(ctx, False)
    torch.cuda.synchronize()
    assert pe == spec.pairs() + 64 * spec.pixels
    tiles = ((spec.H + 1) // 2) * ((spec.W + 7) // 8)
    assert te == tp == tiles
    assert pp < pe


def test_lambda_zero_spectral_only(ctx):
    """lambda = 0: the K nearest PC1 values in the window (a realistic band,
    so distances tie only by value), both searches, every pixel."""
    pc1, prob = inputs.g_brain(60, 90, 12)
    ref = oracle.knn_filter(pc1, prob, 16, 7, 0.0)
    for plan in (PRU24, EXH8):
        say(f"lambda 0 realistic band plan={plan}")
        assert_parity(run_gpu(ctx, pc1, prob, 16, 7, 0.0, plan), ref, "lambda0")


def test_unwindowed_whole_frame(ctx):
    """R beyond the frame: every pixel of the frame is a candidate (the
    paper's base definition without a window), every pixel compared."""
    pc1, prob = inputs.g_brain(96, 128, 13)
    ref = oracle.knn_filter(pc1, prob, 40, 500, 0.01)
    for plan in (PRU24, EXH8):
        say(f"unwindowed 96x128 plan={plan}")
        assert_parity(run_gpu(ctx, pc1, prob, 40, 500, 0.01, plan), ref, "unwindowed")


def test_frame_past_24_bit_indices_sampled(ctx):
    """W 4100 x H 4100 (16.81 M pixels, past 2^24): the linear indices no
    longer fit the 24-bit multiply-adds of the Eq. 2 gathers and output
    stores, so their 64-bit address paths run.  Default pruned plan; the
    first and last 64 pixels and 200 random ones against the oracle."""
    H = W = 4100
    K, R, lam = 8, 2, 0.01
    assert H * W > 1 << 24
    pc1, prob = inputs.g_unif(H, W, 41)
    say("past 2^24 pixels")
    go, gc, gn, gd = run_gpu(ctx, pc1, prob, K, R, lam, PRU18)
    rng = np.random.default_rng(41)
    pix = np.concatenate([np.arange(64), np.arange(H * W - 64, H * W),
                          rng.choice(H * W, 200, replace=False)])
    ro, rc, rn, rd = oracle.knn_pixels(pc1, prob, K, R, lam, pix)
    assert np.array_equal(gn.reshape(H * W, K)[pix], rn)
    assert np.array_equal(gd.reshape(H * W, K)[pix].view(np.uint32), rd.view(np.uint32))
    assert np.array_equal(gc.reshape(-1)[pix], rc)
    assert float(np.max(np.abs(go.reshape(H * W, -1)[pix].astype(np.float64) - ro))) <= PROB_TOL


def test_unwindowed_full_size_sampled(ctx):
    """W 480 x H 380, K = 40, whole-frame window, pruned search: 300 sampled
    pixels against the oracle (182,400 candidates each)."""
    spec = inputs.config1().frames[0]
    pc1, prob = spec.make()
    H, W, K, R = spec.H, spec.W, 40, spec.H - 1
    say("unwindowed full size")
    go, gc, gn, gd = run_gpu(ctx, pc1, prob, K, R, spec.lam, PRU24)
    pix = np.random.default_rng(31).choice(H * W, 300, replace=False)
    ro, rc, rn, rd = oracle.knn_pixels(pc1, prob, K, R, spec.lam, pix)
    assert np.array_equal(gn.reshape(H * W, K)[pix], rn)
    assert np.array_equal(gc.reshape(-1)[pix], rc)
    assert np.array_equal(gd.reshape(H * W, K)[pix].view(np.uint32), rd.view(np.uint32))
    assert float(np.max(np.abs(go.reshape(H * W, -1)[pix].astype(np.float64) - ro))) <= PROB_TOL
