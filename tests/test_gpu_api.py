"""GPU checks of the C-ABI's error conventions, window-chunk plans and the
autotuner's plan cache.

* Non-finite pc1 or prob values are rejected with KNNF_EINVAL before any
  filtering work is enqueued (outputs and work counters untouched), by
  knnf_filter, knnf_filter_batch and knnf_server_submit.
* A failed context stays failed: every later call returns KNNF_EDEVICE
  (forced from the host with knnf_inject_fault; no kernel is made to fail).
* Every window chunk of the pruned search gives the oracle's bits.
* knnf_tune caches the plan it picks per frame key, writes it to the JSON file
  named by KNNF_TUNE_CACHE, later contexts load it, and calls without a plan
  use it -- with outputs bitwise equal to the default plan's.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2404_10631_amd import _lib, inputs
from paper_2404_10631_amd.frames import DeviceFrame, current_stream
from paper_2404_10631_amd.serve import HostFrame, Server

pytestmark = pytest.mark.gpu

NOCHECK = _lib.KNNF_PLAN_NO_INPUT_CHECK


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


def untouched(df):
    go, gc, gn, gd = df.results()
    return all(np.all(a.view(np.uint8) == 0x7f) for a in (go, gc, gn, gd))


@pytest.mark.parametrize("where", ["pc1-nan", "pc1-inf", "prob-nan", "prob-neginf"])
def test_non_finite_input_rejected_before_launch(ctx, where):
    import torch

    pc1, prob = inputs.g_brain(40, 70, 1)
    if where.startswith("pc1"):
        pc1[17, 33] = np.nan if where.endswith("nan") else np.inf
    else:
        prob[39, 69, 3] = np.nan if where.endswith("nan") else -np.inf
    df = DeviceFrame(pc1, prob, 16, 5, 0.01)
    df.clear_outputs()
    good = DeviceFrame(*inputs.g_brain(30, 50, 2), 16, 5, 0.01)
    good.clear_outputs()
    _lib.knnf_stats_enable(ctx, True)
    try:
        _lib.knnf_stats_read(ctx, reset=True)
        say(f"non-finite input {where}: knnf_filter")
        with pytest.raises(_lib.KnnfError) as ei:
            _lib.knnf_filter(ctx, df.as_c(), None, current_stream())
        assert ei.value.status == _lib.KNNF_EINVAL and "non-finite" in str(ei.value)
        say(f"non-finite input {where}: knnf_filter_batch")
        for launch in (1, 2):
            with pytest.raises(_lib.KnnfError) as ei:
                _lib.knnf_filter_batch(ctx, [good.as_c(), df.as_c()], dict(search=1, launch=launch),
                                       current_stream())
            assert ei.value.status == _lib.KNNF_EINVAL
        torch.cuda.synchronize()
        _, tiles = _lib.knnf_stats_read(ctx, reset=True)
    finally:
        _lib.knnf_stats_enable(ctx, False)
    assert tiles == 0
    assert untouched(df) and untouched(good)
    assert _lib.knnf_ctx_status(ctx) == _lib.KNNF_OK  # EINVAL leaves the context usable
    # the same frames with finite values pass the check and match the oracle
    ok = DeviceFrame(*inputs.g_brain(40, 70, 1), 16, 5, 0.01)
    _lib.knnf_filter(ctx, ok.as_c(), None, current_stream())
    torch.cuda.synchronize()
    ref = oracle.knn_filter(*inputs.g_brain(40, 70, 1), 16, 5, 0.01)
    got = ok.results()
    assert np.array_equal(got[2], ref[2]) and np.array_equal(got[1], ref[1])


def test_server_rejects_non_finite_host_input(ctx):
    pc1, prob = inputs.g_derma(50, 50, 3)
    prob[7, 9, 1] = np.nan
    hf = HostFrame(pc1, prob, 16, 7, 0.01)
    with Server(ctx, 64 << 20) as srv:
        say("server submit with a NaN probability")
        with pytest.raises(_lib.KnnfError) as ei:
            _lib.knnf_server_submit(srv.handle, hf.as_c())
        assert ei.value.status == _lib.KNNF_EINVAL
    with Server(ctx, 64 << 20, plan=dict(search=1, flags=NOCHECK)) as srv:
        # the caller vouches for its inputs: no host check (finite frame here)
        ok = HostFrame(*inputs.g_derma(50, 50, 3), 16, 7, 0.01)
        st, tk = _lib.knnf_server_submit(srv.handle, ok.as_c())
        assert st == _lib.KNNF_OK
        _lib.knnf_server_drain(srv.handle, 30.0)
        _lib.knnf_server_release(srv.handle, tk)


def test_failed_context_is_sticky():
    import torch

    c = _lib.knnf_create(0)
    try:
        df = DeviceFrame(*inputs.g_unif(16, 16, 1), 4, 2, 0.01)
        _lib.knnf_filter(c, df.as_c(), None, current_stream())
        torch.cuda.synchronize()
        pool = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
        opts = _lib.knnf_server_opts()
        srv = _lib.knnf_server_create(c, pool.data_ptr(), pool.numel(), opts)
        assert _lib.knnf_ctx_status(c) == _lib.KNNF_OK
        say("inject a device failure into a context")
        _lib.knnf_inject_fault(c)
        assert _lib.knnf_ctx_status(c) == _lib.KNNF_EDEVICE
        for call in (lambda: _lib.knnf_filter(c, df.as_c(), None, current_stream()),
                     lambda: _lib.knnf_filter_batch(c, [df.as_c()], None, current_stream()),
                     lambda: _lib.knnf_tune(c, [df.as_c()], 1, current_stream()),
                     lambda: _lib.knnf_stats_enable(c, True),
                     lambda: _lib.knnf_server_submit(srv, HostFrame(*inputs.g_unif(16, 16, 1), 4, 2,
                                                                    0.01).as_c())):
            with pytest.raises(_lib.KnnfError) as ei:
                call()
            assert ei.value.status == _lib.KNNF_EDEVICE
            assert "failed" in str(ei.value)
        with pytest.raises(_lib.KnnfError) as ei:
            _lib.knnf_server_drain(srv, 1.0)
        assert ei.value.status == _lib.KNNF_EDEVICE
        _lib.knnf_server_destroy(srv)
    finally:
        _lib.knnf_destroy(c)


@pytest.mark.parametrize("chunk", [8, 16, 32])
def test_window_chunks_bit_exact(ctx, chunk):
    cases = [("brain", 33, 129, 16, 7, 0.01), ("unif", 25, 90, 12, 4, 1.0),
             ("brain", 17, 130, 40, 14, 0.01), ("unif", 1, 70, 5, 0, 0.01),
             ("brain", 60, 90, 16, 7, 0.0)]
    for shape in ((1, 8), (2, 4), (4, 4), (1, 16)):
        plan = dict(search=1, tile_rows=shape[0], tile_cols=shape[1], waves=1, chunk_rows=chunk)
        for gen, H, W, K, R, lam in cases:
            say(f"chunk {chunk} tile {shape} {gen} {H}x{W} K={K} R={R} lam={lam}")
            pc1, prob = inputs.GENERATORS[gen](H, W, 5)
            df = DeviceFrame(pc1, prob, K, R, lam)
            df.clear_outputs()
            _lib.knnf_filter(ctx, df.as_c(), plan, current_stream())
            go, gc, gn, gd = df.results()
            ro, rc, rn, rd = oracle.knn_filter(pc1, prob, K, R, lam)
            assert np.array_equal(gn, rn) and np.array_equal(gc, rc)
            assert np.array_equal(gd.view(np.uint32), rd.view(np.uint32))
            assert float(np.max(np.abs(go.astype(np.float64) - ro))) <= 1e-6


def test_window_chunks_full_frame_equal(ctx):
    """The headline frame: every chunk (and both searches) gives the same bits."""
    import torch

    spec = inputs.config1().frames[0]
    pc1, prob = spec.make()
    outs = []
    for plan in (dict(search=0), dict(search=1, chunk_rows=8), dict(search=1, chunk_rows=16),
                 dict(search=1, chunk_rows=32)):
        say(f"config1 plan {plan}")
        df = DeviceFrame(pc1, prob, spec.K, spec.R, spec.lam)
        _lib.knnf_filter(ctx, df.as_c(), dict(plan, flags=NOCHECK), current_stream())
        torch.cuda.synchronize()
        outs.append(df.results())
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert np.array_equal(x, y)


def test_tune_cache_round_trip(tmp_path, monkeypatch):
    import torch

    path = str(tmp_path / "tune.json")
    monkeypatch.setenv("KNNF_TUNE_CACHE", path)
    c = _lib.knnf_create(0)
    try:
        specs = [inputs.FrameSpec("brain", 70, 130, 1, K=40, R=14),
                 inputs.FrameSpec("derma", 50, 50, 2, K=16, R=7),
                 inputs.FrameSpec("derma", 50, 50, 3, K=16, R=7)]
        data = [s.make() for s in specs]
        frames = [DeviceFrame(p, q, s.K, s.R, s.lam) for s, (p, q) in zip(specs, data)]
        one = frames[:1]
        st, _ = _lib.knnf_tune_lookup(c, [f.as_c() for f in one])
        assert st == _lib.KNNF_ESTATE
        say("tune one frame and a batch")
        best1 = _lib.knnf_tune(c, [f.as_c() for f in one], 1, current_stream()).as_dict()
        bestb = _lib.knnf_tune(c, [f.as_c() for f in frames], 1, current_stream()).as_dict()
        st, p1 = _lib.knnf_tune_lookup(c, [f.as_c() for f in one])
        assert st == _lib.KNNF_OK and p1.as_dict() == best1
        st, pb = _lib.knnf_tune_lookup(c, [f.as_c() for f in frames])
        assert st == _lib.KNNF_OK and pb.as_dict() == bestb
        doc = json.load(open(path))
        keys = {e["key"] for e in doc["entries"]}
        assert "frame H=70 W=130 K=40 R=14 C=4" in keys and len(keys) == 2
        # calls without a plan use the cached plans; outputs equal the default plan's
        for f in frames:
            f.clear_outputs()
        _lib.knnf_filter(c, one[0].as_c(), None, current_stream())
        torch.cuda.synchronize()
        tuned_one = one[0].results()
        _lib.knnf_filter_batch(c, [f.as_c() for f in frames], None, current_stream())
        torch.cuda.synchronize()
        tuned = [f.results() for f in frames]
        for x, y in zip(tuned_one, tuned[0]):
            assert np.array_equal(x, y)
        for f, (s, (p, q)), t in zip(frames, zip(specs, data), tuned):
            f.clear_outputs()
            _lib.knnf_filter(c, f.as_c(), dict(search=1), current_stream())
            torch.cuda.synchronize()
            for x, y in zip(t, f.results()):
                assert np.array_equal(x, y)
    finally:
        _lib.knnf_destroy(c)
    # a new context loads the file
    c2 = _lib.knnf_create(0)
    try:
        st, p = _lib.knnf_tune_lookup(c2, [f.as_c() for f in frames])
        assert st == _lib.KNNF_OK and p.as_dict() == bestb
    finally:
        _lib.knnf_destroy(c2)
