"""GPU parity at the benchmark's full sizes, in the launch configurations the
benchmark times: the 64 uneven brain-like frames and the 1024 dermatology-like
50 x 50 frames in one batched launch, and the mixed S/M/L serving stream
through the batching server.  The 1024 small frames are checked at every
pixel against the oracle run here.  The uneven and served frames are checked
at sampled positions against the oracle run here (neighbour indices,
distances and classes bit-exact, probabilities within 1e-6) and at every
pixel against digests of the oracle's whole-frame outputs that
tests/golden/oracle_digests.py wrote (the oracle needs about half an hour of
CPU for them): indices, distance bits, classes and probability bits equal.
"""
import importlib.util
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2404_10631_amd import _lib, inputs
from paper_2404_10631_amd.frames import DeviceFrame, current_stream
from paper_2404_10631_amd.serve import HostFrame, Server, replay

pytestmark = pytest.mark.gpu

PROB_TOL = 1e-6
PERSISTENT = dict(search=1, tile_rows=2, tile_cols=4, waves=1, launch=1)
GRID = dict(search=1, tile_rows=2, tile_cols=4, waves=1, launch=2)  # the context's default


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = _lib.knnf_create(0)
    yield c
    _lib.knnf_destroy(c)


def sample_pixels(H, W, n, rng):
    """Corners, edge midpoints and n random pixels (linear indices)."""
    fixed = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, 0), (H // 2, W - 1),
             (0, W // 2), (H - 1, W // 2)]
    r = rng.integers(0, H, n)
    c = rng.integers(0, W, n)
    pix = np.array([i * W + j for i, j in fixed] + list(r * W + c), np.int64)
    return np.unique(pix)


_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _digest_module():
    spec = importlib.util.spec_from_file_location("oracle_digests",
                                                  os.path.join(_GOLDEN, "oracle_digests.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def oracle_digests(name):
    with open(os.path.join(_GOLDEN, "oracle_digests.json")) as f:
        return json.load(f)[name]


def check_digests(label, spec, data, outs, want):
    """Every pixel of the device's outputs against the oracle's digests."""
    dig = _digest_module()
    got = dig.frame_record(spec, outs, data)
    for key in ("gen", "H", "W", "seed", "K", "R"):
        assert got[key] == want[key], f"{label}: digest file is for another frame ({key})"
    assert got["inputs"] == want["inputs"], f"{label}: the input generator changed"
    for key in ("nbr", "dist", "class", "prob"):
        assert got[key] == want[key], f"{label}: {key} differs from the oracle's whole frame"


def check_sampled(label, spec, data, outs, pix):
    go, gc, gn, gd = outs
    pc1, prob = data
    ro, rc, rn, rd = oracle.knn_pixels(pc1, prob, spec.K, spec.R, spec.lam, pix)
    H, W = spec.H, spec.W
    fo = go.reshape(H * W, -1)[pix]
    fc = gc.reshape(-1)[pix]
    if gn is not None:
        assert np.array_equal(gn.reshape(H * W, -1)[pix], rn), f"{label}: neighbours differ"
        assert np.array_equal(gd.reshape(H * W, -1)[pix].view(np.uint32), rd.view(np.uint32)), \
            f"{label}: distances differ"
    assert np.array_equal(fc, rc), f"{label}: class differs"
    assert float(np.max(np.abs(fo.astype(np.float64) - ro))) <= PROB_TOL, f"{label}: prob differs"


@pytest.mark.parametrize("plan", [PERSISTENT, GRID], ids=["persistent", "grid"])
def test_config2_uneven_batch_full_size(ctx, plan):
    """64 brain-like frames, H and W uniform in [50, 1000], K = 40, +-14 rows,
    one batched launch; 128 sampled pixels per frame against the oracle."""
    import torch

    wl = inputs.config2()
    say(f"config2: generating {len(wl.frames)} frames, {wl.pixels} pixels")
    data = [s.make() for s in wl.frames]
    frames = [DeviceFrame(p, q, s.K, s.R, s.lam, with_nbr=True) for s, (p, q) in zip(wl.frames, data)]
    say(f"config2: one batched launch, plan={plan}")
    _lib.knnf_filter_batch(ctx, [f.as_c() for f in frames], plan, current_stream())
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    want = oracle_digests("config2")
    assert len(want) == len(wl.frames)
    for k, (s, d, f) in enumerate(zip(wl.frames, data, frames)):
        outs = f.results()
        check_sampled(f"config2 frame {k} ({s.H}x{s.W})", s, d, outs,
                      sample_pixels(s.H, s.W, 120, rng))
        check_digests(f"config2 frame {k} ({s.H}x{s.W})", s, d, outs, want[k])
    say("config2: sampled pixels bit-exact, every pixel equal to the oracle's digests")


def test_config3_small_frame_batch_full_size(ctx):
    """1024 derma-like 50 x 50 frames, K = 16, +-7 rows, one batched launch
    (the default grid launch; the persistent launch must give the same bits):
    every frame at every pixel against the oracle."""
    import torch

    wl = inputs.config3()
    say(f"config3: generating {len(wl.frames)} frames")
    data = [s.make() for s in wl.frames]
    frames = [DeviceFrame(p, q, s.K, s.R, s.lam, with_nbr=True) for s, (p, q) in zip(wl.frames, data)]
    say("config3: one batched launch, persistent")
    _lib.knnf_filter_batch(ctx, [f.as_c() for f in frames], PERSISTENT, current_stream())
    torch.cuda.synchronize()
    persistent = [f.results() for f in frames]
    for f in frames:
        f.clear_outputs()
    say("config3: one batched launch, default plan")
    _lib.knnf_filter_batch(ctx, [f.as_c() for f in frames], None, current_stream())
    torch.cuda.synchronize()
    for k, (s, d, f) in enumerate(zip(wl.frames, data, frames)):
        go, gc, gn, gd = f.results()
        for x, y in zip((go, gc, gn, gd), persistent[k]):
            assert np.array_equal(x, y), f"config3 frame {k}: launch modes differ"
        ro, rc, rn, rd = oracle.knn_filter(d[0], d[1], s.K, s.R, s.lam)
        assert np.array_equal(gn, rn) and np.array_equal(gc, rc), f"config3 frame {k}"
        assert np.array_equal(gd.view(np.uint32), rd.view(np.uint32)), f"config3 frame {k}"
        assert float(np.max(np.abs(go.astype(np.float64) - ro))) <= PROB_TOL
    say("config3: all 1024 frames bit-exact at every pixel")


def test_config4_served_mix_full_size(ctx):
    """The serving stream's S/M/L classes at full size (50x50 K=16 +-7,
    W480xH380 K=40 +-14, 1000x1000 K=40 +-14), Poisson arrivals, through the
    batching server, neighbour outputs kept; every frame checked at sampled
    pixels (indices, distances, classes, probabilities)."""
    stream = inputs.serve_stream(n=40, rate_hz=2000.0, seed=11)
    specs = [s for _, _, s in stream]
    arrivals = [t for t, _, _ in stream]
    say(f"config4: generating {len(specs)} frames "
        f"({sum(1 for _, c, _ in stream if c == 'L')} of 1000x1000)")
    data = [s.make() for s in specs]
    hosts = [HostFrame(p, q, s.K, s.R, s.lam) for s, (p, q) in zip(specs, data)]
    pool = 2 << 30
    results = {}
    say("config4: replaying through the server")
    with Server(ctx, pool) as srv:
        replay(srv, hosts, arrivals, keep=lambda k, v: results.__setitem__(k, srv.view_arrays(v)),
               with_nbr=True)
    rng = np.random.default_rng(9)
    want = oracle_digests("config4")
    assert len(want) == len(specs)
    for k, (s, d) in enumerate(zip(specs, data)):
        go, gc, gn, gd = results[k]
        assert gn is not None and gd is not None
        check_sampled(f"config4 frame {k} ({s.H}x{s.W})", s, d, (go, gc, gn, gd),
                      sample_pixels(s.H, s.W, 64, rng))
        check_digests(f"config4 frame {k} ({s.H}x{s.W})", s, d, (go, gc, gn, gd), want[k])
    say("config4: sampled pixels bit-exact, every pixel equal to the oracle's digests")
