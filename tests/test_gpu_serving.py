"""GPU tests of the serving path: a frame's outputs are the same alone and in
the served mix, admission respects the pool, and the error paths behave."""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_10631_amd import _lib, inputs
from paper_2404_10631_amd.frames import DeviceFrame, current_stream
from paper_2404_10631_amd.serve import HostFrame, Server, replay

pytestmark = pytest.mark.gpu


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


def _alone(ctx, spec, data):
    import torch

    df = DeviceFrame(data[0], data[1], spec.K, spec.R, spec.lam)
    _lib.knnf_filter(ctx, df.as_c(), None, current_stream())
    torch.cuda.synchronize()
    return df.results()


@pytest.mark.parametrize("mode", [_lib.KNNF_SERVE_BATCHED, _lib.KNNF_SERVE_PLAIN], ids=["batched", "plain"])
def test_served_mix_equals_alone(ctx, mode):
    specs = [inputs.FrameSpec("derma", 50, 50, 1, K=16, R=7),
             inputs.FrameSpec("brain", 120, 160, 2, K=40, R=14),
             inputs.FrameSpec("derma", 50, 50, 3, K=16, R=7),
             inputs.FrameSpec("derma", 300, 260, 4, K=40, R=14),
             inputs.FrameSpec("unif", 64, 64, 5, K=8, R=4),
             inputs.FrameSpec("derma", 50, 50, 6, K=16, R=7)]
    data = [s.make() for s in specs]
    frames = [HostFrame(p, q, s.K, s.R, s.lam) for s, (p, q) in zip(specs, data)]
    say(f"serve mode {mode}")
    with Server(ctx, 64 << 20, mode=mode, step_tiles=2048) as srv:
        # all arrive almost together: several frames share each step
        arrivals = [0.0, 0.0002, 0.0004, 0.0006, 0.0008, 0.001]
        results = {}

        def keep_copy(k, view):
            results[k] = srv.view_arrays(view)

        res = replay(srv, frames, arrivals, keep=keep_copy)
    assert np.all(res["latency_s"] > 0)
    for k, (s, d) in enumerate(zip(specs, data)):
        alone = _alone(ctx, s, d)
        assert np.array_equal(results[k][0], alone[0]), f"prob differs for frame {k}"
        assert np.array_equal(results[k][1], alone[1]), f"class differs for frame {k}"
        ro, rc, _, _ = oracle.knn_filter(d[0], d[1], s.K, s.R, s.lam, with_nbr=False)
        assert np.array_equal(results[k][1], rc)
        assert np.max(np.abs(results[k][0] - ro)) <= 1e-6


def test_split_frames_wait_for_their_inputs(ctx):
    """Frames split over many small steps run on both compute streams; every
    step waits for the copy of its frame's inputs, so the results equal the
    frames filtered alone (regression: only the first step of a frame used
    to wait, so later steps on the other stream could read inputs still
    being copied)."""
    specs = [inputs.FrameSpec("derma", 400, 420, 11 + k, K=40, R=14) for k in range(3)]
    data = [s.make() for s in specs]
    frames = [HostFrame(p, q, s.K, s.R, s.lam) for s, (p, q) in zip(specs, data)]
    say("split frames over small steps")
    with Server(ctx, 256 << 20, max_inflight=2, step_tiles=512) as srv:
        results = {}
        replay(srv, frames, [0.0] * len(frames),
               keep=lambda k, v: results.__setitem__(k, srv.view_arrays(v)))
    for k, (s, d) in enumerate(zip(specs, data)):
        alone = _alone(ctx, s, d)
        assert np.array_equal(results[k][1], alone[1]), f"class differs for frame {k}"
        assert np.array_equal(results[k][0], alone[0]), f"prob differs for frame {k}"


def test_tiny_pool_admits_as_memory_frees(ctx):
    """A pool that holds one large frame at a time still serves a burst."""
    spec = inputs.FrameSpec("brain", 200, 200, 9, K=40, R=14)
    p, q = spec.make()
    one = _lib.knnf_frame_bytes(200, 200, 4, 40, 0)
    frames = [HostFrame(p, q, spec.K, spec.R, spec.lam) for _ in range(5)]
    say("tiny pool burst")
    with Server(ctx, one + 4096, step_tiles=1024) as srv:
        results = {}
        res = replay(srv, frames, [0.0] * 5, keep=lambda k, v: results.__setitem__(k, srv.view_arrays(v)))
    ref = _alone(ctx, spec, (p, q))
    for k in range(5):
        assert np.array_equal(results[k][1], ref[1])
        assert np.array_equal(results[k][0], ref[0])
    # served one after another: completion times are strictly ordered
    assert np.all(np.diff(np.sort(res["t_done"])) > 0)


def test_server_errors(ctx):
    small = inputs.FrameSpec("derma", 50, 50, 1, K=16, R=7)
    p, q = small.make()
    hf = HostFrame(p, q, small.K, small.R, small.lam)
    with Server(ctx, 1 << 20, max_queue=2) as srv:
        # larger than the whole pool
        big = inputs.FrameSpec("unif", 600, 600, 2, K=8, R=2)
        bp, bq = big.make()
        hb = HostFrame(bp, bq, big.K, big.R, big.lam)
        with pytest.raises(_lib.KnnfError) as ei:
            _lib.knnf_server_submit(srv.handle, hb.as_c())
        assert ei.value.status == _lib.KNNF_ENOMEM
        # invalid parameters
        bad = hf.as_c()
        bad.K = 1000
        with pytest.raises(_lib.KnnfError) as ei:
            _lib.knnf_server_submit(srv.handle, bad)
        assert ei.value.status == _lib.KNNF_EINVAL
        # unknown ticket
        with pytest.raises(_lib.KnnfError):
            _lib.knnf_server_poll(srv.handle, 987654321)
        st, tk = _lib.knnf_server_submit(srv.handle, hf.as_c())
        assert st == _lib.KNNF_OK
        _lib.knnf_server_drain(srv.handle, 30.0)
        info = _lib.knnf_server_poll(srv.handle, tk)
        assert info.done == 1 and info.t_done >= info.t_launch >= info.t_admit >= info.t_arrival
        _lib.knnf_server_release(srv.handle, tk)
        with pytest.raises(_lib.KnnfError):
            _lib.knnf_server_release(srv.handle, tk)


def test_server_pool_must_be_aligned(ctx):
    """The pool is sub-allocated at 256-byte offsets and the server's stream
    warm-up writes its first word: a misaligned or tiny pool is rejected."""
    import torch

    pool = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    for ptr, size in ((pool.data_ptr() + 16, (1 << 20) - 16), (pool.data_ptr(), 1024)):
        with pytest.raises(_lib.KnnfError) as ei:
            _lib.knnf_server_create(ctx, ptr, size)
        assert ei.value.status == _lib.KNNF_EINVAL
    h = _lib.knnf_server_create(ctx, pool.data_ptr(), 1 << 20)
    _lib.knnf_server_destroy(h)


class _PageableFrame:
    """A host frame in ordinary (pageable) numpy memory: the server copies it
    with the copy engine, never with the copy kernel."""

    def __init__(self, pc1, prob, K, R, lam):
        self.pc1 = np.ascontiguousarray(pc1, np.float32)
        self.prob = np.ascontiguousarray(prob, np.float32)
        self.H, self.W = self.pc1.shape
        self.C = self.prob.shape[2]
        self.K, self.R, self.lam = K, R, lam

    def as_c(self, t_arrival=-1.0, with_nbr=False):
        f = _lib.knnf_host_frame()
        f.H, f.W, f.C, f.K, f.R, f.lam = self.H, self.W, self.C, self.K, self.R, self.lam
        f.pc1 = self.pc1.ctypes.data
        f.prob = self.prob.ctypes.data
        f.with_nbr = 0
        f.t_arrival = t_arrival
        return f


@pytest.mark.parametrize("mode", [_lib.KNNF_SERVE_BATCHED, _lib.KNNF_SERVE_PLAIN], ids=["batched", "plain"])
def test_burst_through_the_copier(ctx, mode):
    """80 frames submitted together back up the copy stream, so most of them
    are copied by the copier thread, in batched mode those in pinned memory
    by the copy kernel; pageable frames (and the plain mode) take the copy
    engine.  Every frame equals the frame filtered alone."""
    specs = ([inputs.FrameSpec("derma", 50, 50, 200 + k, K=16, R=7) for k in range(60)]
             + [inputs.FrameSpec("brain", 120, 160, 300 + k, K=40, R=14) for k in range(12)]
             + [inputs.FrameSpec("derma", 300, 260, 400 + k, K=40, R=14) for k in range(4)]
             + [inputs.FrameSpec("unif", 40, 70, 500 + k, K=8, R=4) for k in range(4)])
    order = np.random.default_rng(3).permutation(len(specs))
    specs = [specs[i] for i in order]
    data = [s.make() for s in specs]
    frames = [(_PageableFrame if s.gen == "unif" else HostFrame)(p, q, s.K, s.R, s.lam)
              for s, (p, q) in zip(specs, data)]
    say(f"burst of {len(frames)} frames, mode {mode}")
    with Server(ctx, 256 << 20, mode=mode) as srv:
        results = {}
        replay(srv, frames, [0.0] * len(frames),
               keep=lambda k, v: results.__setitem__(k, srv.view_arrays(v)))
    for k, (s, d) in enumerate(zip(specs, data)):
        alone = _alone(ctx, s, d)
        assert np.array_equal(results[k][1], alone[1]), f"class differs for frame {k} ({s})"
        assert np.array_equal(results[k][0], alone[0]), f"prob differs for frame {k} ({s})"
