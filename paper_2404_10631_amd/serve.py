"""Serving harness: replay timed frame arrivals against a knnf server.

The server (C++, inside libknnf.so) does admission, batching and completion;
this module only keeps host frames in pinned memory, submits them at their
arrival times, releases finished frames and computes latency statistics.
Latency = completion observed by the server - scheduled arrival (the copy of
the inputs to the device is included).
"""
from __future__ import annotations

import time

import numpy as np

from . import _lib


class HostFrame:
    """One frame's inputs in pinned host memory plus its filter parameters."""

    def __init__(self, pc1, prob, K: int, R: int, lam: float, cls: str = ""):
        import torch

        self.pc1 = torch.from_numpy(np.ascontiguousarray(pc1, np.float32)).pin_memory()
        self.prob = torch.from_numpy(np.ascontiguousarray(prob, np.float32)).pin_memory()
        # The first device copy from a pinned buffer costs milliseconds in the
        # HIP runtime; pay it here rather than when the server admits the frame.
        for t in (self.pc1, self.prob):
            t.to("cuda", non_blocking=False)
        self.H, self.W = self.pc1.shape
        self.C = self.prob.shape[2]
        self.K, self.R, self.lam, self.cls = int(K), int(R), float(lam), cls

    @property
    def pixels(self) -> int:
        return self.H * self.W

    def as_c(self, t_arrival: float = -1.0, with_nbr: bool = False) -> _lib.knnf_host_frame:
        f = _lib.knnf_host_frame()
        f.H, f.W, f.C, f.K, f.R, f.lam = self.H, self.W, self.C, self.K, self.R, self.lam
        f.pc1 = self.pc1.data_ptr()
        f.prob = self.prob.data_ptr()
        f.with_nbr = 1 if with_nbr else 0
        f.t_arrival = t_arrival
        return f


class Server:
    """A knnf server over a torch-allocated device pool."""

    def __init__(self, ctx: int, pool_bytes: int, mode: int = _lib.KNNF_SERVE_BATCHED,
                 max_inflight: int = 2, step_tiles: int = 0, max_queue: int = 0, plan=None):
        import torch

        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        opts = _lib.knnf_server_opts()
        opts.mode, opts.max_queue = mode, max_queue
        opts.max_inflight, opts.step_tiles = max_inflight, step_tiles
        if plan is not None:
            opts.plan = _lib.make_plan(plan)
        else:
            dp = _lib.knnf_get_default_plan(ctx)
            opts.plan = dp
        self.handle = _lib.knnf_server_create(ctx, self.pool.data_ptr(), int(pool_bytes), opts)

    def view_arrays(self, view: _lib.knnf_frame):
        """Host copies of a finished frame's outputs (slices of the pool tensor):
        (out_prob (H,W,C), out_class (H,W), nbr or None, dist or None)."""
        import torch

        base = self.pool.data_ptr()
        H, W, C, K = view.H, view.W, view.C, view.K

        def grab(ptr, shape, dtype):
            n = int(np.prod(shape)) * torch.tensor([], dtype=dtype).element_size()
            off = ptr - base
            assert 0 <= off and off + n <= self.pool.numel(), "view outside the pool"
            return self.pool[off:off + n].view(dtype).reshape(shape).cpu().numpy()

        out_prob = grab(view.out_prob, (H, W, C), torch.float32)
        out_class = grab(view.out_class, (H, W), torch.int32)
        nbr = grab(view.out_nbr, (H, W, K), torch.int32) if view.out_nbr else None
        dist = grab(view.out_dist, (H, W, K), torch.float32) if view.out_dist else None
        return out_prob, out_class, nbr, dist

    def close(self):
        if self.handle:
            _lib.knnf_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def replay(server: Server, frames, arrivals, warmup: int = 0, keep=None, timeout_s: float = 120.0,
           with_nbr: bool = False):
    """Submit frames[k] at server-clock time t0 + arrivals[k]; release each frame
    as soon as it is done (after `keep(k, view)` if given).  With `with_nbr`
    the server also keeps each frame's neighbour indices and distances.

    Returns a dict with per-frame latencies (seconds), the server's per-frame
    timestamps (arrival, admission, first launch, completion) and the makespan.
    """
    h = server.handle
    n = len(frames)
    order = np.argsort(np.asarray(arrivals, np.float64), kind="stable")
    t0 = _lib.knnf_server_clock() + 0.01
    tickets = {}
    info = {}
    pending = []
    k = 0
    deadline = time.perf_counter() + timeout_s
    while len(info) < n:
        now = _lib.knnf_server_clock()
        while k < n and t0 + arrivals[order[k]] <= now:
            idx = int(order[k])
            st, tk = _lib.knnf_server_submit(h, frames[idx].as_c(t0 + arrivals[idx], with_nbr))
            if st == _lib.KNNF_EAGAIN:
                break
            tickets[tk] = idx
            pending.append(tk)
            k += 1
        still = []
        for tk in pending:
            inf = _lib.knnf_server_poll(h, tk)
            if inf.done:
                idx = tickets[tk]
                if keep is not None:
                    keep(idx, _lib.knnf_server_result(h, tk))
                info[idx] = (inf.t_arrival, inf.t_admit, inf.t_launch, inf.t_done)
                _lib.knnf_server_release(h, tk)
            else:
                still.append(tk)
        pending = still
        if time.perf_counter() > deadline:
            raise TimeoutError(f"replay: {len(info)} of {n} frames done before the timeout")
        if k < n:
            wait = t0 + arrivals[order[k]] - _lib.knnf_server_clock()
            if wait > 0.002:
                time.sleep(min(wait - 0.001, 0.002))
    t = np.array([info[i] for i in range(n)])
    lat = t[:, 3] - t[:, 0]
    sel = np.arange(n) >= warmup
    return {"latency_s": lat, "measured": sel, "t_arrival": t[:, 0], "t_admit": t[:, 1],
            "t_launch": t[:, 2], "t_done": t[:, 3],
            "makespan_s": float(t[sel, 3].max() - t[sel, 0].min())}


def summarize(frames, res, classes=None):
    lat = res["latency_s"][res["measured"]]
    px = sum(frames[i].pixels for i in np.nonzero(res["measured"])[0])
    out = {"frames": int(res["measured"].sum()),
           "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "max_ms": float(lat.max() * 1e3),
           "pixels_per_s": float(px / res["makespan_s"])}
    if classes:
        per = {}
        for c in classes:
            m = np.array([frames[i].cls == c for i in range(len(frames))]) & res["measured"]
            if m.any():
                lc = res["latency_s"][m]
                per[c] = {"n": int(m.sum()), "p50_ms": float(np.percentile(lc, 50) * 1e3),
                          "p99_ms": float(np.percentile(lc, 99) * 1e3)}
        out["per_class"] = per
    return out
