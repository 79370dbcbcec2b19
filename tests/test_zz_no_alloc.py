"""knnf_pc1_noalloc: the PC1 projection on the library's static scratch, for
callers that cannot allocate.  Its outputs must equal knnf_pc1's (the same
kernels) on two calls in a row, the second on a smaller cube, and stay within
one binary32 ulp of the oracle; sizes beyond the scratch are rejected; device
memory in use does not change across calls."""
import sys

import numpy as np
import pytest

from paper_2404_10631_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(*arrays):
    import torch

    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def project(ctx, fn, cube, mean, vec, normalize):
    import torch

    from paper_2404_10631_amd.frames import current_stream

    dc, dm, dv = to_dev(cube, mean, vec)
    out = torch.full((cube.shape[0],), float("nan"), dtype=torch.float32, device="cuda")
    fn(ctx, dc.data_ptr(), cube.shape[0], cube.shape[1], dm.data_ptr(), dv.data_ptr(),
       out.data_ptr(), normalize, current_stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_pc1_on_consecutive_calls():
    from oracle import pc1_oracle

    ctx = _lib.knnf_create(0)
    try:
        big = inputs.g_cube(380, 480, 128, 1)            # 182,400 pixels, 128 bands
        small = inputs.g_cube(37, 53, 100, 2, "derma")   # 1,961 pixels, 100 bands
        for normalize in (True, False):
            say(f"noalloc: big cube then small cube, normalize={normalize}")
            got = [project(ctx, _lib.knnf_pc1_noalloc, *c, normalize) for c in (big, small)]
            want = [project(ctx, _lib.knnf_pc1, *c, normalize) for c in (big, small)]
            for g, w, c in zip(got, want, (big, small)):
                assert np.array_equal(g.view(np.uint32), w.view(np.uint32))
                ref = pc1_oracle.pc1(*c, normalize)
                assert np.all(np.abs(g.astype(np.float64) - ref) <= np.spacing(np.abs(ref)))
    finally:
        _lib.knnf_destroy(ctx)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import torch

    from paper_2404_10631_amd.frames import current_stream

    ctx = _lib.knnf_create(0)
    try:
        buf = torch.zeros(64, dtype=torch.float64, device="cuda")
        p = buf.data_ptr()
        with pytest.raises(_lib.KnnfError) as ei:
            _lib.knnf_pc1_noalloc(ctx, p, _lib.KNNF_PC1_NOALLOC_MAX_PIXELS + 1, 4, p, p, p, True,
                                  current_stream())
        assert ei.value.status == _lib.KNNF_EINVAL and "scratch" in str(ei.value)
        assert _lib.knnf_ctx_status(ctx) == _lib.KNNF_OK
    finally:
        _lib.knnf_destroy(ctx)


def test_noalloc_allocates_nothing():
    import torch

    ctx = _lib.knnf_create(0)
    try:
        cubes = [inputs.g_cube(200, 300, 128, 3), inputs.g_cube(20, 30, 64, 4)]
        dev = [to_dev(*c) for c in cubes]
        outs = [torch.empty(c[0].shape[0], dtype=torch.float32, device="cuda") for c in cubes]
        from paper_2404_10631_amd.frames import current_stream

        def run(k):
            (dc, dm, dv), c = dev[k], cubes[k][0]
            _lib.knnf_pc1_noalloc(ctx, dc.data_ptr(), c.shape[0], c.shape[1], dm.data_ptr(),
                                  dv.data_ptr(), outs[k].data_ptr(), True, current_stream())

        run(0)
        run(1)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        for k in (0, 1, 0, 1):
            run(k)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0
    finally:
        _lib.knnf_destroy(ctx)
