"""GPU parity of knnf_svm_pc1: the SVM probability maps and the PC1 band
from one read of the cube.

Bars: the maps are bitwise equal to knnf_svm's (the same decision-value and
coupling arithmetic) and so within 1e-6 of the SVM oracle; the band is
within one binary32 ulp of the PC1 oracle (its binary64 sum runs band by band,
so it may differ from knnf_pc1's in the last bit), with min 0 and max 1
exactly when normalised.  Cases: the 16-byte and scalar staging paths, partial
band chunks, partial blocks, 2 to 8 classes, raw and normalised bands, the
full W 480 x H 380 x 128 and 1000 x 1000 x 100 cubes, and the fused output
fed straight into the filter.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import pc1_oracle, svm_oracle
from paper_2404_10631_amd import _lib, inputs
from paper_2404_10631_amd.frames import DeviceFrame, current_stream

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


def dev(a, dtype=None):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a if dtype is None else a.astype(dtype))).cuda()


def run(ctx, cube, mean, vec, model, C, normalize, offset_floats=0):
    """(fused maps, fused band, knnf_svm maps, knnf_pc1 band) as numpy arrays."""
    import torch

    npix, nb = cube.shape
    flat = torch.zeros(offset_floats + npix * nb, dtype=torch.float32, device="cuda")
    flat[offset_floats:] = dev(cube.reshape(-1))
    cp = flat.data_ptr() + 4 * offset_floats
    w, bias, A, B = (dev(a, np.float64) for a in model)
    dm, dv = dev(mean, np.float64), dev(vec, np.float64)
    maps = torch.full((npix, C), float("nan"), dtype=torch.float32, device="cuda")
    band = torch.full((npix,), float("nan"), dtype=torch.float32, device="cuda")
    _lib.knnf_svm_pc1(ctx, cp, npix, nb, C, w.data_ptr(), bias.data_ptr(), A.data_ptr(),
                      B.data_ptr(), dm.data_ptr(), dv.data_ptr(), maps.data_ptr(), band.data_ptr(),
                      normalize, current_stream())
    maps2 = torch.full_like(maps, float("nan"))
    band2 = torch.full_like(band, float("nan"))
    _lib.knnf_svm(ctx, cp, npix, nb, C, w.data_ptr(), bias.data_ptr(), A.data_ptr(), B.data_ptr(),
                  maps2.data_ptr(), current_stream())
    _lib.knnf_pc1(ctx, cp, npix, nb, dm.data_ptr(), dv.data_ptr(), band2.data_ptr(), normalize,
                  current_stream())
    torch.cuda.synchronize()
    return maps.cpu().numpy(), band.cpu().numpy(), maps2.cpu().numpy(), band2.cpu().numpy()


def check(ctx, cube, mean, vec, model, C, normalize, label, offset_floats=0):
    fm, fb, sm, pb = run(ctx, cube, mean, vec, model, C, normalize, offset_floats)
    assert np.array_equal(fm.view(np.uint32), sm.view(np.uint32)), f"{label}: maps differ from knnf_svm"
    ref = svm_oracle.svm_prob(cube, *model, C)
    assert float(np.max(np.abs(fm.astype(np.float64) - ref))) <= 1e-6, f"{label}: maps vs oracle"
    rb = pc1_oracle.pc1(cube, mean, vec, normalize)
    ulp = np.spacing(np.abs(rb)).astype(np.float64)
    bad = np.abs(fb.astype(np.float64) - rb) > ulp
    assert not bad.any(), f"{label}: band beyond one ulp at {np.nonzero(bad)[0][:5].tolist()}"
    assert np.all(np.abs(fb.astype(np.float64) - pb.astype(np.float64)) <= 2 * ulp)
    if normalize and fb.size > 1 and rb.max() > rb.min():
        assert fb.min() == 0.0 and fb.max() == 1.0


CASES = [
    # label, H, W, bands, classes, kind
    ("brain-128-C4", 50, 70, 128, 4, "brain"),
    ("derma-100-C4", 40, 60, 100, 4, "derma"),
    ("bands-300-C4", 30, 31, 300, 4, "brain"),
    ("bands-33-scalar", 20, 45, 33, 4, "brain"),
    ("bands-7-scalar", 27, 37, 7, 3, "derma"),
    ("C2", 33, 33, 128, 2, "derma"),
    ("C5", 20, 20, 128, 5, "brain"),
    ("C8", 19, 23, 96, 8, "brain"),
    ("one-pixel", 1, 1, 128, 4, "brain"),
    ("ragged-block", 1, 257, 128, 4, "brain"),
    ("bands-100-C8", 11, 29, 100, 8, "derma"),
    ("ragged-129-100", 1, 129, 100, 4, "derma"),
    ("runs-700-100", 1, 700, 100, 4, "derma"),
    ("C3-36", 17, 43, 36, 3, "brain"),
    ("bands-4", 13, 11, 4, 4, "derma"),
]


@pytest.mark.parametrize("normalize", [True, False], ids=["normalised", "raw"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_fused_matches_both_steps(ctx, case, normalize):
    label, H, W, nb, C, kind = case
    cube, mean, vec = inputs.g_cube(H, W, nb, 11, kind)
    model = inputs.g_svm_model(C, nb, 12)
    say(f"fused {label} normalize={normalize}")
    check(ctx, cube, mean, vec, model, C, normalize, label)


def test_fused_unaligned_cube(ctx):
    cube, mean, vec = inputs.g_cube(24, 30, 128, 13)
    model = inputs.g_svm_model(4, 128, 14)
    say("fused unaligned cube (scalar staging)")
    check(ctx, cube, mean, vec, model, 4, True, "unaligned", offset_floats=1)


@pytest.mark.parametrize("shape", [(380, 480, 128, "brain"), (1000, 1000, 100, "derma")],
                         ids=["brain480x380x128", "derma1000x1000x100"])
def test_fused_full_size_cubes(ctx, shape):
    H, W, nb, kind = shape
    cube, mean, vec = inputs.g_cube(H, W, nb, 1, kind)
    model = inputs.g_svm_model(4, nb, 2)
    say(f"fused full size {shape}")
    check(ctx, cube, mean, vec, model, 4, True, f"{kind} full")


def test_fused_output_feeds_the_filter(ctx):
    """Cube -> knnf_svm_pc1 -> knnf_filter on the device; the filter is bit-exact
    against the oracle run on the fused maps and band."""
    import torch

    H, W, nb = 60, 80, 128
    cube, mean, vec = inputs.g_cube(H, W, nb, 21)
    model = inputs.g_svm_model(4, nb, 22)
    dc = dev(cube.reshape(-1))
    w, bias, A, B = (dev(a, np.float64) for a in model)
    dm, dv = dev(mean, np.float64), dev(vec, np.float64)
    df = DeviceFrame(np.zeros((H, W), np.float32), np.zeros((H, W, 4), np.float32), 16, 5, 0.01)
    _lib.knnf_svm_pc1(ctx, dc.data_ptr(), H * W, nb, 4, w.data_ptr(), bias.data_ptr(), A.data_ptr(),
                      B.data_ptr(), dm.data_ptr(), dv.data_ptr(), df.prob.data_ptr(),
                      df.pc1.data_ptr(), True, current_stream())
    _lib.knnf_filter(ctx, df.as_c(), None, current_stream())
    torch.cuda.synchronize()
    band = df.pc1.cpu().numpy()
    maps = df.prob.cpu().numpy()
    go, gc, gn, gd = df.results()
    ro, rc, rn, rd = oracle.knn_filter(band, maps, 16, 5, 0.01)
    assert np.array_equal(gn, rn) and np.array_equal(gc, rc)
    assert np.array_equal(gd.view(np.uint32), rd.view(np.uint32))
    assert float(np.max(np.abs(go.astype(np.float64) - ro))) <= 1e-6
