"""GPU parity of the SVM probability stage (knnf_svm) against the binary64
oracle.

Bar: both sides evaluate every step in binary64 and round once to binary32;
the GPU sums the decision values and the coupling products in its own order,
so values agree to a few binary64 ulps before the final rounding: every
output within 1e-6 of the oracle's (in practice equal or one binary32 ulp
apart).  Cases cover the three staging paths (16-byte band chunks, scalar
band chunks, and linear runs of whole pixel rows for rows that are not whole
128-byte lines, up to four classes), band counts that leave a partial
32-band chunk, pixel counts that leave a partial block or a partial run, two
to eight classes, and the full W 480 x H 380 x 128 and 1000 x 1000 x 100
cubes at every pixel.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import pc1_oracle, svm_oracle
from paper_2404_10631_amd import _lib, inputs
from paper_2404_10631_amd.frames import DeviceFrame, current_stream

pytestmark = pytest.mark.gpu

TOL = 1e-6


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


def run_svm(ctx, cube, model, C, offset_floats=0, out=None):
    import torch

    npix, nb = cube.shape
    w, bias, A, B = (torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda() for a in model)
    flat = torch.zeros(offset_floats + npix * nb, dtype=torch.float32, device="cuda")
    flat[offset_floats:] = torch.from_numpy(np.ascontiguousarray(cube).reshape(-1)).cuda()
    res = torch.full((npix, C), float("nan"), dtype=torch.float32, device="cuda") if out is None else out
    _lib.knnf_svm(ctx, flat.data_ptr() + 4 * offset_floats, npix, nb, C, w.data_ptr(),
                  bias.data_ptr(), A.data_ptr(), B.data_ptr(), res.data_ptr(), current_stream())
    torch.cuda.synchronize()
    return res.cpu().numpy().reshape(npix, C)


def check(got, ref, label):
    assert got.shape == ref.shape and np.all(np.isfinite(got)), label
    err = np.abs(got.astype(np.float64) - ref.astype(np.float64))
    bad = np.nonzero(err.max(axis=1) > TOL)[0]
    assert bad.size == 0, f"{label}: {bad.size} pixels beyond {TOL}, first {bad[:5].tolist()}"


CASES = [
    # label, H, W, bands, classes, kind
    ("brain-128-C4", 50, 70, 128, 4, "brain"),
    ("derma-100-C4", 40, 60, 100, 4, "derma"),
    ("bands-300-C4", 30, 31, 300, 4, "brain"),
    ("bands-33-scalar", 20, 45, 33, 4, "brain"),
    ("bands-7-scalar", 27, 37, 7, 3, "derma"),
    ("C2", 33, 33, 128, 2, "derma"),
    ("C3", 21, 50, 64, 3, "brain"),
    ("C5", 20, 20, 128, 5, "brain"),
    ("C6", 17, 31, 100, 6, "derma"),
    ("C7", 23, 29, 40, 7, "brain"),
    ("C8", 19, 23, 96, 8, "brain"),
    ("one-pixel", 1, 1, 128, 4, "brain"),
    ("ragged-block", 1, 257, 128, 4, "brain"),
    ("bands-4", 13, 11, 4, 4, "derma"),
    ("bands-12-C2", 7, 300, 12, 2, "brain"),
    ("bands-100-C8", 11, 29, 100, 8, "derma"),
    ("bands-124-C5", 9, 31, 124, 5, "brain"),
    ("bands-124-C2", 5, 40, 124, 2, "brain"),
    ("one-pixel-100", 1, 1, 100, 4, "derma"),
    ("ragged-129-100", 1, 129, 100, 4, "derma"),
    ("runs-700-100", 1, 700, 100, 4, "derma"),
    ("C3-36", 17, 43, 36, 3, "brain"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_svm_matches_oracle(ctx, case):
    label, H, W, nb, C, kind = case
    cube, _, _ = inputs.g_cube(H, W, nb, 31, kind)
    model = inputs.g_svm_model(C, nb, 32)
    say(f"svm {label} npix={H * W} bands={nb} classes={C}")
    got = run_svm(ctx, cube, model, C)
    check(got, svm_oracle.svm_prob(cube, *model, C), label)


def test_svm_unaligned_cube_uses_the_scalar_path(ctx):
    cube, _, _ = inputs.g_cube(30, 40, 128, 5)
    model = inputs.g_svm_model(4, 128, 6)
    say("svm unaligned cube")
    got = run_svm(ctx, cube, model, 4, offset_floats=1)
    check(got, svm_oracle.svm_prob(cube, *model, 4), "unaligned")


def test_svm_saturated_decisions_hit_the_clamp(ctx):
    """Hyperplanes scaled so that most binary probabilities clamp."""
    cube, _, _ = inputs.g_cube(24, 40, 128, 7)
    w, bias, A, B = inputs.g_svm_model(4, 128, 8)
    model = (w * 200.0, bias * 200.0, A, B)
    say("svm saturated")
    got = run_svm(ctx, cube, model, 4)
    check(got, svm_oracle.svm_prob(cube, *model, 4), "saturated")


def test_svm_full_size_brain_cube(ctx):
    """W 480 x H 380, 128 bands, four classes: every pixel."""
    cube, _, _ = inputs.g_cube(380, 480, 128, 1)
    model = inputs.g_svm_model(4, 128, 2)
    say("svm full-size brain cube")
    got = run_svm(ctx, cube, model, 4)
    check(got, svm_oracle.svm_prob(cube, *model, 4), "full-size")


def test_svm_full_size_derma_cube(ctx):
    """1000 x 1000, 100 bands (400-byte pixel rows, staged as linear runs of
    whole rows), four classes: every pixel."""
    cube, _, _ = inputs.g_cube(1000, 1000, 100, 3, "derma")
    model = inputs.g_svm_model(4, 100, 4)
    say("svm full-size derma cube")
    got = run_svm(ctx, cube, model, 4)
    check(got, svm_oracle.svm_prob(cube, *model, 4), "derma full-size")


def test_cube_to_class_map_on_the_device(ctx):
    """Cube -> knnf_svm and knnf_pc1 -> knnf_filter, all on the device: each
    stage against its oracle (the filter run by the oracle on the band and
    maps the device produced, so the filter's bar stays bit-exact)."""
    import torch

    H, W, K, R, C = 60, 90, 16, 7, 4
    cube, mean, vec = inputs.g_cube(H, W, 128, 9)
    model = inputs.g_svm_model(C, 128, 10)
    df = DeviceFrame(np.zeros((H, W), np.float32), np.zeros((H, W, C), np.float32), K, R, 0.01,
                     with_nbr=True)
    dcube = torch.from_numpy(cube).cuda()
    dmean, dvec = torch.from_numpy(mean).cuda(), torch.from_numpy(vec).cuda()
    dmodel = [torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda() for a in model]
    say("svm + pc1 -> filter")
    _lib.knnf_svm(ctx, dcube.data_ptr(), H * W, 128, C, *(t.data_ptr() for t in dmodel),
                  df.prob.data_ptr(), current_stream())
    _lib.knnf_pc1(ctx, dcube.data_ptr(), H * W, 128, dmean.data_ptr(), dvec.data_ptr(),
                  df.pc1.data_ptr(), True, current_stream())
    _lib.knnf_filter(ctx, df.as_c(), None, current_stream())
    torch.cuda.synchronize()
    prob = df.prob.cpu().numpy()
    band = df.pc1.cpu().numpy()
    check(prob.reshape(H * W, C), svm_oracle.svm_prob(cube, *model, C), "maps")
    ref_band = pc1_oracle.pc1(cube, mean, vec, True)
    assert np.all(np.abs(band.reshape(-1).astype(np.float64) - ref_band)
                  <= np.spacing(np.abs(ref_band).astype(np.float32)))
    go, gc, gn, gd = df.results()
    ro, rc, rn, rd = oracle.knn_filter(band, prob, K, R, 0.01)
    assert np.array_equal(gn, rn) and np.array_equal(gc, rc)
    assert np.max(np.abs(go.astype(np.float64) - ro)) <= 1e-6
