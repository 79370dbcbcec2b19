"""GPU parity of the PC1 projection (knnf_pc1) against the binary64 oracle.

Bar: both sides evaluate in binary64 and round once to binary32; the GPU sums
the bands in a different order (per-lane partial sums, then a butterfly), so
a value may round to the neighbouring binary32 number: every output is within
one binary32 ulp of the oracle's, and the normalised band has its minimum 0 and
maximum 1 exactly.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import pc1_oracle
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


def run_pc1(ctx, cube, mean, vec, normalize, offset_floats=0):
    """cube [npix, B] float32; offset_floats shifts the device cube off 16-byte alignment."""
    import torch

    npix, nb = cube.shape
    flat = torch.zeros(offset_floats + npix * nb, dtype=torch.float32, device="cuda")
    flat[offset_floats:] = torch.from_numpy(np.ascontiguousarray(cube).reshape(-1)).cuda()
    dmean = torch.from_numpy(np.asarray(mean, np.float64)).cuda()
    dvec = torch.from_numpy(np.asarray(vec, np.float64)).cuda()
    out = torch.full((npix,), float("nan"), dtype=torch.float32, device="cuda")
    _lib.knnf_pc1(ctx, flat.data_ptr() + 4 * offset_floats, npix, nb, dmean.data_ptr(),
                  dvec.data_ptr(), out.data_ptr(), normalize, current_stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_within_one_ulp(got, ref, label):
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got)), label
    tol = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    err = np.abs(got.astype(np.float64) - ref.astype(np.float64))
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{label}: {bad.size} values beyond one ulp, first {bad[:5].tolist()}"


CASES = [
    # label, npix, bands, kind -- vectorised paths (bands % 4 == 0, <= 256) and the scalar one
    ("brain-128", 50 * 70, 128, "brain"),
    ("derma-100", 40 * 60, 100, "derma"),
    ("bands-256", 900, 256, "brain"),
    ("bands-64", 1100, 64, "brain"),
    ("bands-12", 1000, 12, "derma"),
    ("bands-7-scalar", 777, 7, "brain"),
    ("bands-300-scalar", 500, 300, "brain"),
    ("one-pixel", 1, 128, "brain"),
    ("ragged-pixels", 8191, 128, "derma"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
@pytest.mark.parametrize("normalize", [True, False], ids=["norm", "raw"])
def test_pc1_matches_oracle(ctx, case, normalize):
    label, npix, nb, kind = case
    H = int(np.ceil(np.sqrt(npix)))
    W = int(np.ceil(npix / H))
    cube, mean, vec = inputs.g_cube(H, W, nb, 17, kind)
    cube = cube[:npix]
    say(f"pc1 {label} npix={npix} bands={nb} normalize={normalize}")
    got = run_pc1(ctx, cube, mean, vec, normalize)
    ref = pc1_oracle.pc1(cube, mean, vec, normalize)
    assert_within_one_ulp(got, ref, label)
    if normalize and npix > 1:
        assert got.min() == 0.0 and got.max() == 1.0


def test_pc1_unaligned_cube_uses_the_scalar_path(ctx):
    cube, mean, vec = inputs.g_cube(30, 40, 128, 3)
    say("pc1 unaligned cube")
    got = run_pc1(ctx, cube, mean, vec, True, offset_floats=1)
    assert_within_one_ulp(got, pc1_oracle.pc1(cube, mean, vec, True), "unaligned")


def test_pc1_constant_image_is_zero(ctx):
    cube = np.full((2000, 128), 0.25, np.float32)
    say("pc1 constant image")
    got = run_pc1(ctx, cube, np.zeros(128), np.full(128, 1.0 / np.sqrt(128)), True)
    assert np.array_equal(got, np.zeros(2000, np.float32))


def test_pc1_repeated_calls_of_different_sizes(ctx):
    """The min/max counter resets itself and the workspace is reused."""
    for k, (H, W) in enumerate([(120, 150), (40, 30), (120, 150), (7, 9)]):
        cube, mean, vec = inputs.g_cube(H, W, 128, 40 + k)
        say(f"pc1 repeated call {k} {H}x{W}")
        got = run_pc1(ctx, cube, mean, vec, True)
        assert_within_one_ulp(got, pc1_oracle.pc1(cube, mean, vec, True), f"call {k}")


def test_pc1_full_size_brain_cube(ctx):
    """W 480 x H 380, 128 bands: every pixel."""
    cube, mean, vec = inputs.g_cube(380, 480, 128, 1)
    say("pc1 full-size brain cube")
    got = run_pc1(ctx, cube, mean, vec, True)
    assert_within_one_ulp(got, pc1_oracle.pc1(cube, mean, vec, True), "full-size")


def test_pc1_feeds_the_filter(ctx):
    """Cube -> knnf_pc1 -> knnf_filter on the device; the filter is bit-exact
    against the oracle filter run on the same band."""
    import torch

    H, W, K, R = 60, 90, 16, 7
    cube, mean, vec = inputs.g_cube(H, W, 128, 8)
    _, prob = inputs.g_brain(H, W, 8)
    df = DeviceFrame(np.zeros((H, W), np.float32), prob, K, R, 0.01, with_nbr=True)
    dcube = torch.from_numpy(cube).cuda()
    dmean = torch.from_numpy(mean).cuda()
    dvec = torch.from_numpy(vec).cuda()
    say("pc1 -> filter")
    _lib.knnf_pc1(ctx, dcube.data_ptr(), H * W, 128, dmean.data_ptr(), dvec.data_ptr(),
                  df.pc1.data_ptr(), True, current_stream())
    _lib.knnf_filter(ctx, df.as_c(), None, current_stream())
    torch.cuda.synchronize()
    band = df.pc1.cpu().numpy()
    assert_within_one_ulp(band.reshape(-1), pc1_oracle.pc1(cube, mean, vec, True), "band")
    go, gc, gn, gd = df.results()
    ro, rc, rn, rd = oracle.knn_filter(band, prob, K, R, 0.01)
    assert np.array_equal(gn, rn) and np.array_equal(gc, rc)
    assert np.max(np.abs(go.astype(np.float64) - ro)) <= 1e-6
