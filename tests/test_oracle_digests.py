"""The stored whole-frame oracle digests (tests/golden/oracle_digests.json)
agree with the oracle run now, on the frames small enough to recompute in a
CPU test: the 50 x 50 frames of the served mix and the smallest of the 64
uneven frames.  Guards the file against a stale write or a changed generator.
"""
import importlib.util
import json
import os

import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _dig():
    spec = importlib.util.spec_from_file_location("oracle_digests",
                                                  os.path.join(GOLDEN, "oracle_digests.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def stored():
    with open(os.path.join(GOLDEN, "oracle_digests.json")) as f:
        return json.load(f)


def test_every_frame_has_a_record(stored):
    from paper_2404_10631_amd import inputs

    dig = _dig()
    assert len(stored["config2"]) == len(inputs.config2().frames) == 64
    assert len(stored["config4"]) == len(dig.config4_stream()) == 40
    for name, specs in (("config2", inputs.config2().frames),
                        ("config4", [s for _, _, s in dig.config4_stream()])):
        for s, r in zip(specs, stored[name]):
            assert (r["gen"], r["H"], r["W"], r["seed"], r["K"], r["R"]) == \
                (s.gen, s.H, s.W, s.seed, s.K, s.R)
            for key in ("inputs", "nbr", "dist", "class", "prob"):
                assert len(r[key]) == 64


def test_small_frames_recomputed(stored):
    from paper_2404_10631_amd import inputs

    dig = _dig()
    cases = [(s, stored["config4"][k]) for k, (_, _, s) in enumerate(dig.config4_stream())
             if s.H * s.W <= 2500][:6]
    c2 = inputs.config2().frames
    k2 = min(range(len(c2)), key=lambda k: c2[k].H * c2[k].W)
    cases.append((c2[k2], stored["config2"][k2]))
    assert len(cases) >= 4
    for s, want in cases:
        data = s.make()
        outs = oracle.knn_filter(data[0], data[1], s.K, s.R, s.lam, with_nbr=True)
        assert dig.frame_record(s, outs, data) == want, f"{s.H}x{s.W} seed {s.seed}"
