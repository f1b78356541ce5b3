"""Seeded input generators: published SplitMix64 outputs and recipe properties."""
import numpy as np

import synth


def test_splitmix64_reference_sequence():
    # SplitMix64 seeded with 0: its first three outputs are mix(G), mix(2G), mix(3G)
    # (Steele, Lea and Flood 2014; the widely published reference sequence).
    G, M = synth.G, synth.MASK
    assert synth.mix_int(G) == 0xE220A8397B1DCDAF
    assert synth.mix_int((2 * G) & M) == 0x6E789E6AA1B965F4
    assert synth.mix_int((3 * G) & M) == 0x06C45D188009454F


def test_vectorised_mix_matches_scalar():
    key = synth.stream_key(123, 1)
    idx = np.array([0, 1, 2, 10 ** 9, 2 ** 40], dtype=np.uint64)
    u = synth.u01(123, 1, idx)
    for i, v in zip(idx, u):
        h = synth.mix_int(key + (int(i) + 1) * synth.G)
        assert v == (h >> 11) * 2.0 ** -53


def test_window_equals_slice_of_full_field():
    shape = (5, 7, 9)
    full = synth.uniform_field(9, 0, shape, -0.1, 0.1)
    win = synth.uniform_field(9, 0, shape, -0.1, 0.1, origin=(3, 5, 7), wshape=(4, 4, 4))
    zz, yy, xx = np.meshgrid((np.arange(4) + 3) % 5, (np.arange(4) + 5) % 7, (np.arange(4) + 7) % 9, indexing="ij")
    assert np.array_equal(win, full[zz, yy, xx])
    u, v = synth.gray_scott_fields(4, shape, ncubes=3, side=2)
    uw, vw = synth.gray_scott_fields(4, shape, ncubes=3, side=2, origin=(3, 5, 7), wshape=(4, 4, 4))
    assert np.array_equal(uw, u[zz, yy, xx]) and np.array_equal(vw, v[zz, yy, xx])


def test_uniform_range_and_mean():
    x = synth.uniform_field(202, 0, (1, 256, 256), -0.05, 0.05)
    assert x.min() >= -0.05 and x.max() < 0.05
    assert abs(x.mean()) < 1e-3


def test_gray_scott_recipe():
    u, v = synth.gray_scott_fields(303, (32, 32, 32), ncubes=20, side=4, noise=0.01)
    inside = np.abs(u - 0.5) <= 0.01
    outside = np.abs(u - 1.0) <= 0.01
    assert np.all(inside | outside)
    assert np.all(np.abs(v[outside]) <= 0.01) and np.all(np.abs(v[inside] - 0.25) <= 0.01)
    assert 0 < inside.sum() <= 20 * 64


def test_serving_trace_shapes():
    tr = synth.serving_trace(200, seed=505, rate=10.0)
    assert len(tr) == 200
    assert all(64 <= r["shape"][2] <= 2048 if r["ndim"] == 2 else 32 <= r["shape"][0] <= 256 for r in tr)
    assert all(100 <= r["steps"] <= 10000 for r in tr)
    t = [r["arrival"] for r in tr]
    assert all(b >= a for a, b in zip(t, t[1:]))
    assert {r["kind"] for r in tr} == {1, 2, 3}
    # the same requests at any rate: only the arrivals change (and scale)
    for other in (synth.serving_trace(200, seed=505, rate=None), synth.serving_trace(200, seed=505, rate=5.0)):
        for a, b in zip(tr, other):
            assert {k: v for k, v in a.items() if k != "arrival"} == {k: v for k, v in b.items() if k != "arrival"}
    slow = synth.serving_trace(200, seed=505, rate=5.0)
    assert all(abs(b["arrival"] - 2.0 * a["arrival"]) <= 1e-9 * max(1.0, b["arrival"]) for a, b in zip(tr, slow))
    assert all(r["arrival"] == 0.0 for r in synth.serving_trace(20, seed=505))
