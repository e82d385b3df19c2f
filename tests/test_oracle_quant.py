"""Pins of the oracle's LPO fake quantiser (uniform K-bit proxy with a
per-channel min/max scale; Sec. 4.3 LPO paragraph, supplementary
low-precision training and video-coding sections).

Each test checks the oracle against something other than itself: numpy's
round-half-to-even on a grid whose step is exactly 1, a brute-force search
for the nearest quantisation level, the endpoints and monotonicity the
definition fixes, and the texels and channels it must leave alone."""
import numpy as np

import oracle


def _atlas(values, F=1, H=None, W=None):
    v = np.asarray(values, np.float32).reshape(-1)
    n = v.size
    W = W or n
    H = H or 1
    a = np.zeros((F, 1, H, W), np.float32)
    a.reshape(F, -1)[:, :n] = v
    return a


def test_unit_step_grid_matches_numpy_rint():
    """lo = 0, hi = 255, K = 8: delta is exactly 1, so the codes are numpy's
    rint of the values (ties to even) and the proxy is the code itself."""
    rng = np.random.default_rng(3)
    v = np.concatenate([[0.0, 255.0, 2.5, 3.5, 100.5, 254.5, 0.5],
                        rng.uniform(0, 255, 500)]).astype(np.float32)
    a = _atlas(v)
    occ = np.ones(a.shape[2:], np.uint8)
    q, r, codes = oracle.fake_quant(a, occ, [8])
    assert r.tolist() == [[0.0, 255.0]]
    expect = np.rint(v.astype(np.float64))
    assert np.array_equal(codes.reshape(-1)[:v.size], expect.astype(np.uint16))
    assert np.array_equal(q.reshape(-1)[:v.size], expect.astype(np.float32))
    assert codes.reshape(-1)[2] == 2 and codes.reshape(-1)[3] == 4   # ties to even


def test_codes_are_nearest_levels_by_brute_force():
    """Every code is (up to 1e-5 of a step) the nearest of all 2^K levels."""
    rng = np.random.default_rng(5)
    for K in (3, 4, 8):
        v = rng.normal(0.3, 2.0, 2000).astype(np.float32)
        a = _atlas(v)
        occ = np.ones(a.shape[2:], np.uint8)
        q, r, codes = oracle.fake_quant(a, occ, [K])
        lo, hi = float(v.min()), float(v.max())
        assert r[0].tolist() == [np.float32(lo), np.float32(hi)]
        step = (hi - lo) / (2 ** K - 1)
        levels = lo + step * np.arange(2 ** K)
        dist = np.abs(v.astype(np.float64)[:, None] - levels[None, :])
        best = dist.min(axis=1)
        got = dist[np.arange(v.size), codes.reshape(-1)[:v.size].astype(np.int64)]
        assert np.all(got <= best + 1e-5 * step), K
        # the proxy is the chosen level (to FP32 rounding)
        assert np.allclose(q.reshape(-1)[:v.size], levels[codes.reshape(-1)[:v.size]], rtol=0, atol=4e-7 * max(abs(lo), abs(hi)))


def test_endpoints_monotonic_and_error_bound():
    rng = np.random.default_rng(9)
    v = np.sort(rng.uniform(-7.0, 3.0, 3000)).astype(np.float32)
    a = _atlas(v)
    occ = np.ones(a.shape[2:], np.uint8)
    K = 8
    q, r, codes = oracle.fake_quant(a, occ, [K])
    c = codes.reshape(-1)[:v.size].astype(np.int64)
    p = q.reshape(-1)[:v.size].astype(np.float64)
    assert c[0] == 0 and p[0] == v[0]                      # min -> code 0, proxy = lo exactly
    assert c[-1] == 2 ** K - 1                             # max -> top code
    assert abs(p[-1] - v[-1]) <= 4 * np.spacing(np.float32(abs(v[-1]) + abs(v[0])))
    assert np.all(np.diff(c) >= 0)                         # monotone in the value
    step = (float(v[-1]) - float(v[0])) / (2 ** K - 1)
    assert np.all(np.abs(p - v) <= 0.5 * step * (1 + 1e-5) + 1e-6)


def test_range_spans_all_frames_and_only_occupied_texels():
    """min/max run over every frame, and unoccupied texels neither set the
    range nor change."""
    F, H, W = 2, 3, 4
    a = np.zeros((F, 2, H, W), np.float32)
    rng = np.random.default_rng(11)
    a[:] = rng.uniform(-1, 1, a.shape)
    occ = np.ones((H, W), np.uint8)
    occ[0, 0] = 0
    a[0, 0, 0, 0] = -50.0          # unoccupied: must not set lo
    a[1, 0, 2, 3] = 9.0            # occupied, frame 1: sets hi
    q, r, codes = oracle.fake_quant(a, occ, [8, 0])
    m = occ.astype(bool)
    assert r[0, 0] == a[:, 0][:, m].min() and r[0, 1] == 9.0
    assert q[0, 0, 0, 0] == -50.0 and codes[0, 0, 0, 0] == 0
    assert np.array_equal(q[:, 1], a[:, 1]) and not codes[:, 1].any() and r[1].tolist() == [0.0, 0.0]
    assert q[1, 0, 2, 3] == 9.0 and codes[1, 0, 2, 3] == 255


def test_constant_channel_and_empty_occupancy():
    a = np.full((1, 1, 2, 2), 0.75, np.float32)
    occ = np.ones((2, 2), np.uint8)
    q, r, codes = oracle.fake_quant(a, occ, [16])
    assert np.array_equal(q, a) and not codes.any() and r[0].tolist() == [0.75, 0.75]
    q, r, codes = oracle.fake_quant(a, np.zeros((2, 2), np.uint8), [8])
    assert np.array_equal(q, a) and not codes.any() and r[0].tolist() == [0.0, 0.0]


def test_sixteen_bit_codes_split_into_two_bytes():
    """A 16-bit code is stored as two 8-bit planes (high, low byte); the
    split is exact and the 16-bit grid is 257 times finer than the 8-bit one."""
    rng = np.random.default_rng(13)
    v = rng.uniform(-1, 1, 4000).astype(np.float32)
    a = _atlas(v)
    occ = np.ones(a.shape[2:], np.uint8)
    q16, _, c16 = oracle.fake_quant(a, occ, [16])
    q8, _, _ = oracle.fake_quant(a, occ, [8])
    c = c16.reshape(-1)[:v.size].astype(np.int64)
    hi_b, lo_b = c >> 8, c & 0xFF
    assert np.array_equal(hi_b * 256 + lo_b, c) and hi_b.max() <= 255
    e16 = np.abs(q16.reshape(-1)[:v.size] - v).max()
    e8 = np.abs(q8.reshape(-1)[:v.size] - v).max()
    assert e16 < e8 / 100
