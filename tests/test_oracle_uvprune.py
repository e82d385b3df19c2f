"""Pins of the oracle's UV-based pruning (Sec. 4.2 pruning paragraph with the
UV projection equation of Sec. 3): the pixel of the axis directions and of
the two edges of the equation (theta = pi wraps, phi = pi stays in the last
row), and a numpy brute force (arctan2, arccos, floor, lexsort) for the
pixels, the ranks by opacity and the top-K kept set."""
import numpy as np

import oracle


def params(mu, logit=None):
    mu = np.asarray(mu, np.float64).reshape(-1, 3)
    P = np.zeros((14, len(mu)))
    P[0:3] = mu.T
    if logit is not None:
        P[10] = logit
    return P


def test_axis_directions_and_equation_edges():
    M, Nv = 8, 4
    mu = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 0, -1), (-1, 0, 0), (0, 0, 0), (0, -1, 0)]
    uv, rank, keep = oracle.uv_prune(params(mu), M, Nv, 4)
    # theta = 0 -> u = M/2; pi/2 -> 3M/4; -pi/2 -> M/4; pi -> M wraps to 0.  phi = pi/2 -> v = N/2
    exp = [2 * M + 4, 2 * M + 6, 0 * M + 4, (Nv - 1) * M + 4, 2 * M + 0, -1, 2 * M + 2]
    assert uv.tolist() == exp
    assert keep.tolist() == [1, 1, 1, 1, 1, 0, 1] and rank[5] == -1


def brute(P, M, Nv, K, expected=None):
    x, y, z = P[0], P[1], P[2]
    rho = np.sqrt(x * x + y * y + z * z)
    ok = rho > 0
    th = np.arctan2(y, x)
    ph = np.arccos(np.clip(z / np.where(ok, rho, 1.0), -1, 1))
    u = np.floor((np.pi + th) / (2 * np.pi) * M).astype(np.int64)
    v = np.floor(ph / np.pi * Nv).astype(np.int64)
    u[u >= M] -= M
    v[v >= Nv] = Nv - 1
    key = v * M + u
    if expected is not None:
        ok &= key == expected
    uv = np.where(ok, key, -1)
    idx = np.flatnonzero(ok)
    order = idx[np.lexsort((idx, -P[10][idx], key[idx]))]
    rank = np.full(P.shape[1], -1)
    start = 0
    for j, i in enumerate(order):
        if j and key[i] != key[order[j - 1]]:
            start = j
        rank[i] = j - start
    keep = (rank >= 0) & (rank < K)
    return uv, rank, keep


def test_matches_numpy_brute_force():
    rng = np.random.default_rng(7)
    N, M, Nv = 3000, 32, 16
    mu = rng.normal(size=(N, 3))
    logit = np.round(rng.normal(size=N), 1)          # ties on purpose
    P = params(mu, logit)
    for K in (1, 2, 5, 100):
        got = oracle.uv_prune(P, M, Nv, K)
        ref = brute(P, M, Nv, K)
        for a, b in zip(got, ref):
            assert np.array_equal(np.asarray(a, np.int64), np.asarray(b, np.int64)), K
    # a pixel holds several Gaussians, and K = 1 keeps one per occupied pixel
    uv, rank, keep = oracle.uv_prune(P, M, Nv, 1)
    assert rank.max() >= 3 and keep.sum() == len(np.unique(uv[uv >= 0]))
    # valid UV projection: only Gaussians at their expected pixel survive
    expected = np.where(rng.random(N) < 0.5, brute(P, M, Nv, 1)[0], 0).astype(np.int32)
    got = oracle.uv_prune(P, M, Nv, 3, expected)
    ref = brute(P, M, Nv, 3, expected)
    for a, b in zip(got, ref):
        assert np.array_equal(np.asarray(a, np.int64), np.asarray(b, np.int64))
