"""GPU parity of UV-based pruning (pg_uv_prune) against the oracle: UV
pixels, ranks by opacity and the kept set must be bit-identical, with and
without the valid-projection check, for K = 0, 1, 3; several frames; the
16-frame window (sampled frame)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import atlas_tensor, renderer, say

pytestmark = pytest.mark.gpu

SCENES = {
    "tiny": lambda: synth.random_scene(side=12, sh_degree=1, views=1, width=64, height=48, seed=0),
    "multiframe": lambda: synth.random_scene(side=16, sh_degree=2, views=2, width=64, height=50, seed=2, frames=3),
    "config2": lambda: synth.make_scene(2),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def run(sc, M, Nv, K, expected=None):
    r = renderer(sc)
    e = None if expected is None else torch.from_numpy(np.ascontiguousarray(expected, np.int32).reshape(-1)).to("cuda:0")
    uv, rank, keep = r.uv_prune(atlas_tensor(sc), M, Nv, K, e)
    torch.cuda.synchronize()
    out = [a.cpu().numpy().reshape(sc.frames, r.N) for a in (uv, rank, keep)]
    r.close()
    return out


def reference(sc, M, Nv, K, expected=None):
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    res = [oracle.uv_prune(params[f], M, Nv, K, None if expected is None else expected[f]) for f in range(sc.frames)]
    return [np.stack([r[k] for r in res]) for k in range(3)]


@pytest.mark.parametrize("name", list(SCENES))
def test_uv_prune_bit_exact(name):
    sc = SCENES[name]()
    M, Nv = (16, 8) if name != "config2" else (64, 32)
    for K in (0, 1, 3):
        got = run(sc, M, Nv, K)
        ref = reference(sc, M, Nv, K)
        for a, b, what in zip(got, ref, ("uv", "rank", "keep")):
            assert np.array_equal(a.astype(np.int64), b.astype(np.int64)), f"{name} K={K}: {what} differs"
        say(f"[gpu] uv prune {name} K={K}: kept {int(ref[2].sum())} of {ref[2].size}, max rank {int(ref[1].max())}")
    # valid projection: half the Gaussians are told a wrong pixel
    uv_true = reference(sc, M, Nv, 1)[0]
    rng = np.random.default_rng(5)
    exp = np.where(rng.random(uv_true.shape) < 0.5, uv_true, (uv_true + 1) % (M * Nv)).astype(np.int32)
    got = run(sc, M, Nv, 2, exp)
    ref = reference(sc, M, Nv, 2, exp)
    for a, b in zip(got, ref):
        assert np.array_equal(a.astype(np.int64), b.astype(np.int64))


def test_uv_prune_temporal_window_sampled_frame():
    sc = synth.make_scene(4)
    M, Nv, K = 512, 256, 2
    got = run(sc, M, Nv, K)
    f = int(np.random.default_rng(6).integers(sc.frames))
    ids, params = oracle.fetch(sc.atlas[f:f + 1], sc.occupancy)
    ref = oracle.uv_prune(params[0], M, Nv, K)
    for a, b in zip(got, ref):
        assert np.array_equal(a[f].astype(np.int64), np.asarray(b, np.int64))
    say(f"[gpu] uv prune window frame {f}: kept {int(ref[2].sum())} of {len(ref[2])}")


def test_uv_prune_degenerate_cases():
    """No Gaussians at all; a map of one pixel (every valid Gaussian shares it,
    so K keeps exactly the K largest opacities); K beyond every pixel count."""
    sc = synth.random_scene(side=4, sh_degree=0, views=1, width=40, height=24, seed=0)
    sc.occupancy[:] = 0
    sc.atlas[:] = 0
    uv, rank, keep = run(sc, 8, 4, 2)
    assert uv.size == 0 and rank.size == 0 and keep.size == 0
    sc = SCENES["tiny"]()
    for M, Nv, K in ((1, 1, 5), (16, 8, 10 ** 6)):
        got = run(sc, M, Nv, K)
        ref = reference(sc, M, Nv, K)
        for a, b in zip(got, ref):
            assert np.array_equal(a.astype(np.int64), b.astype(np.int64)), (M, Nv, K)
    say(f"[gpu] uv prune one-pixel map: kept {int(ref[2].sum())}; empty atlas: nothing")
