"""pg_atlas_fetch_noalloc (the fetch whose workspace is the library's fixed
per-GPU scratch array) against pg_atlas_fetch with a caller workspace, through
the C ABI: ids, the texel -> id map, the gathered channels and the count must
be bit-identical.  Three calls in a row on one stream, each smaller than the
one before it (the largest at the documented maximum of 8192 x 8192 texels),
so a later call runs over what the earlier one left in the scratch."""
import numpy as np
import pytest
import torch

from paper_2602_23040_amd import _abi as abi

pytestmark = pytest.mark.gpu

CASES = [  # (frames, channels, H, W, occupancy probability, seed)
    (1, 2, 8192, 8192, 0.75, 11),
    (1, 59, 512, 512, 0.85, 12),
    (2, 14, 48, 67, 0.6, 13),
]


def _inputs(F, C, H, W, p, seed):
    g = torch.Generator(device="cuda:0").manual_seed(seed)
    occ = (torch.rand(H * W, generator=g, device="cuda:0") < p).to(torch.uint8)
    atlas = torch.randn(F * C * H * W, generator=g, device="cuda:0")
    return atlas, occ


def _outputs(F, C, H, W, n_cap, fill):
    dev = "cuda:0"
    return (torch.full((n_cap,), fill, dtype=torch.int32, device=dev),
            torch.full((H * W,), fill, dtype=torch.int32, device=dev),
            torch.full((F * C * n_cap,), float(fill), dtype=torch.float32, device=dev),
            torch.full((1,), fill, dtype=torch.int64, device=dev))


def test_fetch_noalloc_matches_fetch_on_calls_of_falling_size():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.lib()
    abi._check(abi.lib().pg_init(0), "pg_init")
    for F, C, H, W, p, seed in CASES:
        print(f"[case] fetch_noalloc F={F} C={C} H={H} W={W} p={p} seed={seed}", flush=True)
        atlas, occ = _inputs(F, C, H, W, p, seed)
        n_cap = H * W
        ref = _outputs(F, C, H, W, n_cap, -3)
        got = _outputs(F, C, H, W, n_cap, -7)
        ws_bytes = abi.pg_fetch_workspace_size(H, W)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0")
        abi.pg_atlas_fetch(atlas, occ, F, C, H, W, n_cap, *ref, ws, ws_bytes)
        abi.pg_atlas_fetch_noalloc(atlas, occ, F, C, H, W, n_cap, *got)
        torch.cuda.synchronize()
        n = int(ref[3].item())
        assert n == int(got[3].item()) == int(occ.sum().item())
        assert torch.equal(ref[0][:n], got[0][:n])
        assert torch.equal(ref[1], got[1])
        pr = ref[2].view(F * C, n_cap)[:, :n]
        pg = got[2].view(F * C, n_cap)[:, :n]
        assert torch.equal(pr.view(torch.int32), pg.view(torch.int32))
        # untouched tails keep the caller's fill
        assert bool((got[0][n:] == -7).all()) and bool((got[2].view(F * C, n_cap)[:, n:] == -7.0).all())
        del atlas, occ, ref, got, ws
        torch.cuda.empty_cache()


def test_fetch_noalloc_respects_a_small_capacity():
    """n_cap below the occupied count: ids past the capacity are not
    written and map to -1, exactly as pg_atlas_fetch does."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi._check(abi.lib().pg_init(0), "pg_init")
    F, C, H, W = 1, 3, 100, 130
    atlas, occ = _inputs(F, C, H, W, 0.5, 21)
    for n_cap in (1000, 0):
        print(f"[case] fetch_noalloc small capacity n_cap={n_cap}", flush=True)
        ref = _outputs(F, C, H, W, max(n_cap, 1), -3)
        got = _outputs(F, C, H, W, max(n_cap, 1), -7)
        ws_bytes = abi.pg_fetch_workspace_size(H, W)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0")
        abi.pg_atlas_fetch(atlas, occ, F, C, H, W, n_cap, *ref, ws, ws_bytes)
        abi.pg_atlas_fetch_noalloc(atlas, occ, F, C, H, W, n_cap, *got)
        torch.cuda.synchronize()
        assert int(ref[3].item()) == int(got[3].item()) == int(occ.sum().item())
        assert torch.equal(ref[1], got[1])
        assert int((got[1] >= 0).sum().item()) == n_cap
        if n_cap:
            assert torch.equal(ref[0][:n_cap], got[0][:n_cap])
            assert torch.equal(ref[2].view(torch.int32), got[2].view(torch.int32))
