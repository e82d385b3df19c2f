"""GPU parity of covariance-aware flow masking (pg_flow_mask, Algorithm 1)
against the oracle: the dynamic label of every Gaussian of every frame
(OR over the frame's views) and its texel form must be bit-identical; the
texel form, used as the gradient-freezing mask, zeroes the adjoint on static
texels; empty and full masks; a sampled frame of the 16-frame window."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import atlas_tensor, renderer, run_forward, say

pytestmark = pytest.mark.gpu

SCENES = {
    "tiny": lambda: synth.random_scene(side=12, sh_degree=1, views=3, width=72, height=56, seed=0,
                                       lscale=(-2.8, 0.5)),
    "multiframe": lambda: synth.random_scene(side=10, sh_degree=2, views=4, width=64, height=50, seed=2, frames=3,
                                             lscale=(-2.7, 0.5), dynamic_frac=0.5),
    "config2": lambda: synth.make_scene(2),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def oracle_labels(sc, masks, frames=None):
    """(F, N) labels: per frame, the OR over its views of the oracle's masking."""
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    N = params.shape[2]
    D = np.zeros((sc.frames, N), np.uint8)
    base = np.concatenate([[0], np.cumsum([c.width * c.height for c in sc.cams])])
    for v, cam in enumerate(sc.cams):
        if frames is not None and cam.frame not in frames:
            continue
        m = masks[base[v]:base[v + 1]].reshape(cam.height, cam.width)
        oracle.flow_mask(params[cam.frame], sc.sh_degree, cam, m, D[cam.frame])
    return ids, D


def gpu_labels(sc, masks):
    r = renderer(sc)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    dg, dt = r.flow_mask(atlas_tensor(sc), torch.from_numpy(masks).to("cuda:0"), counters=cnt)
    torch.cuda.synchronize()
    out = dg.cpu().numpy().reshape(sc.frames, r.N), dt.cpu().numpy().reshape(sc.H, sc.W), int(cnt.item())
    r.close()
    return out


@pytest.mark.parametrize("name", list(SCENES))
def test_flow_mask_bit_exact(name):
    sc = SCENES[name]()
    masks = synth.flow_masks(sc, seed=40, coverage=0.02, mean_radius=0.02)
    say(f"[gpu] flow mask {name}: {len(sc.cams)} views, F={sc.frames}")
    D, Dt, tests = gpu_labels(sc, masks)
    ids, ref = oracle_labels(sc, masks)
    assert np.array_equal(D, ref), f"labels differ at {np.argwhere(D != ref)[:5].tolist()}"
    assert 0 < ref.sum() < ref.size, "the masks must split the Gaussians"
    exp_t = np.zeros(sc.H * sc.W, np.uint8)
    exp_t[ids] = ref.max(axis=0)
    assert np.array_equal(Dt.reshape(-1), exp_t)
    assert tests > 0
    say(f"[gpu] flow mask {name}: {int(ref.sum())} of {ref.size} dynamic, {tests} pixel tests")


def test_flow_mask_empty_and_full():
    sc = SCENES["tiny"]()
    P = sum(c.width * c.height for c in sc.cams)
    D, Dt, tests = gpu_labels(sc, np.zeros(P, np.uint8))
    assert not D.any() and not Dt.any() and tests == 0
    full = np.ones(P, np.uint8)
    D, _, _ = gpu_labels(sc, full)
    _, ref = oracle_labels(sc, full)
    assert np.array_equal(D, ref)


def test_labels_freeze_the_adjoint():
    """The texel labels as the freezing mask: static texels get exactly zero
    gradient, dynamic ones the unfrozen gradient, bit for bit."""
    sc = SCENES["multiframe"]()
    masks = synth.flow_masks(sc, seed=41, coverage=0.01, mean_radius=0.02)
    r = renderer(sc, dynamic=None)
    atlas = atlas_tensor(sc)
    _, dt = r.flow_mask(atlas, torch.from_numpy(masks).to("cuda:0"))
    dyn = dt.clone()
    run_forward(r, atlas)
    g = torch.rand(3 * r.n_pixels, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(3))
    free = r.backward(g).clone()
    r.dynamic = dyn
    frozen = r.backward(g).clone()
    torch.cuda.synchronize()
    F, C = sc.frames, sc.C
    fr = frozen.reshape(F, C, -1)
    fe = free.reshape(F, C, -1)
    d = dyn.bool()
    assert 0 < int(d.sum()) < int(torch.from_numpy(sc.occupancy.reshape(-1)).sum())
    assert torch.equal(fr[:, :, ~d], torch.zeros_like(fr[:, :, ~d]))
    assert torch.equal(fr[:, :, d], fe[:, :, d])
    r.close()


def test_temporal_window_sampled_frame():
    """The 16-frame window (8 ring views per frame, 1080p and 720p): every
    frame labelled on the GPU; one sampled frame against the oracle."""
    sc = synth.make_scene(4)
    masks = synth.flow_masks(sc, seed=44, coverage=0.02, mean_radius=0.02)
    say(f"[gpu] flow mask temporal window: {len(sc.cams)} views, N = {sc.n_gauss} per frame")
    D, Dt, tests = gpu_labels(sc, masks)
    f = int(np.random.default_rng(4).integers(sc.frames))
    ids, ref = oracle_labels(sc, masks, frames={f})
    assert np.array_equal(D[f], ref[f])
    say(f"[gpu] frame {f}: {int(ref[f].sum())} of {ref.shape[1]} dynamic; {tests} pixel tests in the window")
