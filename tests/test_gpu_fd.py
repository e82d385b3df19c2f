"""GPU texel gradients against finite differences of the FP64 oracle on the
ring-of-8 workload (256^2 atlas, 8 views of 512^2, SH 3): 64 visible
Gaussians (seeded draw) on all 59 channels, plus 4 invisible ones that must
read exactly zero.  The GPU gradient is atlas.grad of <G, images> through
PackUVRender (the torch.autograd.Function around the forward and the
hand-written adjoint).  Both sides take the same fixed image cotangent G, so
the reference is d<G, I(theta)>/dtheta; the oracle's difference keeps its own
footprint decisions fixed and is Richardson-extrapolated,
(4 D(h/2) - D(h)) / 3 with h = 1e-3.  Acceptance: per element
|g - d| <= 1e-3 max(|d|, 0.01 max over the channel |d|), and per channel
||g - d|| <= 1e-3 ||d||."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2602_23040_amd.pipeline import PackUVRender
from parity import atlas_tensor, renderer, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def test_texel_gradient_matches_oracle_finite_differences():
    sc = synth.make_scene(2)
    fw = oracle.Forward(sc)
    rng = np.random.default_rng(402)
    G = {v: rng.standard_normal(fw.image[v].shape) for v in fw.views}
    r = renderer(sc, dynamic=None)
    # through the autograd function: atlas.grad of <G, images>
    atlas = atlas_tensor(sc).reshape(sc.frames, sc.C, sc.H, sc.W).clone().requires_grad_()
    img = PackUVRender.apply(atlas, r)
    g = torch.from_numpy(np.concatenate([G[v].reshape(-1) for v in fw.views]).astype(np.float32)).to("cuda:0")
    (g * img).sum().backward()
    torch.cuda.synchronize()
    C = sc.C
    got = atlas.grad.cpu().numpy().reshape(sc.frames, C, -1)[0][:, fw.ids].astype(np.float64)
    vis = fw.visible()[0].astype(bool)
    pick = rng.choice(np.flatnonzero(vis), 64, replace=False)
    hidden = np.flatnonzero(~vis)[:4]
    fw.fd(G, 0, int(pick[0]), 0, 1e-3)       # first call initialises the oracle's tables
    jobs = [(int(i), ch) for i in pick for ch in range(C)]

    def richardson(job):
        i, ch = job
        h = 1e-3
        return (4.0 * fw.fd(G, 0, i, ch, h / 2) - fw.fd(G, 0, i, ch, h)) / 3.0

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        fd = np.array(list(ex.map(richardson, jobs))).reshape(len(pick), C).T    # [C][64]
    mine = got[:, pick]
    floor = 0.01 * np.abs(fd).max(axis=1, keepdims=True)
    bad = np.abs(mine - fd) > 1e-3 * np.maximum(np.abs(fd), floor)
    l2 = np.linalg.norm(mine - fd, axis=1) / np.maximum(np.linalg.norm(fd, axis=1), 1e-300)
    worst = int(np.argmax(l2))
    say(f"[gpu] finite differences: {len(jobs)} (texel, channel) pairs, {int(bad.sum())} beyond the rule, "
        f"worst channel {worst} rel L2 {l2[worst]:.2e}")
    assert not bad.any(), [(int(c), int(pick[k]), mine[c, k], fd[c, k]) for c, k in zip(*np.nonzero(bad))][:8]
    assert l2.max() <= 1e-3
    if len(hidden):
        assert np.all(got[:, hidden] == 0.0)
    r.close()
