"""GPU parity of the full photometric objective (pg_loss_photo: L1 / SSIM
blend) and of the scale / opacity regularisers against the oracle, and of a
fitting step that uses them.

The loss value must match to 1e-5 relative, the image cotangent to the
gradient rule (1e-3 relative per element with a floor of 1 % of the
channel's largest magnitude, 1e-3 relative L2 per channel).  Views of
ragged sizes exercise the zero-padded borders and partial 32 x 32 blocks."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2602_23040_amd import _abi as abi
from parity import atlas_tensor, explain, gpu_images, grad_compare, renderer, run_forward, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def ragged_scene():
    sc = synth.random_scene(side=16, sh_degree=1, views=3, width=72, height=56, seed=31, lscale=(-2.6, 0.6))
    # ragged sizes: a view that is not a multiple of 32 in either direction
    sc.cams[1].width, sc.cams[1].height = 45, 37
    sc.cams[1].cx, sc.cams[1].cy = 22.5, 18.5
    sc.cams[2].width, sc.cams[2].height = 100, 33
    sc.cams[2].cx, sc.cams[2].cy = 50.0, 16.5
    return sc


@pytest.mark.parametrize("lam", [0.0, 0.2, 1.0])
def test_photo_loss_matches_oracle(lam):
    sc = ragged_scene()
    r = renderer(sc)
    run_forward(r, atlas_tensor(sc))
    rng = np.random.default_rng(9)
    tgt = rng.uniform(0, 1, 3 * r.n_pixels).astype(np.float32)
    loss = float(r.loss_photo(torch.from_numpy(tgt).to("cuda:0"), lam).item())
    torch.cuda.synchronize()
    img = r.image.cpu().numpy()
    G = r.dL_dimage.cpu().numpy()
    imgs, tgts, offs = {}, {}, {}
    for v, c in enumerate(r.cams):
        o = 3 * r.pix_base[v]
        n = 3 * c.width * c.height
        imgs[v] = img[o:o + n].reshape(3, c.height, c.width).astype(np.float64)
        tgts[v] = tgt[o:o + n].reshape(3, c.height, c.width).astype(np.float64)
        offs[v] = (o, n)
    L, Gref = oracle.photo_loss(imgs, tgts, lam)
    say(f"[gpu] photo loss lam={lam}: {loss:.9g} vs {L:.9g}")
    assert abs(loss - L) <= 1e-5 * abs(L)
    got = np.concatenate([G[o:o + n] for (o, n) in offs.values()]).reshape(1, 3, -1)
    ref = np.concatenate([Gref[v].reshape(-1) for v in offs]).reshape(1, 3, -1)
    st = grad_compare(got, ref)
    say(f"[gpu] photo loss lam={lam} dL/dimage: {st}")
    assert st["n_bad"] == 0 and st["worst_l2"] <= 1e-3, st
    r.close()


def test_step_with_ssim_texel_gradient():
    """forward -> blended loss -> adjoint, against the oracle chain with the
    same target (the image cotangent comes from each side's own loss)."""
    sc = ragged_scene()
    lam = 0.2
    fw = oracle.Forward(sc)
    r = renderer(sc)
    atlas = atlas_tensor(sc)
    run_forward(r, atlas)
    imgs = gpu_images(r)
    flips = {}
    for v in range(len(sc.cams)):
        fl, unexp, _ = explain(fw, v, imgs[v][0], imgs[v][1])
        assert not unexp
        if fl:
            flips[v] = fl
    rng = np.random.default_rng(10)
    targets = {v: rng.uniform(0, 1, fw.image[v].shape) for v in fw.views}
    tflat = np.concatenate([targets[v].reshape(-1) for v in fw.views]).astype(np.float32)
    r.step(atlas, torch.from_numpy(tflat).to("cuda:0"), lambda_ssim=lam)
    torch.cuda.synchronize()
    _, G = oracle.photo_loss({v: fw.image[v] for v in fw.views}, {v: targets[v].astype(np.float32).astype(np.float64) for v in fw.views}, lam)
    ref_atlas, _ = fw.backward(G, flips=flips)
    got = r.dL_datlas.cpu().numpy().reshape(sc.frames, sc.C, sc.H, sc.W)
    occ = sc.occupancy.astype(bool)
    st = grad_compare(got.reshape(sc.frames, sc.C, -1)[:, :, occ.reshape(-1)],
                      ref_atlas.reshape(sc.frames, sc.C, -1)[:, :, occ.reshape(-1)])
    say(f"[gpu] step with SSIM dL/datlas: {st}")
    assert st["n_bad"] == 0 and st["worst_l2"] <= 1e-3, st
    r.close()


def test_regularisers_match_oracle():
    """Scale / opacity regularisers on every Gaussian and on a dynamic subset:
    means to 1e-6, texel gradient to the gradient rule (FP64 on both sides)."""
    sc = synth.random_scene(side=14, sh_degree=1, views=2, width=64, height=48, seed=33, frames=2,
                            lscale=(-1.2, 0.8))
    r = renderer(sc)
    r.fetch(atlas_tensor(sc))
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    F, C, N = params.shape
    s_max, ws, wo = float(np.exp(-1.0)), 0.7, 1.3
    rng = np.random.default_rng(12)
    dyn = (rng.random((F, N)) < 0.4).astype(np.uint8)
    for d in (None, dyn):
        r.dL_datlas.zero_()
        dt = None if d is None else torch.from_numpy(d.reshape(-1)).to("cuda:0")
        loss = r.regularisers(s_max, ws, wo, dt).cpu().numpy()
        Ls, Lo, g, n = oracle.regularisers(params, s_max, ws, wo, dyn=d)
        say(f"[gpu] regularisers ({n} Gaussians): {loss.tolist()} vs {[Ls, Lo]}")
        assert Ls > 0 and abs(loss[0] - Ls) <= 1e-6 * Ls and abs(loss[1] - Lo) <= 1e-6 * Lo
        got = r.dL_datlas.cpu().numpy().reshape(F, C, -1)[:, :, ids]
        st = grad_compare(got[:, [3, 4, 5, 10]], g[:, [3, 4, 5, 10]])
        assert st["n_bad"] == 0 and st["worst_l2"] <= 1e-3, st
        others = [c for c in range(C) if c not in (3, 4, 5, 10)]
        assert not got[:, others].any()
    r.close()


@pytest.mark.parametrize("batched", [True, False])
def test_fused_l1_adjoint_equals_the_separate_calls(batched):
    """pg_render_bwd_l1 + pg_loss_l1_tiles (the step's L1 path) against
    pg_loss_l1 + pg_render_bwd: the same slots and texel gradients bit for bit,
    and the loss value of the same sums in another order (FP32 inside rows of
    16 lanes: within 1e-5 relative); with ragged
    views, tiles partly outside the image, and one loss over several view
    tables in the plain path."""
    sc = ragged_scene()
    r = renderer(sc, batched=batched)
    run_forward(r, atlas_tensor(sc))
    rng = np.random.default_rng(41)
    tgt = torch.from_numpy(rng.uniform(0, 1, 3 * r.n_pixels).astype(np.float32)).to("cuda:0")
    r.loss_l1(tgt)
    g_sep = r.backward().clone()
    loss_sep = float(r.loss.item())
    slots_sep = [s.inst_grad.clone() for s in r.sets]
    r.dL_datlas.fill_(float("nan"))
    r.loss.fill_(float("nan"))
    r.backward_l1(tgt)
    torch.cuda.synchronize()
    loss_fused = float(r.loss.item())
    say(f"[gpu] fused L1 adjoint (batched={batched}): loss {loss_fused:.9g} vs {loss_sep:.9g}")
    assert torch.equal(r.dL_datlas, g_sep)
    for s, ref in zip(r.sets, slots_sep):
        n = abi.SLOT_WORDS * int(s.n_inst[0].item())
        assert torch.equal(s.inst_grad[:n], ref[:n])
    assert abs(loss_fused - loss_sep) <= 1e-5 * abs(loss_sep)
    # the loss value against the oracle's
    img = r.image.cpu().numpy().astype(np.float64)
    assert abs(loss_fused - np.abs(img - tgt.cpu().numpy().astype(np.float64)).mean()) <= 1e-5 * loss_fused
    r.close()
