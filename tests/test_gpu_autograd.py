"""PackUVRender, the torch.autograd.Function around the forward chain and the
hand-written adjoint (pg_backward), on the ring-of-8 workload (256^2 atlas,
SH 3, eight 512x512 views): atlas.grad from loss.backward() against the FP64
oracle's dL/datlas under the gradient rule (per element 1e-3 relative with a
floor of 1 % of the channel's largest magnitude, 1e-3 relative L2 per
channel), both sides taking the same image cotangent.

Also: an eager step that overflows its instance capacity grows and renders
again inside the function (never the background an overflowed sort leaves);
a backward after the renderer has run another forward raises; the function
refuses graph capture."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2602_23040_amd.pipeline import PackUVRender
from parity import atlas_tensor, explain, gpu_images, grad_compare, renderer, say

pytestmark = pytest.mark.gpu

_case = {}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    _case.clear()


def ring():
    if "ring" not in _case:
        say("[case] ring of 8 (256^2 atlas, 8 x 512^2): scene and oracle forward")
        sc = synth.make_scene(2)
        _case["ring"] = (sc, oracle.Forward(sc))
    return _case["ring"]


def leaf_atlas(sc):
    return atlas_tensor(sc).reshape(sc.frames, sc.C, sc.H, sc.W).clone().requires_grad_()


def flips_of(fw, r):
    imgs = gpu_images(r)
    flips = {}
    for v in fw.views:
        fl, unexp, _ = explain(fw, v, imgs[v][0], imgs[v][1])
        assert not unexp, f"view {v}: {len(unexp)} unexplained pixels"
        if fl:
            flips[v] = fl
    return flips


def compare_atlas_grad(sc, got, ref):
    occ = sc.occupancy.astype(bool).reshape(-1)
    got = got.reshape(sc.frames, sc.C, -1)
    ref = ref.reshape(sc.frames, sc.C, -1)
    assert np.all(got[:, :, ~occ] == 0.0)
    st = grad_compare(got[:, :, occ], ref[:, :, occ])
    say(f"[gpu] autograd dL/datlas: {st}")
    assert st["n_bad"] == 0 and st["worst_l2"] <= 1e-3, st


def test_autograd_fixed_cotangent_matches_oracle():
    """loss = <G, images> with a seeded G: atlas.grad is the adjoint applied to G."""
    sc, fw = ring()
    r = renderer(sc)
    atlas = leaf_atlas(sc)
    img = PackUVRender.apply(atlas, r)
    assert img.shape == (3 * r.n_pixels,) and img.requires_grad
    rng = np.random.default_rng(402)
    G = {v: rng.standard_normal(fw.image[v].shape) for v in fw.views}
    Gt = torch.from_numpy(np.concatenate([G[v].reshape(-1) for v in fw.views]).astype(np.float32)).to("cuda:0")
    (Gt * img).sum().backward()
    torch.cuda.synchronize()
    assert atlas.grad.shape == atlas.shape
    ref, _ = fw.backward(G, flips=flips_of(fw, r))
    compare_atlas_grad(sc, atlas.grad.cpu().numpy().astype(np.float64), ref)
    r.close()


def test_autograd_l1_loss_end_to_end():
    """loss = mean |images - target| computed by torch: autograd hands the
    adjoint torch's own L1 cotangent.  The oracle takes that same cotangent;
    the pixels where its sign differs from the oracle's own L1 sign (residual
    within the image tolerance of zero) are counted and reported."""
    sc, fw = ring()
    r = renderer(sc)
    atlas = leaf_atlas(sc)
    rng = np.random.default_rng(502)
    targets = {v: rng.uniform(0, 1, fw.image[v].shape) for v in fw.views}
    tgt = torch.from_numpy(np.concatenate([targets[v].reshape(-1) for v in fw.views]).astype(np.float32)).to("cuda:0")
    img = PackUVRender.apply(atlas, r)
    loss = (img - tgt).abs().mean()
    loss.backward()
    torch.cuda.synchronize()
    n = img.numel()
    cot = (torch.sign(img.detach() - tgt) / n).double().cpu().numpy()
    L_ref, G_ref = fw.loss(targets)
    assert abs(float(loss.detach()) - L_ref) <= 1e-6 * max(1.0, L_ref)
    G, o = {}, 0
    for v in fw.views:
        k = fw.image[v].size
        G[v] = cot[o:o + k].reshape(fw.image[v].shape)
        o += k
    flips_sign = int(sum(int((np.sign(G[v]) != np.sign(G_ref[v])).sum()) for v in fw.views))
    say(f"[gpu] autograd L1: loss {float(loss.detach()):.9f} (oracle {L_ref:.9f}); cotangent sign flips against the "
        f"oracle's own: {flips_sign}")
    ref, _ = fw.backward(G, flips=flips_of(fw, r))
    compare_atlas_grad(sc, atlas.grad.cpu().numpy().astype(np.float64), ref)
    r.close()


def test_autograd_grows_after_an_overflow():
    """A renderer whose instance capacity is far too small: the function's
    forward grows it to the reported count and renders again; the image and
    the gradient equal those of a renderer that had room from the start."""
    sc = synth.random_scene(side=16, sh_degree=2, views=3, width=90, height=64, seed=12, lscale=(-2.9, 0.5))
    fw = oracle.Forward(sc)
    small, roomy = renderer(sc, cap=32), renderer(sc, cap=1 << 20)
    out = []
    for r in (small, roomy):
        atlas = leaf_atlas(sc)
        img = PackUVRender.apply(atlas, r)
        img.square().sum().backward()
        torch.cuda.synchronize()
        assert r.check()
        out.append((img.detach().clone(), atlas.grad.clone()))
    assert small.sets[0].cap > 32
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    flips_of(fw, small)
    small.close()
    roomy.close()


def test_autograd_refuses_a_stale_backward():
    sc = synth.random_scene(side=8, sh_degree=0, views=2, width=48, height=32, seed=4, lscale=(-2.8, 0.5))
    r = renderer(sc)
    a1, a2 = leaf_atlas(sc), leaf_atlas(sc)
    img1 = PackUVRender.apply(a1, r)
    img2 = PackUVRender.apply(a2, r)
    with pytest.raises(RuntimeError, match="another forward"):
        img1.sum().backward()
    img2.sum().backward()            # the latest forward's backward is fine
    torch.cuda.synchronize()
    assert torch.isfinite(a2.grad).all()
    r.close()


def test_autograd_refuses_graph_capture(monkeypatch):
    """The capture guard, exercised without a capture: the function asks
    torch whether the current stream is capturing and raises before any
    library call when it is."""
    sc = synth.random_scene(side=8, sh_degree=0, views=1, width=32, height=32, seed=4, lscale=(-2.8, 0.5))
    r = renderer(sc)
    gen = r.generation
    monkeypatch.setattr(torch.cuda, "is_current_stream_capturing", lambda: True)
    with pytest.raises(RuntimeError, match="cannot be captured"):
        PackUVRender.apply(leaf_atlas(sc), r)
    monkeypatch.undo()
    assert r.generation == gen
    r.close()
