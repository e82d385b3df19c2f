"""Buffers and call chains for one fitting step of PackUV-GS splatting.

``Renderer`` owns every device buffer the C ABI needs (torch is used only to
allocate device memory and to supply the current stream) and runs the chain

    pg_atlas_fetch -> pg_project -> pg_bin_sort -> pg_render_fwd   (forward)
    pg_loss_l1                                                      (L1 term)
    pg_render_bwd -> pg_project_bwd                                 (adjoint)
    pg_adam_step                                                    (optional)

in one of two modes over the same kernels:

* batched: one view table holding every view (and frame); one call chain,
  no host synchronisation, so the whole step can be captured in a HIP graph
  and replayed;
* plain: one view table per view; each view runs its own
  project / bin-sort / render chain and the host reads that view's instance
  count (one synchronisation per view) before compositing it.

``PackUVRender`` wraps the forward and adjoint as a ``torch.autograd.Function``.

Instance capacity.  How many (Gaussian, tile) instances a step needs is
decided on the device.  A sort that would exceed the capacity sets the
overflow flag and leaves the step's outputs undefined (background images,
zero gradient).  The protocol is the C ABI's: ``pg_status_check`` after the
step reports the count that suffices, the caller grows the instance buffers
and runs the step again.

* Eager steps do this by themselves.  ``forward`` checks after the sort
  (one synchronisation) and, after an overflow, grows and renders again, so
  an eager image is never the undefined one.
* A captured step cannot synchronise.  The caller calls ``check()`` (or
  ``ensure_capacity()``) after each replay and re-captures after a growth,
  because the graph holds the old buffers.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _abi as abi


def _u8(x, device):
    return torch.as_tensor(np.ascontiguousarray(x, np.uint8)).to(device)


class _ViewSet:
    """One pg_views table plus the per-(view, Gaussian) and per-instance buffers."""

    def __init__(self, cams, frames, n_gauss, sh_degree, tiling, device, inst_capacity):
        self.cams = list(cams)
        self.handle = abi.pg_views_create(self.cams, frames, n_gauss, sh_degree, tiling)
        self.info = abi.pg_views_get_info(self.handle)
        self.tile_base, self.pix_base = abi.pg_views_offsets(self.handle, len(self.cams))
        n_gv = self.info.n_gv
        self.splats = torch.empty(max(n_gv, 1) * abi.SPLAT_BYTES // 4, dtype=torch.float32, device=device)
        self.bins = torch.empty(max(n_gv, 1) * abi.BIN_BYTES // 4, dtype=torch.int32, device=device)
        self.tiles = torch.empty(2 * max(n_gv, 1), dtype=torch.int64, device=device)   # pg_tile_set [n_gv]
        self.grad2d = torch.empty(max(9 * n_gv, 1), dtype=torch.float32, device=device)
        self.ranges = torch.empty(2 * max(self.info.n_tiles, 1), dtype=torch.int32, device=device)
        self.tile_entries = torch.empty(max(self.info.n_tiles, 1), dtype=torch.int32, device=device)
        self.order = torch.empty(max(self.info.n_tiles, 1), dtype=torch.int32, device=device)   # dispatch order
        self.inst_first = torch.empty(max(n_gv, 1), dtype=torch.int32, device=device)
        self.n_inst = torch.zeros(2, dtype=torch.int64, device=device)   # instances, sort generation
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)
        self.device = device
        self.set_capacity(inst_capacity)

    def set_capacity(self, cap):
        cap = int(max(cap, 1))
        self.cap = cap
        self.keys = torch.empty(cap, dtype=torch.int32, device=self.device)
        self.values = torch.empty(cap, dtype=torch.int32, device=self.device)
        self.entries = torch.empty(cap, dtype=torch.int32, device=self.device)
        # gradient slots, zero-filled once: a zero tag never matches a sort generation
        self.inst_grad = torch.zeros(abi.SLOT_WORDS * cap, dtype=torch.float32, device=self.device)
        self.ws_bytes = abi.pg_sort_workspace_size(self.handle, cap)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def close(self):
        if self.handle:
            abi.pg_views_destroy(self.handle)
            self.handle = None


class Renderer:
    """Device state for fitting one atlas window rendered into a set of views.

    occupancy: (H, W) uint8 (host array), shared by all frames.
    cams: camera objects with R (3x3), t, fx, fy, cx, cy, width, height, frame.
    """

    def __init__(self, occupancy, frames, sh_degree, cams, tiling=(16, 16, 256), batched=True, bg=(0.0, 0.0, 0.0),
                 dynamic=None, inst_capacity=None, device="cuda", init=True, quant_bits=None):
        """quant_bits: per-channel widths of the LPO fake quantiser (e.g.
        ``_abi.lpo_bits(C)``); None renders the FP32 texel values as they are."""
        self.device = torch.device(device)
        if init:
            abi.pg_init(self.device.index or 0)
        occ = np.ascontiguousarray(occupancy, np.uint8)
        self.H, self.W = occ.shape
        self.frames = int(frames)
        self.sh_degree = int(sh_degree)
        self.C = 11 + 3 * (self.sh_degree + 1) ** 2
        self.N = int(np.count_nonzero(occ))
        self.cams = list(cams)
        self.V = len(self.cams)
        self.bg = tuple(float(b) for b in bg)
        self.batched = bool(batched)
        # plain path: check each view's instance count on the host (False once
        # the capacities are known, e.g. to capture the per-view chain in a graph)
        self.plain_sync = True
        # dispatch the compositing kernels' tiles longest-first (pg_bin_sort's
        # tile order); False keeps the default order (neighbouring tiles together)
        self.tile_order = True
        self.tiling = abi.make_tiling(*tiling)
        dev = self.device
        self.occ = _u8(occ, dev)
        self.dynamic = None if dynamic is None else _u8(dynamic, dev)
        self.gauss_texel = torch.empty(max(self.N, 1), dtype=torch.int32, device=dev)
        self.texel_gauss = torch.empty(self.H * self.W, dtype=torch.int32, device=dev)
        self.params = torch.empty(max(self.frames * self.C * self.N, 1), dtype=torch.float32, device=dev)
        self.n_gauss_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.fetch_ws_bytes = abi.pg_fetch_workspace_size(self.H, self.W)
        self.fetch_ws = torch.empty(self.fetch_ws_bytes, dtype=torch.uint8, device=dev)
        self.quant_bits = None if quant_bits is None else [int(b) for b in quant_bits]
        if self.quant_bits is not None:
            assert len(self.quant_bits) == self.C
            self.quant_range = torch.zeros(2 * self.C, dtype=torch.float32, device=dev)
            self.quant_partial = torch.empty(2 * abi.QUANT_BLOCKS * self.C, dtype=torch.float32, device=dev)
        self.visible = torch.zeros(max(self.frames * self.N, 1), dtype=torch.uint8, device=dev)
        self.dL_datlas = torch.empty(self.frames * self.C * self.H * self.W, dtype=torch.float32, device=dev)
        self.loss_partial = torch.empty(1024, dtype=torch.float64, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        if inst_capacity is None:
            # first guess (about the tile count of a Gaussian at the 50-view workload);
            # the first eager forward reports the count that suffices and grows to it
            inst_capacity = max(4096, 2 * max(self.N, 1) * (self.V if batched else 1))
        if batched:
            self.sets = [_ViewSet(self.cams, self.frames, self.N, self.sh_degree, self.tiling, dev, inst_capacity)]
            self.pix_base = self.sets[0].pix_base
        else:
            self.sets = [_ViewSet([c], self.frames, self.N, self.sh_degree, self.tiling, dev, inst_capacity)
                         for c in self.cams]
            pb = [0]
            for c in self.cams:
                pb.append(pb[-1] + c.width * c.height)
            self.pix_base = pb
        self.n_pixels = self.pix_base[-1]
        # per-tile sums of |image - target| of the fused L1 adjoint, the view sets' tiles side by side
        self.tile_off = [0]
        for s in self.sets:
            self.tile_off.append(self.tile_off[-1] + s.info.n_tiles)
        self.tile_loss = torch.empty(max(self.tile_off[-1], 1), dtype=torch.float64, device=dev)
        self.fuse_l1 = True          # step(): the L1 term inside the compositing adjoint
        self.image = torch.empty(3 * self.n_pixels, dtype=torch.float32, device=dev)
        self.final_T = torch.empty(self.n_pixels, dtype=torch.float32, device=dev)
        self.n_contrib = torch.empty(self.n_pixels, dtype=torch.int32, device=dev)
        self.dL_dimage = torch.empty(3 * self.n_pixels, dtype=torch.float32, device=dev)
        self.counters = torch.zeros(2, dtype=torch.int64, device=dev)
        self.adam_m = None
        self.adam_v = None
        self.adam_t = None           # device step counter of the Adam update
        self._photo = None           # (view table, workspace, bytes, own table) of the photometric loss
        self.reg_loss = None         # (L_scale, L_opacity) of the last regulariser call
        # eager forward: read the overflow flag after the chain and, after an overflow,
        # grow the instance buffers and render again (one synchronisation per forward).
        # Never done under graph capture, where check() after each replay does it.
        self.check_overflow = True
        self.generation = 0          # forwards run so far (PackUVRender ties a backward to its forward)

    # ------------------------------------------------------------------ helpers
    def close(self):
        for s in self.sets:
            s.close()
        if self._photo is not None and self._photo[3]:
            abi.pg_views_destroy(self._photo[0])
        self._photo = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def view_image(self, v):
        c = self.cams[v]
        o = 3 * self.pix_base[v]
        return self.image[o:o + 3 * c.width * c.height].view(3, c.height, c.width)

    def view_slice(self, buf, v, per_pixel=1):
        c = self.cams[v]
        o = per_pixel * self.pix_base[v]
        return buf[o:o + per_pixel * c.width * c.height]

    def _off(self, t, elems):
        return t.data_ptr() + elems * t.element_size()

    def status(self):
        """[(overflowed, instances needed)] of each view set's last sort, from
        pg_status_check (synchronises the current stream)."""
        return [abi.pg_status_check(s.overflow, s.n_inst) for s in self.sets]

    def check(self) -> bool:
        """True when no view set's last sort overflowed; call it after each
        replay of a captured step (an overflowed replay's outputs are undefined)."""
        return not any(ovf for ovf, _ in self.status())

    def grow_capacity(self, factor=1.25, headroom=False) -> bool:
        """Re-size the instance buffers from the last sort's counts: to
        ceil(need * factor) where it overflowed, or, with headroom=True,
        wherever need * factor exceeds the capacity (room for counts that grow,
        e.g. while Adam moves the Gaussians between replays).  Returns True
        when a buffer was re-allocated (a captured step must then be captured
        again)."""
        grew = False
        for s, (ovf, need) in zip(self.sets, self.status()):
            want = int(math.ceil(need * factor))
            if ovf or (headroom and want > s.cap):
                s.set_capacity(max(want, need, 1))
                grew = True
        return grew

    def ensure_capacity(self, headroom=1.25) -> bool:
        """After an overflow, grow to ceil(need * headroom); see grow_capacity."""
        return self.grow_capacity(headroom)

    def overflowed(self) -> bool:
        return not self.check()

    def plan(self, inst_capacity=None) -> dict:
        """pg_workspace_query for the batched view table: bytes of every buffer
        of one step (host only)."""
        s = self.sets[0]
        return abi.pg_workspace_query(s.handle, self.H, self.W, s.cap if inst_capacity is None else inst_capacity)

    # ------------------------------------------------------------------ stages
    def fetch(self, atlas: torch.Tensor):
        assert atlas.is_contiguous() and atlas.dtype == torch.float32
        assert atlas.numel() == self.frames * self.C * self.H * self.W
        abi.pg_atlas_fetch(atlas, self.occ, self.frames, self.C, self.H, self.W, self.N, self.gauss_texel,
                           self.texel_gauss, self.params, self.n_gauss_dev, self.fetch_ws, self.fetch_ws_bytes)
        if self.quant_bits is not None:
            # LPO: the rest of the step runs on the proxy; its texel gradient passes
            # straight through to the FP32 master atlas
            abi.pg_atlas_fake_quant(self.params, self.n_gauss_dev, self.N, self.frames, self.C, self.quant_bits,
                                    self.quant_range, None, self.quant_partial)

    def _order(self, s):
        return s.order if self.tile_order else None

    def _project_sort_render(self, s: _ViewSet, pix_off: int, counters):
        abi.pg_project(s.handle, self.params, s.splats, s.bins, s.tiles, self.visible)
        abi.pg_bin_sort(s.handle, s.bins, s.tiles, s.cap, s.keys, s.values, s.ranges, self._order(s), s.inst_first, s.n_inst, s.overflow,
                        s.ws, s.ws_bytes)
        if not self.batched and self.plain_sync:
            # plain path: one instance-count synchronisation per view
            ovf, need = abi.pg_status_check(s.overflow, s.n_inst)      # raises if a sort pass failed
            if ovf:
                s.set_capacity(int(math.ceil(need * 1.25)))
                abi.pg_bin_sort(s.handle, s.bins, s.tiles, s.cap, s.keys, s.values, s.ranges, self._order(s), s.inst_first, s.n_inst,
                                s.overflow, s.ws, s.ws_bytes)
        abi.pg_render_fwd(s.handle, s.splats, s.values, s.ranges, self._order(s), self.bg, self._off(self.image, 3 * pix_off),
                          self._off(self.final_T, pix_off), self._off(self.n_contrib, pix_off), s.tile_entries,
                          s.entries, counters)

    def _forward_chain(self, atlas, counters):
        self.fetch(atlas)
        self.visible.zero_()
        cnt = self.counters if counters else None
        if counters:
            self.counters.zero_()
        for k, s in enumerate(self.sets):
            self._project_sort_render(s, self.pix_base[k] if not self.batched else 0, cnt)

    def forward(self, atlas: torch.Tensor, counters: bool = False, check=None) -> torch.Tensor:
        """Render every view; returns the flat image buffer (valid until the next call).

        check (default: self.check_overflow) reads the overflow flag after the
        chain and, after an overflow, grows the instance buffers and renders
        again.  Under graph capture nothing is read: call check() after the
        replay."""
        self.generation += 1
        self._forward_chain(atlas, counters)
        # the plain path with per-view synchronisation has already grown every view's buffers
        checked = not self.batched and self.plain_sync
        if (self.check_overflow if check is None else check) and not checked \
                and not torch.cuda.is_current_stream_capturing():
            if self.ensure_capacity():
                self._forward_chain(atlas, counters)
                if not self.check():
                    raise RuntimeError("instance capacity overflowed again after growing to the reported count")
        return self.image

    def flow_mask(self, atlas: torch.Tensor, masks: torch.Tensor, counters=None):
        """Covariance-aware flow masking of the fetched Gaussians against per-view
        motion masks (uint8, the views' [H][W] masks concatenated like final_T):
        returns (dyn_gauss [F N], dyn_texel [H W]), both uint8; dyn_texel is the
        gradient-freezing mask the adjoint takes (set it as ``self.dynamic``)."""
        assert self.batched, "flow masking runs on the batched view table"
        assert masks.dtype == torch.uint8 and masks.numel() == self.n_pixels
        self.fetch(atlas)
        dg = torch.empty(max(self.frames * self.N, 1), dtype=torch.uint8, device=self.device)
        dt = torch.empty(self.H * self.W, dtype=torch.uint8, device=self.device)
        s = self.sets[0]
        tm = torch.empty(max(s.info.n_tiles, 1), dtype=torch.uint8, device=self.device)
        abi.pg_flow_mask(s.handle, self.params, masks, tm, dg, self.texel_gauss, self.H, self.W, dt, counters)
        return dg[:self.frames * self.N], dt

    def loss_photo(self, target: torch.Tensor, lambda_ssim: float) -> torch.Tensor:
        """(1 - lambda) L1 + lambda (1 - SSIM) over every view; fills dL_dimage."""
        if self._photo is None:
            h = self.sets[0].handle if self.batched else abi.pg_views_create(self.cams, self.frames, self.N,
                                                                            self.sh_degree, self.tiling)
            nb = abi.pg_photo_workspace_size(h)
            self._photo = (h, torch.empty(nb, dtype=torch.uint8, device=self.device), nb, not self.batched)
        h, ws, nb, _ = self._photo
        abi.pg_loss_photo(h, self.image, target, lambda_ssim, self.dL_dimage, self.loss, ws, nb)
        return self.loss

    def regularisers(self, s_max: float, w_scale: float = 1e-4, w_opacity: float = 1e-4, dyn_gauss=None):
        """Adds w_scale dL_scale + w_opacity dL_opacity to dL_datlas (after the
        adjoint); returns the device tensor (L_scale, L_opacity)."""
        if self.reg_loss is None:
            self.reg_loss = torch.zeros(2, dtype=torch.float32, device=self.device)
            self.reg_partial = torch.empty(3 * abi.REG_BLOCKS + 1, dtype=torch.float64, device=self.device)
        abi.pg_loss_regularisers(self.params, self.n_gauss_dev, self.N, self.frames, self.C, self.gauss_texel, self.H,
                                 self.W, dyn_gauss, s_max, w_scale, w_opacity, self.dL_datlas, self.reg_loss,
                                 self.reg_partial)
        return self.reg_loss

    def uv_prune(self, atlas: torch.Tensor, M: int, Nv: int, K: int, expected_uv=None):
        """UV-based pruning of the fetched Gaussians on an M x Nv UV map:
        returns (uv, rank, keep) as device tensors of shape [F N]."""
        self.fetch(atlas)
        n = self.frames * self.N
        uv = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        rank = torch.empty_like(uv)
        keep = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        nb = abi.pg_uv_prune_workspace_size(self.N, self.frames, M, Nv)
        ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        abi.pg_uv_prune(self.params, self.n_gauss_dev, self.N, self.frames, self.C, M, Nv, K, expected_uv, uv, rank,
                        keep, ws, nb)
        return uv[:n], rank[:n], keep[:n]

    def loss_l1(self, target: torch.Tensor) -> torch.Tensor:
        n = 3 * self.n_pixels
        abi.pg_loss_l1(self.image, target, n, self.dL_dimage, self.loss_partial, self.loss)
        return self.loss

    def backward(self, dL_dimage: torch.Tensor | None = None) -> torch.Tensor:
        """Texel gradients for the cotangent of the flat image (default: the L1 gradient)."""
        g = self.dL_dimage if dL_dimage is None else dL_dimage
        assert g.is_contiguous() and g.numel() == 3 * self.n_pixels
        if self.batched:
            s = self.sets[0]
            abi.pg_backward(s.handle, self.params, s.splats, s.bins, s.tiles, s.values, s.ranges, self._order(s),
                            s.inst_first, s.n_inst, s.cap, s.tile_entries, s.entries, self.n_contrib, self.bg,
                            self.final_T, g, s.inst_grad, self.gauss_texel, self.dynamic, self.H, self.W, s.grad2d,
                            self.dL_datlas, 0)
        else:
            self.dL_datlas.zero_()
            for k, s in enumerate(self.sets):
                po = self.pix_base[k]
                abi.pg_render_bwd(s.handle, s.splats, s.tiles, s.values, s.ranges, self._order(s), s.inst_first, s.n_inst, s.cap,
                                  s.tile_entries, s.entries, self._off(self.n_contrib, po), self.bg,
                                  self._off(self.final_T, po), self._off(g, 3 * po), s.inst_grad)
                abi.pg_project_bwd(s.handle, self.params, s.splats, s.bins, s.inst_first, s.n_inst, s.cap,
                                   s.inst_grad, self.gauss_texel, self.dynamic, self.H, self.W, s.grad2d,
                                   self.dL_datlas, 1)
        return self.dL_datlas

    def backward_l1(self, target: torch.Tensor) -> torch.Tensor:
        """The L1 loss and its texel gradients in one pass: the compositing adjoint
        forms the L1 cotangent from the image and target itself (pg_render_bwd_l1)
        and the loss value comes from its per-tile sums.  dL/datlas equals that of
        loss_l1() + backward() bit for bit; self.dL_dimage is not written."""
        assert target.is_contiguous() and target.numel() == 3 * self.n_pixels
        n = 3 * self.n_pixels
        if self.batched:
            s = self.sets[0]
            abi.pg_render_bwd_l1(s.handle, s.splats, s.tiles, s.values, s.ranges, self._order(s), s.inst_first,
                                 s.n_inst, s.cap, s.tile_entries, s.entries, self.n_contrib, self.bg, self.final_T,
                                 self.image, target, n, self.tile_loss, s.inst_grad)
            abi.pg_loss_l1_tiles(self.tile_loss, s.info.n_tiles, n, self.loss)
            abi.pg_project_bwd(s.handle, self.params, s.splats, s.bins, s.inst_first, s.n_inst, s.cap, s.inst_grad,
                               self.gauss_texel, self.dynamic, self.H, self.W, s.grad2d, self.dL_datlas, 0)
        else:
            self.dL_datlas.zero_()
            for k, s in enumerate(self.sets):
                po = self.pix_base[k]
                abi.pg_render_bwd_l1(s.handle, s.splats, s.tiles, s.values, s.ranges, self._order(s), s.inst_first,
                                     s.n_inst, s.cap, s.tile_entries, s.entries, self._off(self.n_contrib, po),
                                     self.bg, self._off(self.final_T, po), self._off(self.image, 3 * po),
                                     self._off(target, 3 * po), n, self._off(self.tile_loss, self.tile_off[k]),
                                     s.inst_grad)
                abi.pg_project_bwd(s.handle, self.params, s.splats, s.bins, s.inst_first, s.n_inst, s.cap,
                                   s.inst_grad, self.gauss_texel, self.dynamic, self.H, self.W, s.grad2d,
                                   self.dL_datlas, 1)
            abi.pg_loss_l1_tiles(self.tile_loss, self.tile_off[-1], n, self.loss)
        return self.loss

    def adam_step(self, atlas: torch.Tensor, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        """Sparse Adam on `atlas` in place; the step count lives on the device, so
        replays of a captured step keep counting."""
        if self.adam_m is None:
            self.adam_m = torch.zeros_like(atlas)
            self.adam_v = torch.zeros_like(atlas)
            self.adam_t = torch.zeros(1, dtype=torch.int32, device=self.device)
        abi.pg_adam_step(atlas, self.dL_datlas, self.adam_m, self.adam_v, self.visible, self.texel_gauss, self.N,
                         self.frames, self.C, self.H, self.W, lr, b1, b2, eps, 0, self.adam_t)

    def step(self, atlas, target, adam=False, lambda_ssim=None, reg=None):
        """One fitting step: forward, loss (L1, or the L1/SSIM blend when
        lambda_ssim is given), adjoint, the regularisers when reg (a dict of
        regularisers() arguments) is given, and Adam."""
        self.forward(atlas)
        if lambda_ssim is None and self.fuse_l1:
            self.backward_l1(target)
        else:
            if lambda_ssim is None:
                self.loss_l1(target)
            else:
                self.loss_photo(target, lambda_ssim)
            self.backward()
        if reg is not None:
            self.regularisers(**reg)
        if adam:
            self.adam_step(atlas)
        return self.loss

    # ------------------------------------------------------------------ readback helpers (tests)
    def splat_records(self, k=0):
        """numpy structured view of a view set's pg_splat records."""
        dt = np.dtype([("mean", "<f8", (2,)), ("conic", "<f4", (3,)), ("opacity", "<f4"), ("color", "<f4", (3,)),
                       ("depth", "<f4")])
        s = self.sets[k]
        return s.splats.cpu().numpy().view(np.uint8)[:s.info.n_gv * 48].view(dt)

    def bin_records(self, k=0):
        dt = np.dtype([("rect", "<i2", (4,)), ("key", "<u4"), ("n_tiles", "<i4")])
        s = self.sets[k]
        return s.bins.cpu().numpy().view(np.uint8)[:s.info.n_gv * 16].view(dt)

    def tile_sets(self, k=0):
        """numpy structured view of a view set's pg_tile_set records."""
        dt = np.dtype([("mask", "<u8"), ("x_lo", "<i2"), ("y_lo", "<i2"), ("width", "<u2"), ("height", "<u2")])
        s = self.sets[k]
        return s.tiles.cpu().numpy().view(np.uint8)[:s.info.n_gv * 16].view(dt)

    def sorted_instances(self, k=0):
        s = self.sets[k]
        n = int(s.n_inst[0].item())
        return s.keys[:n].cpu().numpy().view(np.uint32), s.values[:n].cpu().numpy()


class PackUVRender(torch.autograd.Function):
    """images = PackUVRender.apply(atlas, renderer): the flat image buffer of
    every view (view v's [3][H_v][W_v] image at offset 3 renderer.pix_base[v]).

    The backward runs the hand-written adjoint (pg_backward: transmittance
    recomputed from the stored final T, gradient freezing with the renderer's
    mask) and returns dL/datlas in the atlas's shape, and nothing for the
    renderer.

    The forward always checks the instance capacity (growing and rendering
    again after an overflow), so it never returns the undefined output of an
    overflowed sort; for that reason it cannot run under graph capture
    (capture Renderer.step instead and call Renderer.check() after each
    replay).  A renderer holds one step's buffers: the backward raises if the
    renderer has run another forward since this one."""

    @staticmethod
    def forward(ctx, atlas, renderer):
        if torch.cuda.is_current_stream_capturing():
            raise RuntimeError("PackUVRender cannot be captured: the instance capacity is only known after the "
                               "step has run; capture Renderer.step and call Renderer.check() after each replay")
        img = renderer.forward(atlas.detach().contiguous().reshape(-1), check=True)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.atlas_shape = atlas.shape
        return img.clone()

    @staticmethod
    def backward(ctx, grad):
        r = ctx.renderer
        if r.generation != ctx.generation:
            raise RuntimeError("PackUVRender: the renderer ran another forward after this one; its buffers hold "
                               "the later step, so this backward cannot be computed")
        return r.backward(grad.contiguous()).clone().view(ctx.atlas_shape), None
