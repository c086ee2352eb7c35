"""Torch-facing wrapper of libfdgs: device tensors in, device tensors out.

PyTorch only provides device memory and the stream; every computation runs
in the library's HIP kernels.  See include/fdgs.h for the semantics of each
call.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib

_HIP = None


def _hip():
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
    return _HIP


def _copy_device(dst: torch.Tensor, src_ptr: int, nbytes: int) -> None:
    if nbytes == 0:
        return
    rc = _hip().hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr), ctypes.c_size_t(nbytes), 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class GaussianModel:
    """4D Gaussians as float32 structure-of-arrays device tensors."""

    FIELDS = ("mean", "log_scale", "q_left", "q_right", "opacity_logit", "sh")

    def __init__(self, mean, log_scale, q_left, q_right, opacity_logit, sh, sh_degree: int = 3,
                 sh_index=None, sh_codebook=None):
        self.mean, self.log_scale = mean, log_scale
        self.q_left, self.q_right = q_left, q_right
        self.opacity_logit, self.sh = opacity_logit, sh
        self.sh_degree = int(sh_degree)
        n = mean.shape[1]
        shapes = {"mean": (4, n), "log_scale": (4, n), "q_left": (4, n), "q_right": (4, n),
                  "opacity_logit": (n,), "sh": (16, 3, n)}
        for k, shp in shapes.items():
            t = getattr(self, k)
            if tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{k}: need a contiguous float32 device tensor of shape {shp}")
        # optional vector-quantised SH: int32 index per Gaussian into a [K, 48] float32 codebook
        self.sh_index, self.sh_codebook = sh_index, sh_codebook
        if (sh_index is None) != (sh_codebook is None):
            raise ValueError("sh_index and sh_codebook go together")
        if sh_index is not None:
            if tuple(sh_index.shape) != (n,) or sh_index.dtype != torch.int32 or not sh_index.is_cuda:
                raise ValueError("sh_index: need an int32 device tensor of shape (n,)")
            if (sh_codebook.dim() != 2 or sh_codebook.shape[1] != 48 or sh_codebook.dtype != torch.float32
                    or not sh_codebook.is_contiguous() or not sh_codebook.is_cuda):
                raise ValueError("sh_codebook: need a contiguous float32 device tensor of shape (K, 48)")

    def quantized(self, sh_index, sh_codebook) -> "GaussianModel":
        """The same Gaussians with SH read from a codebook."""
        return GaussianModel(self.mean, self.log_scale, self.q_left, self.q_right, self.opacity_logit, self.sh,
                             self.sh_degree, sh_index, sh_codebook)

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @classmethod
    def from_scene(cls, scene, device="cuda"):
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return cls(t(scene.mean), t(scene.log_scale), t(scene.q_left), t(scene.q_right),
                   t(scene.opacity_logit), t(scene.sh), scene.sh_degree)

    def struct(self) -> _lib.Model:
        m = _lib.Model()
        for k in self.FIELDS:
            setattr(m, k, getattr(self, k).data_ptr())
        m.n = self.n
        m.sh_degree = self.sh_degree
        if self.sh_index is not None:
            m.sh_index = self.sh_index.data_ptr()
            m.sh_codebook = self.sh_codebook.data_ptr()
            m.sh_codebook_size = int(self.sh_codebook.shape[0])
        return m

    def tensors(self):
        return [getattr(self, k) for k in self.FIELDS]


class State:
    """Handle of a forward pass kept for the adjoint or for inspection."""

    def __init__(self, ctx: "Context", handle: ctypes.c_void_p, shape):
        self.ctx, self.handle, self.shape = ctx, handle, shape

    def release(self):
        if self.handle is not None and self.handle.value:
            self.ctx.release(self)


class Context:
    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        self.device = torch.device("cuda", device)
        self.handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.fdgs_create(ctypes.byref(self.handle), device))

    def close(self):
        if self.handle.value:
            torch.cuda.synchronize(self.device)
            _lib.check(self.lib.fdgs_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # (1) ------------------------------------------------------------------
    def slice_4d(self, model: GaussianModel, t: float, idx: Optional[torch.Tensor] = None):
        m = model.n if idx is None else int(idx.numel())
        dev = self.device
        mean3 = torch.empty((3, m), dtype=torch.float32, device=dev)
        cov3 = torch.empty((6, m), dtype=torch.float32, device=dev)
        p = torch.empty((m,), dtype=torch.float32, device=dev)
        ms = model.struct()
        _lib.check(self.lib.fdgs_slice_4d(self.handle, ctypes.byref(ms), float(t), _ptr(idx), m,
                                          _ptr(mean3), _ptr(cov3), _ptr(p), _stream(dev)))
        return mean3, cov3, p

    # (2) ------------------------------------------------------------------
    def build_active_mask(self, model: GaussianModel, frame_times, key_lo: float, key_hi: float,
                          mode: int = _lib.MASK_TEMPORAL, views=(), alpha_min: float = 0.0,
                          dilation: float = -1.0):
        n = model.n
        dev = self.device
        bits = torch.empty(((n + 31) // 32,), dtype=torch.int32, device=dev)
        idx = torch.empty((max(n, 1),), dtype=torch.int32, device=dev)
        count = torch.zeros((1,), dtype=torch.int64, device=dev)
        ft = np.ascontiguousarray(np.asarray(frame_times, dtype=np.float64))
        cams = (_lib.Camera * max(len(views), 1))(*[_lib.camera_struct(v) for v in views])
        spec = _lib.MaskSpec()
        spec.frame_times = ft.ctypes.data
        spec.n_frames = ft.size
        spec.views = ctypes.cast(cams, ctypes.c_void_p)
        spec.n_views = len(views)
        spec.key_lo, spec.key_hi = float(key_lo), float(key_hi)
        spec.mode = int(mode)
        spec.alpha_min = float(alpha_min)
        spec.dilation = float(dilation)
        ms = model.struct()
        _lib.check(self.lib.fdgs_build_active_mask(self.handle, ctypes.byref(ms), ctypes.byref(spec),
                                                   _ptr(bits), _ptr(idx), _ptr(count), _stream(dev)))
        return bits, idx, count

    def measure_peaks(self) -> dict:
        """Measured LDS and vector-ALU rates of the device (see fdgs_measure_peaks)."""
        out = (ctypes.c_double * 4)()
        _lib.check(self.lib.fdgs_measure_peaks(self.handle, out, _stream(self.device)))
        return {"lds_broadcast_Bps": out[0], "lds_distinct_Bps": out[1], "valu_fma_lane_ops_per_s": out[2],
                "compute_units": int(out[3])}

    def mask_overlap(self, bits_a: torch.Tensor, bits_b: torch.Tensor, n: int) -> torch.Tensor:
        """Device int64[3]: |a|, |b| and |a and b| over the first n bits."""
        out = torch.empty((3,), dtype=torch.int64, device=bits_a.device)
        _lib.check(self.lib.fdgs_mask_overlap(_ptr(bits_a), _ptr(bits_b), int(n), _ptr(out), _stream(bits_a.device)))
        return out

    # (3) ------------------------------------------------------------------
    def render(self, model: GaussianModel, cam, t: float, cfg: Optional[_lib.RenderCfg] = None,
               idx: Optional[torch.Tensor] = None, n_idx: Optional[torch.Tensor] = None,
               want_T: bool = False, keep_state=False, out_rgb: Optional[torch.Tensor] = None):
        """keep_state: False, True (new state) or an existing State to reuse."""
        cfg = cfg if cfg is not None else _lib.default_cfg()
        cs = _lib.camera_struct(cam)
        dev = self.device
        H, W = cs.height, cs.width
        rgb = out_rgb if out_rgb is not None else torch.empty((3, H, W), dtype=torch.float32, device=dev)
        T = torch.empty((H, W), dtype=torch.float32, device=dev) if want_T else None
        ms = model.struct()
        st_ptr = None
        handle = None
        if keep_state is not False and keep_state is not None:
            handle = keep_state.handle if isinstance(keep_state, State) else ctypes.c_void_p()
            st_ptr = ctypes.byref(handle)
        _lib.check(self.lib.fdgs_render_forward(self.handle, ctypes.byref(ms), _ptr(idx), _ptr(n_idx),
                                                ctypes.byref(cs), float(t), ctypes.byref(cfg), _ptr(rgb),
                                                _ptr(T), st_ptr, _stream(dev)))
        state = None
        if handle is not None:
            state = keep_state if isinstance(keep_state, State) else State(self, handle, (H, W))
        return rgb, T, state

    # (4) ------------------------------------------------------------------
    def backward(self, state: State, dL_drgb: torch.Tensor, model: GaussianModel, grads=None):
        if grads is None:
            grads = {k: torch.zeros_like(getattr(model, k)) for k in GaussianModel.FIELDS}
        g = _lib.Grads()
        for k in GaussianModel.FIELDS:
            setattr(g, k, grads[k].data_ptr())
        dL = dL_drgb.contiguous()
        _lib.check(self.lib.fdgs_render_backward(self.handle, state.handle, _ptr(dL), ctypes.byref(g),
                                                 _stream(self.device)))
        return grads

    def backward_2d(self, state: State, dL_drgb: torch.Tensor):
        """First phase of the adjoint (the blend), into the state's own 2D gradients."""
        dL = dL_drgb.contiguous()
        _lib.check(self.lib.fdgs_render_backward_2d(self.handle, state.handle, _ptr(dL), _stream(self.device)))

    def backward_params(self, state: State, model: GaussianModel, grads=None):
        """Second phase: the state's 2D gradients added into the model's gradients."""
        if grads is None:
            grads = {k: torch.zeros_like(getattr(model, k)) for k in GaussianModel.FIELDS}
        g = _lib.Grads()
        for k in GaussianModel.FIELDS:
            setattr(g, k, grads[k].data_ptr())
        _lib.check(self.lib.fdgs_render_backward_params(self.handle, state.handle, ctypes.byref(g),
                                                        _stream(self.device)))
        return grads

    def release(self, state: State):
        _lib.check(self.lib.fdgs_state_release(self.handle, state.handle))
        state.handle = ctypes.c_void_p()

    def binning(self, state: State) -> dict:
        b = _lib.Binning()
        _lib.check(self.lib.fdgs_state_binning(self.handle, state.handle, ctypes.byref(b), _stream(self.device)))
        dev = self.device
        out = {
            "sorted_ids": torch.empty((b.n_inst,), dtype=torch.int32, device=dev),
            "tile_ranges": torch.empty((b.n_tiles, 2), dtype=torch.int32, device=dev),
            "rects": torch.empty((b.n_proc, 4), dtype=torch.int32, device=dev),
            "depth": torch.empty((b.n_proc,), dtype=torch.float64, device=dev),
            "visible": torch.empty((b.n_proc,), dtype=torch.uint8, device=dev),
        }
        _copy_device(out["sorted_ids"], b.sorted_ids, 4 * b.n_inst)
        _copy_device(out["tile_ranges"], b.tile_ranges, 8 * b.n_tiles)
        _copy_device(out["rects"], b.rects, 16 * b.n_proc)
        _copy_device(out["depth"], b.depth, 8 * b.n_proc)
        _copy_device(out["visible"], b.visible, b.n_proc)
        out.update(n_inst=b.n_inst, n_vis=b.n_vis, n_proc=b.n_proc, n_tiles=b.n_tiles,
                   tiles_x=b.tiles_x, tiles_y=b.tiles_y)
        return out

    # (5) ------------------------------------------------------------------
    @staticmethod
    def _batch_structs(scenes, views):
        ms = (_lib.Model * len(scenes))(*[m.struct() for m in scenes])
        vs = (_lib.View * len(views))()
        for k, v in enumerate(views):
            scene, cam, t = v[0], v[1], v[2]
            idx = v[3] if len(v) > 3 else None
            n_idx = v[4] if len(v) > 4 else (int(idx.numel()) if idx is not None else 0)
            vs[k].scene = int(scene)
            vs[k].cam = _lib.camera_struct(cam)
            vs[k].t = float(t)
            vs[k].idx = idx.data_ptr() if idx is not None else None
            vs[k].n_idx = int(n_idx)
        return ms, vs

    def render_batch(self, scenes, views, cfg: Optional[_lib.RenderCfg] = None, views_per_launch: int = 0,
                     use_graph: bool = False, out: Optional[torch.Tensor] = None):
        """views: sequence of (scene index, camera, t[, idx tensor[, n_idx]]).  Returns [V, 3, H, W]."""
        cfg = cfg if cfg is not None else _lib.default_cfg()
        ms, vs = self._batch_structs(scenes, views)
        H, W = vs[0].cam.height, vs[0].cam.width
        if out is None:
            out = torch.empty((len(views), 3, H, W), dtype=torch.float32, device=self.device)
        _lib.check(self.lib.fdgs_render_batch(self.handle, ms, len(scenes), vs, len(views), ctypes.byref(cfg),
                                              int(views_per_launch), 1 if use_graph else 0, _ptr(out),
                                              _stream(self.device)))
        self._keep = (ms, vs)
        return out

    def autotune(self, scenes, views, cfg: Optional[_lib.RenderCfg] = None, views_per_launch: int = 0,
                 repeats: int = 3):
        """Returns (best cfg, list of per-configuration results)."""
        cfg = _lib.default_cfg() if cfg is None else cfg
        best = _lib.RenderCfg()
        ctypes.memmove(ctypes.byref(best), ctypes.byref(cfg), ctypes.sizeof(cfg))
        ms, vs = self._batch_structs(scenes, views)
        res = (_lib.TuneResult * 128)()
        n = ctypes.c_int32()
        status = self.lib.fdgs_autotune(self.handle, ms, len(scenes), vs, len(views), int(views_per_launch),
                                        int(repeats), ctypes.byref(best), res, 128, ctypes.byref(n),
                                        _stream(self.device))
        out = [dict(tile=(r.tile_w, r.tile_h), batch=r.batch, pixels_per_thread=r.pixels_per_thread,
                    schedule=r.schedule, ms=r.ms, identical=bool(r.identical)) for r in res[: n.value]]
        _lib.check(status)
        return best, out

    # (7) pruning score ----------------------------------------------------
    def spatial_score(self, model: GaussianModel, views, cfg: Optional[_lib.RenderCfg] = None,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """views: sequence of (camera, t).  Adds Eq. 4's per-Gaussian sums to `out`
        (zeros if None) and returns it."""
        score = out if out is not None else torch.zeros((model.n,), dtype=torch.float32, device=self.device)
        cams = (_lib.Camera * max(len(views), 1))(*[_lib.camera_struct(v[0]) for v in views])
        ts = np.ascontiguousarray(np.asarray([float(v[1]) for v in views], dtype=np.float64))
        ms = model.struct()
        _lib.check(self.lib.fdgs_spatial_score(self.handle, ctypes.byref(ms), cams, ts.ctypes.data_as(ctypes.c_void_p),
                                               len(views), ctypes.byref(cfg) if cfg is not None else None,
                                               _ptr(score), _stream(self.device)))
        return score

    def variation_score(self, model: GaussianModel, times, spatial: torch.Tensor) -> torch.Tensor:
        out = torch.empty((model.n,), dtype=torch.float32, device=self.device)
        ts = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        ms = model.struct()
        _lib.check(self.lib.fdgs_variation_score(self.handle, ctypes.byref(ms), ts.ctypes.data_as(ctypes.c_void_p),
                                                 ts.size, _ptr(spatial.contiguous()), _ptr(out),
                                                 _stream(self.device)))
        return out

    def prune(self, score: torch.Tensor, n_keep: int):
        n = int(score.numel())
        bits = torch.empty(((n + 31) // 32 or 1,), dtype=torch.int32, device=self.device)
        idx = torch.empty((max(n, 1),), dtype=torch.int32, device=self.device)
        count = torch.zeros((1,), dtype=torch.int64, device=self.device)
        _lib.check(self.lib.fdgs_prune(self.handle, _ptr(score.contiguous()), ctypes.c_int64(n),
                                       ctypes.c_int64(int(n_keep)), _ptr(bits), _ptr(idx), _ptr(count),
                                       _stream(self.device)))
        return bits, idx, count

    def sh_kmeans(self, model: GaussianModel, k: int, iterations: int, init_index: Optional[torch.Tensor] = None,
                  seed: int = 0):
        """Vector quantisation of the SH vectors: (codebook [k, 48], assignment [n] int32).  The
        initial codebook is the vectors of init_index (default: k distinct Gaussians drawn with
        `seed`)."""
        n = model.n
        if init_index is None:
            rng = np.random.default_rng(seed)
            init_index = torch.from_numpy(rng.choice(n, size=k, replace=k > n).astype(np.int32)).to(self.device)
        code = torch.empty((k, 48), dtype=torch.float32, device=self.device)
        assign = torch.empty((max(n, 1),), dtype=torch.int32, device=self.device)
        ms = model.struct()
        _lib.check(self.lib.fdgs_sh_kmeans(self.handle, ctypes.byref(ms), _ptr(init_index.contiguous()),
                                           ctypes.c_int64(k), int(iterations), _ptr(code), _ptr(assign),
                                           _stream(self.device)))
        return code, assign[:n]

    def check_overflow(self):
        _lib.check(self.lib.fdgs_check_overflow(self.handle, _stream(self.device)))

    def profile(self, enable, count_pairs: bool = False):
        level = 0 if not enable else (2 if count_pairs else 1)
        _lib.check(self.lib.fdgs_profile_enable(self.handle, level))

    def profile_read(self, reset: bool = True) -> dict:
        p = _lib.Profile()
        _lib.check(self.lib.fdgs_profile_read(self.handle, ctypes.byref(p), 1 if reset else 0))
        return {"ms": {name: p.ms[k] for k, name in enumerate(_lib.STAGES)},
                "calls": {name: p.calls[k] for k, name in enumerate(_lib.STAGES)},
                "processed": p.processed, "visible": p.visible, "instances": p.instances, "pairs": p.pairs,
                "blended": p.blended}


def _own_stream(ctx: Context) -> "torch.cuda.Stream":
    """A stream of the context's own (default priority), created on first use."""
    s = getattr(ctx, "_own_stream", None)
    if s is None:
        s = torch.cuda.Stream(ctx.device)
        ctx._own_stream = s
    return s


def forward_backward_views(ctxs, model: GaussianModel, views, cfg: Optional[_lib.RenderCfg], loss_grad, grads,
                           states=None):
    """Forward pass and adjoint of several views, adding the gradients of
    sum_v L_v into `grads` (caller-zeroed tensors in the model's layout).

    views: (cam, t, idx, n_idx) per view (idx, n_idx may be None: dense).
    loss_grad(v, rgb) returns dL_v/drgb for view v's image.  View v is rendered
    and differentiated by ctxs[v % len(ctxs)] on a stream of that context's
    own, so a view's forward (short launches that fill the device poorly) and
    the blend adjoint (into the view's own state) run beside other views'
    work.  Only the adjoints' second phase, which adds into `grads`, is chained
    in view order by events, so the gradients are added in the same order as
    in a loop over the views on one stream.  states: States to
    reuse (one per view, each owned by the context that renders its view) or
    None; the list of states is returned.  The work starts after everything
    queued on the caller's current stream, and that stream waits for the last
    adjoint before this returns."""
    dev = ctxs[0].device
    cur = torch.cuda.current_stream(dev)
    begin = torch.cuda.Event()
    begin.record(cur)
    streams = [_own_stream(c) for c in ctxs]
    for s in streams:
        s.wait_event(begin)
    states = list(states) if states is not None else [None] * len(views)
    if len(states) != len(views):
        raise ValueError("forward_backward_views: one state per view")
    prev = None
    for v, (cam, t, idx, n_idx) in enumerate(views):
        c, s = ctxs[v % len(ctxs)], streams[v % len(ctxs)]
        st = states[v]
        if st is not None and st.ctx is not c:
            raise ValueError(f"forward_backward_views: state of view {v} belongs to another context")
        with torch.cuda.stream(s):
            rgb, _, st = c.render(model, cam, t, cfg, idx=idx, n_idx=n_idx, keep_state=st if st is not None else True)
            states[v] = st
            c.backward_2d(st, loss_grad(v, rgb))
            if prev is not None:
                s.wait_event(prev)
            c.backward_params(st, model, grads)
            prev = torch.cuda.Event()
            prev.record(s)
    if prev is not None:
        cur.wait_event(prev)
    return states


class Render4DGS(torch.autograd.Function):
    """rgb = Render4DGS.apply(context, cam, t, cfg, idx, n_idx, mean, log_scale, q_left, q_right,
    opacity_logit, sh).  The backward runs the library's adjoint kernels."""

    @staticmethod
    def forward(ctx, context: Context, cam, t, cfg, idx, n_idx, mean, log_scale, q_left, q_right,
                opacity_logit, sh):
        model = GaussianModel(mean.detach(), log_scale.detach(), q_left.detach(), q_right.detach(),
                              opacity_logit.detach(), sh.detach())
        rgb, _, state = context.render(model, cam, t, cfg, idx=idx, n_idx=n_idx, keep_state=True)
        ctx.context, ctx.state, ctx.model = context, state, model
        return rgb

    @staticmethod
    def backward(ctx, dL_drgb):
        grads = ctx.context.backward(ctx.state, dL_drgb, ctx.model)
        ctx.context.release(ctx.state)
        g = [grads[k] for k in GaussianModel.FIELDS]
        return (None, None, None, None, None, None, *g)
