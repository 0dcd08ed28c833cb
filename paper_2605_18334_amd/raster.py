"""Python surface of the MI355X skew-Gaussian rasterizer.

Thin layer over the C ABI (include/sgs.h): PyTorch provides device memory and
the stream; every computation step runs in the HIP library.

    gs   = GaussianSet.from_scene(scene)              # device SoA parameters
    cams = CameraBatch.from_poses([pose], opt)        # CoordEngine + layout
    fr   = render(gs, cams)                           # preprocess, bin/sort, blend
    img  = fr.image(0)                                # [3, H, W]
    g    = render_backward(fr, dL_drgb)               # gradients of all parameters
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi
from ._abi import check, load

DEV = "cuda"


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


@dataclass
class GaussianSet:
    """Gaussian parameters as float32 structure-of-arrays device tensors."""
    mean: torch.Tensor                 # [3, N]
    log_scale: torch.Tensor            # [3, N]
    quat: torch.Tensor                 # [4, N] (w, x, y, z)
    skew: torch.Tensor | None          # [3, N] or None (symmetric)
    opa_logit: torch.Tensor            # [N]
    sh: torch.Tensor                   # [K, 3, N]
    sh_degree: int
    opa2_logit: torch.Tensor | None = None
    opa_dir: torch.Tensor | None = None

    FIELDS = ("mean", "log_scale", "quat", "skew", "opa_logit", "opa2_logit", "opa_dir", "sh")

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @property
    def enhanced(self) -> bool:
        return self.opa2_logit is not None

    @classmethod
    def from_scene(cls, sc, device=DEV) -> "GaussianSet":
        t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return cls(t(sc.mean), t(sc.log_scale), t(sc.quat), t(sc.skew), t(sc.opa_logit),
                   t(sc.sh), int(sc.sh_degree), t(sc.opa2_logit), t(sc.opa_dir))

    def struct(self) -> _abi.Params:
        p = _abi.Params()
        p.n = self.n
        p.sh_degree = self.sh_degree
        for f in self.FIELDS:
            v = getattr(self, f)
            if v is not None:
                assert v.dtype == torch.float32 and v.is_contiguous() and v.is_cuda, f
            setattr(p, f, _ptr(v))
        return p


class CameraBatch:
    """n_views cameras laid out in one global tile/pixel space, kept both in
    host memory (ctypes array) and as an identical device copy."""

    def __init__(self, cams: list, opt: _abi.Options, device=DEV):
        lib = load()
        n = len(cams)
        self.host = (_abi.Camera * n)(*cams)
        tt, tp = C.c_int64(), C.c_int64()
        check("sgs_camera_layout", lib.sgs_camera_layout(self.host, n, C.byref(opt), C.byref(tt), C.byref(tp)))
        self.n_views = n
        self.total_tiles = int(tt.value)
        self.total_pixels = int(tp.value)
        self.tile_w, self.tile_h = opt.tile_w, opt.tile_h
        raw = bytes(memoryview(self.host).cast("B"))
        self.dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)

    @staticmethod
    def camera_from_pose(pose) -> _abi.Camera:
        """CoordEngine + intrinsic mapping in the library (sgs_camera_from_gl)."""
        lib = load()
        cam = _abi.Camera()
        m = (C.c_double * 16)(*np.asarray(pose.c2w_gl, np.float64).reshape(-1).tolist())
        bg = (C.c_float * 3)(*[float(x) for x in pose.bg])
        check("sgs_camera_from_gl", lib.sgs_camera_from_gl(
            m, int(pose.width), int(pose.height), math.radians(pose.fovx_deg), 0.0,
            float(pose.near), bg, C.byref(cam)))
        return cam

    @classmethod
    def from_poses(cls, poses, opt: _abi.Options | None = None, device=DEV) -> "CameraBatch":
        opt = opt if opt is not None else _abi.default_options()
        return cls([cls.camera_from_pose(p) for p in poses], opt, device)

    def view(self, v: int) -> _abi.Camera:
        return self.host[v]

    def upload(self) -> None:
        """Re-copies the host array into the existing device buffer (poses
        changed in place, layout unchanged)."""
        raw = bytes(memoryview(self.host).cast("B"))
        self.dev.copy_(torch.frombuffer(bytearray(raw), dtype=torch.uint8))


@dataclass
class Frame:
    """Everything one forward render produced (kept for the backward)."""
    gs: GaussianSet
    cams: CameraBatch
    opt: _abi.Options
    geom: _abi.Geom
    bufs: dict
    n_inst: int
    out_rgb: torch.Tensor        # [3, P]
    out_T: torch.Tensor          # [P]
    out_last: torch.Tensor       # [P] (int32 storage of u32)

    @property
    def m(self) -> int:
        return self.gs.n * self.cams.n_views

    def image(self, v: int = 0) -> torch.Tensor:
        c = self.cams.view(v)
        s = c.pix_base
        return self.out_rgb[:, s:s + c.width * c.height].reshape(3, c.height, c.width)

    def transmittance(self, v: int = 0) -> torch.Tensor:
        c = self.cams.view(v)
        s = c.pix_base
        return self.out_T[s:s + c.width * c.height].reshape(c.height, c.width)


def alloc_geom(m: int, n: int, n_views: int, enhanced: bool, device=DEV) -> tuple[_abi.Geom, dict]:
    lib = load()
    b = {
        "rec": torch.empty(int(lib.sgs_geom_rec_floats(m, int(enhanced))), dtype=torch.float32, device=device),
        "depth": torch.empty(max(m, 1), dtype=torch.float32, device=device),
        "rect": torch.empty(max(2 * m, 2), dtype=torch.int32, device=device),
        "tiles": torch.empty(max(m, 1), dtype=torch.int32, device=device),
        "block_off": torch.empty(int(lib.sgs_geom_block_entries(n, n_views)), dtype=torch.int32, device=device),
        "rows": torch.empty(max(m, 1), dtype=torch.int32, device=device),
    }
    g = _abi.Geom(_ptr(b["rec"]), _ptr(b["depth"]), _ptr(b["rect"]), _ptr(b["tiles"]), _ptr(b["block_off"]),
                  _ptr(b["rows"]), int(enhanced), 0)
    return g, b


def preprocess(gs: GaussianSet, cams: CameraBatch, opt: _abi.Options, stream=None):
    lib = load()
    m = gs.n * cams.n_views
    geom, bufs = alloc_geom(m, gs.n, cams.n_views, gs.enhanced)
    p = gs.struct()
    check("sgs_preprocess", lib.sgs_preprocess(C.byref(p), cams.host, _ptr(cams.dev), cams.n_views,
                                               C.byref(opt), C.byref(geom), _stream(stream)))
    return geom, bufs


def bin_sort(geom, bufs, m: int, cams: CameraBatch, opt: _abi.Options, capacity: int,
             keep_keys: bool = False, stream=None) -> dict:
    lib = load()
    dev = bufs["depth"].device
    out = {
        "vals": torch.empty(max(capacity, 1), dtype=torch.int32, device=dev),
        "ranges": torch.empty(2 * cams.total_tiles, dtype=torch.int32, device=dev),
        "n_inst": torch.zeros(1, dtype=torch.int32, device=dev),
        "keys": torch.empty(max(capacity, 1), dtype=torch.int64, device=dev) if (keep_keys or opt.sort_mode == 0) else None,
    }
    sb = int(lib.sgs_bin_sort_scratch_bytes(m, capacity, cams.total_tiles, C.byref(opt)))
    out["scratch"] = torch.empty(sb, dtype=torch.uint8, device=dev)
    check("sgs_bin_sort", lib.sgs_bin_sort(
        C.byref(geom), m, cams.host, _ptr(cams.dev), cams.n_views, C.byref(opt), capacity,
        _ptr(out["keys"]), _ptr(out["vals"]), _ptr(out["ranges"]), _ptr(out["n_inst"]), None,
        _ptr(out["scratch"]), sb, _stream(stream)))
    return out


N_INVALID = 0xFFFFFFFF     # instance count after a sort look-back that did not complete


def check_instance_count(n: int, capacity: int, fn: str = "sgs_bin_sort") -> None:
    """Raises SgsError when the device instance count reports a failed sort
    (0xffffffff) or more instances than the buffers hold."""
    n &= 0xFFFFFFFF
    if n == N_INVALID:
        raise _abi.SgsError(f"{fn}: a sort look-back did not complete; outputs invalid", 3)
    if n > capacity:
        raise _abi.SgsError(f"{fn}: {n} instances exceed the capacity {capacity}", 2)


def render(gs: GaussianSet, cams: CameraBatch, opt: _abi.Options | None = None,
           keep_keys: bool = False, capacity: int | None = None, stream=None,
           count: bool = False, check_count: bool = True) -> Frame:
    """Forward render of all views.  Without ``capacity`` the instance count
    is read back after the preprocess (one 4-byte device-to-host copy) and
    buffers are sized exactly.  With ``check_count`` the sort's instance
    count is read back after the blend (a second host sync) and a failed or
    overflowed sort raises instead of returning its image."""
    lib = load()
    opt = opt if opt is not None else _abi.default_options()
    m = gs.n * cams.n_views
    geom, bufs = preprocess(gs, cams, opt, stream)
    if capacity is None:
        capacity = int(bufs["block_off"][-1].item()) & 0xFFFFFFFF
        if capacity == 0xFFFFFFFF:
            raise _abi.SgsError("sgs_preprocess: instance count exceeds 2^32-1", 2)
    bs = bin_sort(geom, bufs, m, cams, opt, capacity, keep_keys, stream)
    bufs.update(bs)
    dev = bufs["depth"].device
    P = cams.total_pixels
    out_rgb = torch.empty((3, P), dtype=torch.float32, device=dev)
    out_T = torch.empty(P, dtype=torch.float32, device=dev)
    out_last = torch.empty(P, dtype=torch.int32, device=dev)
    bufs["count"] = torch.empty(P, dtype=torch.int32, device=dev) if count else None
    bufs["eval"] = torch.empty(P, dtype=torch.int32, device=dev) if count else None
    check("sgs_render_fwd", lib.sgs_render_fwd(
        C.byref(geom), m, _ptr(bufs["vals"]), capacity, _ptr(bufs["ranges"]), None, cams.host, _ptr(cams.dev),
        cams.n_views, int(gs.enhanced), C.byref(opt), _ptr(out_rgb), _ptr(out_T), _ptr(out_last),
        _ptr(bufs["count"]), _ptr(bufs["eval"]), P, _stream(stream)))
    if check_count:
        check_instance_count(int(bufs["n_inst"].item()), capacity)
    return Frame(gs, cams, opt, geom, bufs, capacity, out_rgb, out_T, out_last)


def densify_stats(gs: "GaussianSet") -> dict:
    """Zeroed accumulators of the densification statistics (Sec. "Depth-Aware
    Densification Strategy"): ``uv`` sums the NDC screen-space gradient norm
    over the views that see a Gaussian, ``z`` keeps the largest |dL/d depth|
    of its centre, ``count`` counts the views; pass to a backward, which
    accumulates into them."""
    dev = gs.mean.device
    return {"uv": torch.zeros(gs.n, dtype=torch.float32, device=dev),
            "z": torch.zeros(gs.n, dtype=torch.float32, device=dev),
            "count": torch.zeros(gs.n, dtype=torch.int32, device=dev)}


def _params_grad(grads: dict, densify: dict | None) -> "_abi.ParamsGrad":
    d = densify or {}
    return _abi.ParamsGrad(*[_ptr(grads[f]) for f in GaussianSet.FIELDS],
                           _ptr(d.get("uv")), _ptr(d.get("z")), _ptr(d.get("count")))


def render_backward(fr: Frame, dL_drgb: torch.Tensor, stream=None, densify: dict | None = None) -> dict:
    """Gradients of the loss w.r.t. every Gaussian parameter, given dL/dC in
    the layout of Frame.out_rgb ([3, P]); with ``densify`` (from
    densify_stats) the densification statistics are accumulated too."""
    lib = load()
    gs = fr.gs
    dL = dL_drgb.contiguous().float()
    assert dL.shape == fr.out_rgb.shape
    g2d = torch.zeros(int(lib.sgs_geom_rec_floats(fr.m, int(gs.enhanced))), dtype=torch.float32,
                      device=dL.device)
    grads = {f: (None if getattr(gs, f) is None else torch.zeros_like(getattr(gs, f)))
             for f in GaussianSet.FIELDS}
    pg = _params_grad(grads, densify)
    gg = _abi.GeomGrad(_ptr(g2d))
    p = gs.struct()
    check("sgs_render_bwd", lib.sgs_render_bwd(
        C.byref(p), C.byref(fr.geom), fr.m, _ptr(fr.bufs["vals"]), fr.n_inst, _ptr(fr.bufs["ranges"]),
        None, fr.cams.host, _ptr(fr.cams.dev), fr.cams.n_views, C.byref(fr.opt), _ptr(fr.out_T),
        _ptr(fr.out_last), _ptr(dL), fr.cams.total_pixels, C.byref(gg), C.byref(pg),
        _stream(stream)))
    grads["g2d"] = g2d
    return grads


class SkewGaussianRasterizer(torch.autograd.Function):
    """Differentiable render of one or more views: the forward returns the
    [3, P] colour planes; the backward runs the library's hand-written
    adjoint (no per-pair state is stored; T is rebuilt from the final T)."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, skew, opa_logit, sh, opa2_logit, opa_dir, cams, opt, sh_degree):
        gs = GaussianSet(mean.detach().contiguous(), log_scale.detach().contiguous(),
                         quat.detach().contiguous(), None if skew is None else skew.detach().contiguous(),
                         opa_logit.detach().contiguous(), sh.detach().contiguous(), int(sh_degree),
                         None if opa2_logit is None else opa2_logit.detach().contiguous(),
                         None if opa_dir is None else opa_dir.detach().contiguous())
        fr = render(gs, cams, opt)
        ctx.frame = fr
        ctx.has = [t is not None for t in (skew, opa2_logit, opa_dir)]
        return fr.out_rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        g = render_backward(ctx.frame, grad_rgb)
        ctx.frame = None
        return (g["mean"], g["log_scale"], g["quat"], g["skew"], g["opa_logit"], g["sh"],
                g["opa2_logit"], g["opa_dir"], None, None, None)


def rasterize(mean, log_scale, quat, skew, opa_logit, sh, cams: CameraBatch, opt=None,
              sh_degree: int | None = None, opa2_logit=None, opa_dir=None) -> torch.Tensor:
    """Autograd entry point: returns the [3, P] colour planes of all views."""
    opt = opt if opt is not None else _abi.default_options()
    if sh_degree is None:
        sh_degree = int(round(math.sqrt(sh.shape[0]))) - 1
    return SkewGaussianRasterizer.apply(mean, log_scale, quat, skew, opa_logit, sh, opa2_logit,
                                        opa_dir, cams, opt, sh_degree)


def layout_totals(poses, opt: _abi.Options | None = None) -> tuple[int, int]:
    """(total tiles, total pixels) of a batch of poses laid out in one tile
    space, computed on the host (no device memory)."""
    lib = load()
    opt = opt if opt is not None else _abi.default_options()
    arr = (_abi.Camera * len(poses))(*[CameraBatch.camera_from_pose(p) for p in poses])
    tt, tp = C.c_int64(), C.c_int64()
    check("sgs_camera_layout", lib.sgs_camera_layout(arr, len(poses), C.byref(opt), C.byref(tt), C.byref(tp)))
    return int(tt.value), int(tp.value)


def renderer_device_bytes(n: int, n_views: int, enhanced: bool, total_tiles: int, total_pixels: int,
                          capacity: int, opt: _abi.Options | None = None, keep_keys: bool = False,
                          count: bool = False, tile_order: bool = True, persistent: bool = False) -> int:
    """Device bytes a Renderer with these sizes allocates for its forward
    buffers, from the library's own size helpers (the same expressions as
    Renderer.__init__ and alloc_geom)."""
    lib = load()
    opt = opt if opt is not None else _abi.default_options()
    m = n * n_views
    cap = max(int(capacity), 1)
    geom = (4 * int(lib.sgs_geom_rec_floats(m, int(enhanced))) + 4 * max(m, 1) + 4 * max(2 * m, 2)
            + 8 * max(m, 1) + 4 * int(lib.sgs_geom_block_entries(n, n_views)))
    sort = (4 * cap + 8 * total_tiles + 4 + (8 * cap if (keep_keys or opt.sort_mode == 0) else 0)
            + int(lib.sgs_bin_sort_scratch_bytes(m, int(capacity), total_tiles, C.byref(opt))))
    out = 20 * total_pixels + (8 * total_pixels if count else 0)
    sched = (4 * total_tiles if tile_order else 0) + (4 if persistent else 0)
    return geom + sort + out + sched


class Renderer:
    """Fixed-buffer renderer for one Gaussian set and one camera batch.

    All buffers are allocated once; forward() and backward() only enqueue
    library calls on the stream (no allocation, no host synchronisation), so
    they can be timed per call or captured in a HIP graph.  The instance
    capacity is fixed at construction (measured once, with headroom); if a
    later pose needs more, overflowed() reports it and instances past the
    capacity are dropped by the library."""

    def __init__(self, gs: GaussianSet, cams: CameraBatch, opt: _abi.Options | None = None,
                 capacity: int | None = None, headroom: float = 1.25, keep_keys: bool = False,
                 count: bool = False, tile_order: bool = True, persistent: bool = False):
        self.lib = load()
        self.gs, self.cams = gs, cams
        self.opt = opt if opt is not None else _abi.default_options()
        self.m = gs.n * cams.n_views
        self.geom, self.bufs = alloc_geom(self.m, gs.n, cams.n_views, gs.enhanced, gs.mean.device)
        self._params = None
        dev = gs.mean.device
        if capacity is None:
            self.preprocess()
            total = int(self.bufs["block_off"][-1].item()) & 0xFFFFFFFF
            if total == 0xFFFFFFFF:
                raise _abi.SgsError("sgs_preprocess: instance count exceeds 2^32-1", 2)
            capacity = min(int(total * headroom) + 1024, 0xFFFFFFFE)
        self.capacity = int(capacity)
        b = self.bufs
        b["vals"] = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        b["ranges"] = torch.empty(2 * cams.total_tiles, dtype=torch.int32, device=dev)
        b["n_inst"] = torch.zeros(1, dtype=torch.int32, device=dev)
        b["keys"] = (torch.empty(max(self.capacity, 1), dtype=torch.int64, device=dev)
                     if (keep_keys or self.opt.sort_mode == 0) else None)
        self.scratch_bytes = int(self.lib.sgs_bin_sort_scratch_bytes(self.m, self.capacity, cams.total_tiles,
                                                                      C.byref(self.opt)))
        b["scratch"] = torch.empty(self.scratch_bytes, dtype=torch.uint8, device=dev)
        P = cams.total_pixels
        self.out_rgb = torch.empty((3, P), dtype=torch.float32, device=dev)
        self.out_T = torch.empty(P, dtype=torch.float32, device=dev)
        self.out_last = torch.empty(P, dtype=torch.int32, device=dev)
        b["count"] = torch.empty(P, dtype=torch.int32, device=dev) if count else None
        b["eval"] = torch.empty(P, dtype=torch.int32, device=dev) if count else None
        b["tile_order"] = torch.empty(cams.total_tiles, dtype=torch.int32, device=dev) if tile_order else None
        b["work_counter"] = torch.zeros(1, dtype=torch.int32, device=dev) if persistent else None
        self.sched = _abi.Schedule(_ptr(b["tile_order"]), _ptr(b["work_counter"]))
        self._bwd = None
        self.graph = None

    @property
    def params(self) -> _abi.Params:
        if self._params is None:
            self._params = self.gs.struct()
        return self._params

    def device_bytes(self) -> int:
        """Bytes of every buffer this renderer holds (forward buffers; the
        backward's gradient buffer is added once backward() has run)."""
        ts = [v for v in self.bufs.values() if isinstance(v, torch.Tensor)]
        ts += [self.out_rgb, self.out_T, self.out_last]
        if self._bwd is not None:
            ts.append(self._bwd[0])
        return sum(t.numel() * t.element_size() for t in ts)

    # ---- forward stages
    def preprocess(self, stream=None):
        check("sgs_preprocess", self.lib.sgs_preprocess(
            C.byref(self.params), self.cams.host, _ptr(self.cams.dev), self.cams.n_views,
            C.byref(self.opt), C.byref(self.geom), _stream(stream)))

    def bin_sort(self, stream=None):
        b = self.bufs
        check("sgs_bin_sort", self.lib.sgs_bin_sort(
            C.byref(self.geom), self.m, self.cams.host, _ptr(self.cams.dev), self.cams.n_views,
            C.byref(self.opt), self.capacity, _ptr(b["keys"]), _ptr(b["vals"]), _ptr(b["ranges"]),
            _ptr(b["n_inst"]), C.byref(self.sched), _ptr(b["scratch"]), self.scratch_bytes,
            _stream(stream)))

    def blend(self, stream=None, count: bool | None = None):
        """The forward blend; ``count`` (default: as constructed) also writes
        the per-pixel composited and evaluated pair counts."""
        b = self.bufs
        cnt = (b["count"] is not None) if count is None else count
        if cnt and b["count"] is None:
            raise ValueError("this Renderer was built without count buffers")
        check("sgs_render_fwd", self.lib.sgs_render_fwd(
            C.byref(self.geom), self.m, _ptr(b["vals"]), self.capacity, _ptr(b["ranges"]),
            C.byref(self.sched), self.cams.host, _ptr(self.cams.dev), self.cams.n_views,
            int(self.gs.enhanced),
            C.byref(self.opt), _ptr(self.out_rgb), _ptr(self.out_T), _ptr(self.out_last),
            _ptr(b["count"]) if cnt else None, _ptr(b["eval"]) if cnt else None,
            self.cams.total_pixels, _stream(stream)))

    def forward(self, stream=None, count: bool | None = None) -> torch.Tensor:
        self.preprocess(stream)
        self.bin_sort(stream)
        self.blend(stream, count)
        return self.out_rgb

    def capture(self):
        """Captures forward() (preprocess, bin/sort, blend: every kernel of the
        frame) into one HIP graph; replay() then launches the whole frame with
        one call.  Camera poses may change between replays through
        CameraBatch.upload() (same layout); the capacity is fixed."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.forward()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.forward()
        self.graph = g
        return g

    def replay(self) -> torch.Tensor:
        self.graph.replay()
        return self.out_rgb

    def n_inst(self) -> int:
        return int(self.bufs["n_inst"].item()) & 0xFFFFFFFF

    def overflowed(self) -> bool:
        n = self.n_inst()
        if n == N_INVALID:
            raise _abi.SgsError("sgs_bin_sort: a sort look-back did not complete; outputs invalid", 3)
        return n > self.capacity

    def image(self, v: int = 0) -> torch.Tensor:
        c = self.cams.view(v)
        return self.out_rgb[:, c.pix_base:c.pix_base + c.width * c.height].reshape(3, c.height, c.width)

    def transmittance(self, v: int = 0) -> torch.Tensor:
        c = self.cams.view(v)
        return self.out_T[c.pix_base:c.pix_base + c.width * c.height].reshape(c.height, c.width)

    # ---- backward
    def backward(self, dL_drgb: torch.Tensor, stream=None, densify: dict | None = None,
                 events=None) -> dict:
        """Gradients (fresh zeroed buffers reused across calls) for dL/dC;
        ``densify`` (from densify_stats) accumulates the densification
        statistics of this backward; ``events`` (two torch.cuda.Events on
        the current stream) are recorded around the library call alone."""
        gs = self.gs
        if self._bwd is None:
            # the 2D gradients and every parameter gradient are views of one
            # buffer (16-byte aligned pieces), zeroed by a single fill
            n2d = int(self.lib.sgs_geom_rec_floats(self.m, int(gs.enhanced)))
            sizes = [(f, getattr(gs, f)) for f in GaussianSet.FIELDS if getattr(gs, f) is not None]
            total = (n2d + 3) // 4 * 4 + sum((v.numel() + 3) // 4 * 4 for _, v in sizes)
            flat = torch.empty(total, dtype=torch.float32, device=gs.mean.device)
            g2d = flat[:n2d]
            off = (n2d + 3) // 4 * 4
            grads = {f: None for f in GaussianSet.FIELDS}
            for f, v in sizes:
                grads[f] = flat[off:off + v.numel()].view(v.shape)
                off += (v.numel() + 3) // 4 * 4
            self._bwd = (flat, g2d, grads, _abi.GeomGrad(_ptr(g2d)))
        flat, g2d, grads, gg = self._bwd
        pg = _params_grad(grads, densify)
        flat.zero_()
        b = self.bufs
        if events is not None:
            events[0].record()
        check("sgs_render_bwd", self.lib.sgs_render_bwd(
            C.byref(self.params), C.byref(self.geom), self.m, _ptr(b["vals"]), self.capacity,
            _ptr(b["ranges"]), C.byref(self.sched), self.cams.host, _ptr(self.cams.dev), self.cams.n_views, C.byref(self.opt),
            _ptr(self.out_T), _ptr(self.out_last), _ptr(dL_drgb), self.cams.total_pixels,
            C.byref(gg), C.byref(pg), _stream(stream)))
        if events is not None:
            events[1].record()
        return grads


def densify(gs: GaussianSet, stats: dict | None, opt: "_abi.DensifyOptions | None" = None,
            capacity: int | None = None, stream=None):
    """Densification step (sgs_densify): decisions (0 keep, 1 clone, 2 split)
    from the statistics of densify_stats() accumulated by backward passes,
    and the new GaussianSet with the cloned and split Gaussians.  Without
    ``capacity`` the number of outputs is read back first (one host sync)
    and the new set is sized exactly.  Returns (new set, decisions, parent
    index of each new Gaussian)."""
    lib = load()
    if opt is None:
        opt = _abi.DensifyOptions()
        lib.sgs_default_densify_options(C.byref(opt))
    dev = gs.mean.device
    n = gs.n
    st = stats or {}
    decision = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    n_out = torch.zeros(1, dtype=torch.int32, device=dev)
    scratch = torch.empty(int(lib.sgs_densify_scratch_words(n)), dtype=torch.int32, device=dev)
    p = gs.struct()

    def call(out):
        check("sgs_densify", lib.sgs_densify(C.byref(p), _ptr(st.get("uv")), _ptr(st.get("count")),
                                             _ptr(st.get("z")), C.byref(opt), _ptr(decision), C.byref(out),
                                             _ptr(n_out), _ptr(scratch), _stream(stream)))

    if capacity is None:
        call(_abi.DensifyOut())
        capacity = int(n_out.item())
    new = {f: (None if getattr(gs, f) is None else
               torch.empty((*getattr(gs, f).shape[:-1], capacity), dtype=torch.float32, device=dev))
           for f in GaussianSet.FIELDS}
    parent = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    out = _abi.DensifyOut(capacity, *[_ptr(new[f]) for f in GaussianSet.FIELDS], _ptr(parent))
    call(out)
    ns = GaussianSet(new["mean"], new["log_scale"], new["quat"], new["skew"], new["opa_logit"], new["sh"],
                     gs.sh_degree, new["opa2_logit"], new["opa_dir"])
    return ns, decision[:n], parent[:capacity]
