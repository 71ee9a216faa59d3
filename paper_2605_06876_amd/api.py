"""Python binding of the C-ABI in include/adpsplit.h (argument marshalling only).

Every step of the path runs in the HIP kernels of libadpsplit.so; this module
builds the C structs from torch tensors and forwards the calls.  If the
library is missing it raises: there is no CPU fallback.

Tensors follow the library layout: Gaussians struct-of-arrays float32 on the
GPU (means [3,n], log_scales [3,n], quats [4,n], opacity_logits [n],
sh [(d+1)^2,3,n]); images [3,H,W]; per-pixel maps [H,W].
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadpsplit.so")
_lib = None

AS_OK, AS_ERR_ARG, AS_ERR_CAPACITY, AS_ERR_HIP, AS_ERR_STATE = 0, 1, 2, 3, 4
MAX_VIEWS = 16   # views of one batched render
MODE_VANILLA, MODE_RESET, MODE_ADAPTIVE = 0, 1, 2


class AdpSplitError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("adpsplit status %d: %s" % (status, msg))
        self.status = status


class _Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("bg", ctypes.c_float * 3)]


class _Gaussians(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity_logits", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("sh_degree", ctypes.c_int32), ("n_dev", ctypes.c_void_p)]


class _GaussiansMut(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity_logits", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("sh_degree", ctypes.c_int32)]

    @staticmethod
    def of(g):
        m = _GaussiansMut()
        m.means, m.log_scales, m.quats = _ptr(g.means), _ptr(g.log_scales), _ptr(g.quats)
        m.opacity_logits, m.sh = _ptr(g.opacity_logits), _ptr(g.sh)
        m.n, m.sh_degree = int(g.means.shape[1]), g.sh_degree
        return m


class _SplitParams(ctypes.Structure):
    _fields_ = [("tau_l1", ctypes.c_double), ("r_erode", ctypes.c_int32), ("m_min", ctypes.c_int32),
                ("L", ctypes.c_int32), ("n_max", ctypes.c_int32), ("gamma_d", ctypes.c_double),
                ("gamma_c", ctypes.c_double), ("eps", ctypes.c_double), ("eta", ctypes.c_double),
                ("variant", ctypes.c_int32), ("flags", ctypes.c_uint32), ("fixed_n", ctypes.c_int32),
                ("noise_n", ctypes.c_int32)]


class _RegionBuf(ctypes.Structure):
    _fields_ = [("records", ctypes.c_void_p), ("capacity", ctypes.c_int64), ("count", ctypes.c_void_p)]


class _FrameView(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("n_cap", ctypes.c_int64), ("key_cap", ctypes.c_int64), ("tile_base", ctypes.c_int32),
                ("ent_base", ctypes.c_uint32)] + [
        (nm, ctypes.c_void_p) for nm in ("n_keys", "keys", "vals", "ranges", "depth_key", "box", "ntiles", "rec",
                                         "t_final", "last", "n_contrib", "dom", "err", "err_minmax", "grad2d")] + [
        ("grad2d_stride", ctypes.c_int64), ("bin_size", ctypes.c_int32), ("bin_base", ctypes.c_int32),
        ("bins_x", ctypes.c_int32), ("bins_y", ctypes.c_int32)]


REGION_DTYPE = np.dtype([
    ("cand", "<i4"), ("view", "<i4"), ("label", "<i4"), ("area", "<i4"), ("band", "<i4"), ("pad0", "<i4"),
    ("sx", "<i8"), ("sy", "<i8"), ("sxx", "<i8"), ("sxy", "<i8"), ("syy", "<i8"),
    ("cx", "<f8"), ("cy", "<f8"), ("cov", "<f8", (3,)), ("e1", "<f8", (2,)), ("sigma1", "<f8"), ("sigma2", "<f8"),
    ("rgb", "<f4", (3,)), ("pad1", "<f4")])
assert REGION_DTYPE.itemsize == 152

class _Reserve(ctypes.Structure):
    _fields_ = [("max_pixels", ctypes.c_int64), ("max_gaussians", ctypes.c_int64), ("max_candidates", ctypes.c_int64),
                ("max_regions", ctypes.c_int64), ("max_views", ctypes.c_int32)]


RESERVE_FIELDS = ("max_pixels", "max_gaussians", "max_candidates", "max_regions", "max_views")
FRAME_FORWARD_ONLY = 1

EXPORTED = ("as_ctx_create", "as_ctx_destroy", "as_last_error", "as_version", "as_ctx_reserve", "as_ctx_get_reserve",
            "as_ctx_reserve_bytes", "as_frame_create", "as_frame_create_batch", "as_frame_reserve_keys",
            "as_frame_bytes", "as_workspace_size", "as_frame_destroy", "as_frame_get_view", "as_frame_get_view_of",
            "as_frame_pair_count", "as_render",
            "as_render_backward", "as_render_batch", "as_render_backward_batch", "as_error_map",
            "as_accumulate_error_stats", "as_accumulate_error_stats_noalloc", "as_adaptive_split", "as_set_tuning", "as_get_tuning", "as_timing_enable",
            "as_timing_read", "as_graph_begin", "as_graph_end", "as_graph_launch", "as_graph_destroy",
            "as_debug_sort_pairs", "as_debug_sort_u32", "as_debug_fp64_ops", "as_debug_blend_alpha", "as_debug_row_addressing", "as_adam_step", "as_l1_loss", "as_densify_select",
            "as_split_row_map", "as_clone_prune", "as_gather_rows", "as_reset_opacity")
_NO_STATUS = ("as_last_error", "as_version", "as_ctx_destroy", "as_frame_destroy", "as_graph_destroy")

STAGES = ("project", "scan", "emit", "sort", "ranges", "blend_fwd", "blend_bwd", "project_bwd", "error_map",
          "error_stats", "split")


def lib():
    """Load libadpsplit.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libadpsplit.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name in EXPORTED:
            getattr(L, name)
        L.as_last_error.restype = ctypes.c_char_p
        L.as_version.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in _NO_STATUS:
                getattr(L, name).restype = ctypes.c_int
        L.as_ctx_destroy.restype = None
        L.as_frame_destroy.restype = None
        L.as_graph_destroy.restype = None
        _lib = L
    return _lib


def _check(status):
    if status != AS_OK:
        raise AdpSplitError(status, lib().as_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def camera_struct(cam):
    c = _Camera()
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    bg = np.asarray(cam.bg, np.float32).reshape(3)
    for k in range(3):
        c.bg[k] = float(bg[k])
    return c


VARIANT_ADPSPLIT, VARIANT_FIXED_N, VARIANT_ADAPTIVE_N, VARIANT_CHILD_INIT = 0, 1, 2, 3
SPLIT_ERODE_SIDE, SPLIT_CROSS_VIEW, SPLIT_EXTENT_MAX, SPLIT_SHARE_OPACITY = 1, 2, 4, 8
MODE_RANDOM = 3


class SplitParams:
    """AdpSplit hyper-parameters; defaults from Sec. 5 (tau_l1 0.1, r_erode 2,
    m_min 5, L 3, N_max 19, gamma_d 2.0, gamma_c 0.15), eps 1e-8, eta 0.8;
    variant / flags / fixed_n / noise_n as as_split_params."""

    def __init__(self, tau_l1=0.1, r_erode=2, m_min=5, L=3, n_max=19, gamma_d=2.0, gamma_c=0.15, eps=1e-8, eta=0.8,
                 variant=0, flags=0, fixed_n=2, noise_n=0):
        self.tau_l1, self.r_erode, self.m_min, self.L, self.n_max = tau_l1, r_erode, m_min, L, n_max
        self.gamma_d, self.gamma_c, self.eps, self.eta = gamma_d, gamma_c, eps, eta
        self.variant, self.flags, self.fixed_n, self.noise_n = variant, flags, fixed_n, noise_n

    def struct(self):
        return _SplitParams(self.tau_l1, self.r_erode, self.m_min, self.L, self.n_max, self.gamma_d, self.gamma_c,
                            self.eps, self.eta, self.variant, self.flags, self.fixed_n, self.noise_n)


class Gaussians:
    """Device-resident Gaussians (torch tensors in the library layout)."""

    FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree, n_dev=None):
        self.means, self.log_scales, self.quats = means, log_scales, quats
        self.opacity_logits, self.sh, self.sh_degree = opacity_logits, sh, int(sh_degree)
        # optional device [1] int64: the rows in use (n is then the capacity)
        self.n_dev = n_dev

    def counted(self, n_dev):
        """The same buffers with a device row count (for the densification calls)."""
        return Gaussians(self.means, self.log_scales, self.quats, self.opacity_logits, self.sh, self.sh_degree, n_dev)

    @property
    def n(self):
        return int(self.means.shape[1])

    @staticmethod
    def from_scene(scene, device="cuda"):
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return Gaussians(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.opacity_logits), t(scene.sh),
                         scene.sh_degree)

    @staticmethod
    def empty(n, sh_degree, device="cuda"):
        nk = (sh_degree + 1) ** 2
        z = lambda *s: torch.zeros(*s, dtype=torch.float32, device=device)
        return Gaussians(z(3, n), z(3, n), z(4, n), z(n), z(nk, 3, n), sh_degree)

    def tensors(self):
        return [getattr(self, f) for f in self.FIELDS]

    def struct(self):
        return _Gaussians(_ptr(self.means), _ptr(self.log_scales), _ptr(self.quats), _ptr(self.opacity_logits),
                          _ptr(self.sh), self.n, self.sh_degree, _ptr(self.n_dev))

    def rows(self, n):
        """First n rows (views with the full row stride are not contiguous, so copy)."""
        return Gaussians(self.means[:, :n].contiguous(), self.log_scales[:, :n].contiguous(),
                         self.quats[:, :n].contiguous(), self.opacity_logits[:n].contiguous(),
                         self.sh[:, :, :n].contiguous(), self.sh_degree)


def _reserve_struct(r):
    unknown = set(r) - set(RESERVE_FIELDS)
    if unknown:
        raise TypeError("unknown reservation fields %s" % sorted(unknown))
    return _Reserve(*[int(r.get(f, 0)) for f in RESERVE_FIELDS])


def reserve_bytes(**r):
    """as_ctx_reserve_bytes: device bytes of a context reservation."""
    out = ctypes.c_size_t()
    _check(lib().as_ctx_reserve_bytes(ctypes.byref(_reserve_struct(r)), ctypes.byref(out)))
    return int(out.value)


def frame_bytes(max_views, entry_cap, pixel_cap, tile_cap, key_cap, forward_only=False):
    """as_frame_bytes: device bytes of a frame with these capacities."""
    out = ctypes.c_size_t()
    _check(lib().as_frame_bytes(ctypes.c_int32(max_views), ctypes.c_int64(entry_cap), ctypes.c_int64(pixel_cap),
                                ctypes.c_int64(tile_cap), ctypes.c_int64(key_cap),
                                ctypes.c_uint32(FRAME_FORWARD_ONLY if forward_only else 0), ctypes.byref(out)))
    return int(out.value)


def workspace_size(ctx, n, cams, key_cap, forward_only=False):
    """as_workspace_size: bytes of the frame for n Gaussians in these cameras."""
    out = ctypes.c_size_t()
    cs = (_Camera * len(cams))(*[camera_struct(c) for c in cams])
    _check(lib().as_workspace_size(ctx.handle, ctypes.c_int64(n), cs, ctypes.c_int32(len(cams)),
                                   ctypes.c_int64(key_cap), ctypes.c_uint32(FRAME_FORWARD_ONLY if forward_only else 0),
                                   ctypes.byref(out)))
    return int(out.value)


class Context:
    """An as_ctx bound to one device.  Keyword arguments (max_pixels,
    max_gaussians, max_candidates, max_regions, max_views) reserve the
    context's scratch at creation (as_ctx_reserve); the error statistics, the
    split and the loop's densification calls raise AS_ERR_CAPACITY beyond
    the reservation, they never allocate."""

    def __init__(self, device=0, **reserve):
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().as_ctx_create(ctypes.c_int(device), ctypes.byref(h)))
        self.handle = h
        if reserve:
            self.reserve(**reserve)

    def reserve(self, **r):
        """Grow the reservation to at least r (fields as as_reserve)."""
        _check(lib().as_ctx_reserve(self.handle, ctypes.byref(_reserve_struct(r))))

    def reserved(self):
        r = _Reserve()
        _check(lib().as_ctx_get_reserve(self.handle, ctypes.byref(r)))
        return {f: int(getattr(r, f)) for f in RESERVE_FIELDS}

    def close(self):
        if self.handle:
            lib().as_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Frame:
    """Rasterizer state (as_frame): one view of a fixed size, or (batch=True
    through BatchFrame) up to 16 views of any sizes.  The library renders into
    a frame without allocating or synchronising; with auto_grow the binding's
    render helpers read the pair count back after each render and, when it
    exceeds the capacity, reserve more (as_frame_reserve_keys) and render
    again.  forward_only frames hold no reverse-pass checkpoints."""

    def __init__(self, ctx, n_cap, width, height, key_cap=None, auto_grow=True, forward_only=False):
        if key_cap is None:
            key_cap = max(1 << 16, 8 * n_cap)
        h = ctypes.c_void_p()
        _check(lib().as_frame_create(ctx.handle, ctypes.c_int64(n_cap), ctypes.c_int32(width), ctypes.c_int32(height),
                                     ctypes.c_int64(key_cap), ctypes.c_uint32(FRAME_FORWARD_ONLY if forward_only else 0),
                                     ctypes.byref(h)))
        self.ctx, self.handle, self.width, self.height, self.n_cap = ctx, h, width, height, n_cap
        self.auto_grow = auto_grow

    def reserve_keys(self, key_cap):
        """as_frame_reserve_keys (a set-up call: synchronises, may allocate)."""
        _check(lib().as_frame_reserve_keys(self.handle, ctypes.c_int64(key_cap)))

    def _check_capturable(self):
        if self.auto_grow and torch.cuda.is_current_stream_capturing():
            raise AdpSplitError(AS_ERR_STATE, "a frame with auto_grow reads its pair count back after each render "
                                              "and cannot be captured in a graph")

    def _fit_keys(self):
        """After a render: True (and the pair buffers grown) when its pairs did
        not fit, so the caller renders again."""
        if not self.auto_grow:
            return False
        K = self.n_keys()
        if K <= self.key_cap:
            return False
        self.reserve_keys(min(K + K // 4 + 1024, 0xFFFFFFFF))
        return True

    def view(self, v=0):
        out = _FrameView()
        _check(lib().as_frame_get_view_of(self.handle, ctypes.c_int32(v), ctypes.byref(out)))
        return out

    def close(self):
        if self.handle:
            lib().as_frame_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # host copies of the frame state, for tests and tools ----------------------
    def _dev(self, addr, nbytes):
        """Copy nbytes of device memory to a host numpy byte array."""
        out = np.empty(max(nbytes, 1), np.uint8)[:nbytes]
        if nbytes:
            torch.cuda.synchronize()
            _memcpy_d2h(out.ctypes.data, addr, nbytes)
        return out

    def n_keys(self):
        """Pairs the last render needed (all views)."""
        v = self.view()
        return int(self._dev(v.n_keys, 4).view(np.uint32)[0])

    def n_emitted(self):
        """Pairs the last render wrote (fewer than n_keys() when over key_cap)."""
        v = self.view()
        return int(self._dev(v.n_keys, 8).view(np.uint32)[1])

    def pair_count_async(self, dst, stream=None):
        """Queue a copy of the last render's pair count into dst (int32 [1], device)."""
        _check(lib().as_frame_pair_count(self.handle, _ptr(dst), _stream(stream)))

    @property
    def key_cap(self):
        return int(self.view().key_cap)

    def host_state(self, n, view=0):
        """Keys, values, ranges, per-Gaussian and per-pixel state of one view
        as numpy arrays.  `tile_keys`/`vals` are the sorted pairs of all views
        (global bin ids, entry ids; bins are the 16 x 16 tiles unless the
        tuning bins by 32, `bin_size`); `keys` restates each pair as
        (bin of the view) << 32 | depth bits, the form of a (bin | depth)
        sort, and `gauss` its Gaussian id (meaningful for this view's pairs);
        `ranges` are per 16 x 16 tile (a tile's range is its bin's)."""
        v = self.view(view)
        K = self.n_emitted()
        H, W = v.height, v.width
        P = W * H
        T = v.tiles_x * v.tiles_y
        tk = self._dev(v.keys, 4 * K).view(np.uint32)
        vals = self._dev(v.vals, 4 * K).view(np.uint32)
        ne = int(vals.max()) + 1 if K else 0
        dk_all = self._dev(v.depth_key - 4 * v.ent_base, 4 * ne).view(np.uint32)
        keys = ((tk.astype(np.int64) - v.bin_base).astype(np.uint64) << np.uint64(32)) | \
            (dk_all[vals].astype(np.uint64) if K else np.zeros(0, np.uint64))
        return dict(
            n_keys=self.n_keys(), tile_keys=tk, keys=keys, vals=vals,
            gauss=(vals.astype(np.int64) - v.ent_base).astype(np.uint32),
            ranges=self._dev(v.ranges, 8 * T).view(np.uint32).reshape(T, 2),
            depth_key=self._dev(v.depth_key, 4 * n).view(np.uint32), box=self._dev(v.box, 8 * n).view(np.int16).reshape(n, 4),
            ntiles=self._dev(v.ntiles, 4 * n).view(np.uint32), rec=self._dev(v.rec, 48 * n).view(np.float32).reshape(n, 12),
            t_final=self._dev(v.t_final, 4 * P).view(np.float32).reshape(H, W),
            last=self._dev(v.last, 4 * P).view(np.uint32).reshape(H, W),
            n_contrib=self._dev(v.n_contrib, 4 * P).view(np.uint32).reshape(H, W),
            dom=self._dev(v.dom, 4 * P).view(np.int32).reshape(H, W),
            err=self._dev(v.err, 8 * P).view(np.float64).reshape(H, W),
            err_minmax=self._dev(v.err_minmax, 16).view(np.uint64),
            tiles_x=v.tiles_x, tiles_y=v.tiles_y, tile_base=v.tile_base, ent_base=v.ent_base, bin_size=v.bin_size,
            bin_base=v.bin_base, bins_x=v.bins_x, bins_y=v.bins_y)

    def device_maps(self, view=0):
        """Device addresses of one view's per-pixel maps (for accumulate_error_stats)."""
        v = self.view(view)
        return dict(err=v.err, err_minmax=v.err_minmax, dom=v.dom, t_final=v.t_final, width=v.width,
                    height=v.height)


class BatchFrame(Frame):
    """as_frame_create_batch: state for batched renders of up to max_views views."""

    def __init__(self, ctx, max_views, entry_cap, pixel_cap, tile_cap, key_cap=None, auto_grow=True,
                 forward_only=False):
        if key_cap is None:
            key_cap = max(1 << 16, 8 * entry_cap)
        h = ctypes.c_void_p()
        _check(lib().as_frame_create_batch(ctx.handle, ctypes.c_int32(max_views), ctypes.c_int64(entry_cap),
                                           ctypes.c_int64(pixel_cap), ctypes.c_int64(tile_cap),
                                           ctypes.c_int64(key_cap),
                                           ctypes.c_uint32(FRAME_FORWARD_ONLY if forward_only else 0),
                                           ctypes.byref(h)))
        self.ctx, self.handle, self.n_cap, self.max_views = ctx, h, entry_cap, max_views
        self.auto_grow = auto_grow

    @staticmethod
    def for_views(ctx, n_per_view, cams, key_cap=None, auto_grow=True, forward_only=False):
        """A frame sized for exactly these views (n_per_view: int or list)."""
        ns = n_per_view if isinstance(n_per_view, (list, tuple)) else [n_per_view] * len(cams)
        tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
        return BatchFrame(ctx, len(cams), sum(ns), sum(c.width * c.height for c in cams), tiles, key_cap, auto_grow,
                          forward_only)


_hiprt = None


def _memcpy_d2h(dst, src, nbytes):
    """Device-to-host copy through the HIP runtime already loaded by torch
    (dlopen by soname returns the loaded object, so there is one runtime)."""
    global _hiprt
    if _hiprt is None:
        _hiprt = ctypes.CDLL("libamdhip64.so.7")
        _hiprt.hipMemcpy.restype = ctypes.c_int
    rc = _hiprt.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes), ctypes.c_int(2))
    if rc != 0:
        raise RuntimeError("hipMemcpy failed: %d" % rc)


# ---- the four calls -------------------------------------------------------------------

def render(ctx, g, cam, frame, gt=None, image=None, stream=None):
    """as_render: image [3,H,W]; the frame keeps the state for backward and
    error statistics."""
    if image is None:
        image = torch.empty(3, cam.height, cam.width, dtype=torch.float32, device="cuda")
    gs = g.struct()
    c = camera_struct(cam)
    frame._check_capturable()
    while True:
        _check(lib().as_render(ctx.handle, ctypes.byref(gs), ctypes.byref(c), frame.handle, _ptr(gt), _ptr(image),
                               _stream(stream)))
        if not frame._fit_keys():
            return image


def render_backward(ctx, g, cam, frame, dL_dimage, grads=None, g2d_norm=None, vis_count=None, stream=None):
    """as_render_backward: gradients w.r.t. the stored parameters."""
    if grads is None:
        grads = Gaussians.empty(g.n, g.sh_degree)
    gs = g.struct()
    c = camera_struct(cam)
    gm = _GaussiansMut.of(grads)
    _check(lib().as_render_backward(ctx.handle, ctypes.byref(gs), ctypes.byref(c), frame.handle, _ptr(dL_dimage),
                                    ctypes.byref(gm), _ptr(g2d_norm), _ptr(vis_count), _stream(stream)))
    return grads


def render_batch(ctx, scenes, cams, frame, gts=None, images=None, stream=None):
    """as_render_batch: scenes is one Gaussians (shared by every view) or a
    list with one per view; returns the list of images [3,H_v,W_v]."""
    V = len(cams)
    if not isinstance(scenes, (list, tuple)):
        scenes = [scenes] * V
    if images is None:
        images = [torch.empty(3, c.height, c.width, dtype=torch.float32, device="cuda") for c in cams]
    ss = (_Gaussians * V)(*[g.struct() for g in scenes])
    cs = (_Camera * V)(*[camera_struct(c) for c in cams])
    ims = (ctypes.c_void_p * V)(*[_ptr(t).value for t in images])
    gp = (ctypes.c_void_p * V)(*[_ptr(t).value for t in gts]) if gts is not None else None
    frame._check_capturable()
    while True:
        _check(lib().as_render_batch(ctx.handle, ss, cs, ctypes.c_int32(V), frame.handle, gp, ims, _stream(stream)))
        if not frame._fit_keys():
            return images


def render_backward_batch(ctx, g, frame, dL_dimages, grads=None, g2d_norm=None, vis_count=None, stream=None):
    """as_render_backward_batch: gradients summed over the views of the last
    batched render of g."""
    if grads is None:
        grads = Gaussians.empty(g.n, g.sh_degree)
    gs = g.struct()
    gm = _GaussiansMut.of(grads)
    V = len(dL_dimages)
    dl = (ctypes.c_void_p * V)(*[_ptr(t).value for t in dL_dimages])
    _check(lib().as_render_backward_batch(ctx.handle, ctypes.byref(gs), frame.handle, dl, ctypes.byref(gm),
                                          _ptr(g2d_norm), _ptr(vis_count), _stream(stream)))
    return grads


class Graph:
    """A HIP graph of library calls recorded on one stream (as_graph_*)."""

    def __init__(self, handle):
        self.handle = handle

    @staticmethod
    def capture(ctx, fn, stream):
        """Record fn() on `stream` (a torch.cuda.Stream, not the null stream)."""
        s = ctypes.c_void_p(stream.cuda_stream)
        _check(lib().as_graph_begin(ctx.handle, s))
        h = ctypes.c_void_p()
        try:
            with torch.cuda.stream(stream):
                fn()
        except BaseException:
            if lib().as_graph_end(ctx.handle, s, ctypes.byref(h)) == AS_OK:
                lib().as_graph_destroy(h)
            raise
        _check(lib().as_graph_end(ctx.handle, s, ctypes.byref(h)))
        return Graph(h)

    def launch(self, stream):
        _check(lib().as_graph_launch(self.handle, ctypes.c_void_p(stream.cuda_stream)))

    def close(self):
        if self.handle:
            lib().as_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def error_map(ctx, image, gt, err=None, err_minmax=None, stream=None):
    """as_error_map: FP64 L1 error map and its min/max bit patterns."""
    H, W = image.shape[1], image.shape[2]
    if err is None:
        err = torch.empty(H, W, dtype=torch.float64, device="cuda")
    if err_minmax is None:
        err_minmax = torch.empty(2, dtype=torch.int64, device="cuda")
    _check(lib().as_error_map(ctx.handle, ctypes.c_int32(W), ctypes.c_int32(H), _ptr(image), _ptr(gt), _ptr(err),
                              _ptr(err_minmax), _stream(stream)))
    return err, err_minmax


class RegionBuffer:
    """Device region records (as_region_buf)."""

    def __init__(self, capacity):
        self.capacity = int(capacity)
        self.records = torch.zeros(self.capacity * REGION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        self.count = torch.zeros(1, dtype=torch.int64, device="cuda")

    def struct(self):
        return _RegionBuf(_ptr(self.records), self.capacity, _ptr(self.count))

    def reset(self):
        self.count.zero_()

    def host(self):
        n = int(self.count.item())
        if n > self.capacity:
            raise AdpSplitError(AS_ERR_CAPACITY, "region buffer overflow: %d > %d" % (n, self.capacity))
        return self.records[: n * REGION_DTYPE.itemsize].cpu().numpy().view(REGION_DTYPE).copy()


def accumulate_error_stats(ctx, width, height, err, err_minmax, dom, gt, view_id, is_candidate, params, regions,
                           attr_count, stream=None):
    """as_accumulate_error_stats for one view.  err/err_minmax/dom may be
    torch tensors or raw device addresses (ints) from a frame."""
    p = params.struct()
    rb = regions.struct()
    addr = lambda x: ctypes.c_void_p(x) if isinstance(x, int) else _ptr(x)
    _check(lib().as_accumulate_error_stats(ctx.handle, ctypes.c_int32(width), ctypes.c_int32(height), addr(err),
                                           addr(err_minmax), addr(dom), _ptr(gt), ctypes.c_int32(view_id),
                                           ctypes.c_int64(is_candidate.shape[0]), _ptr(is_candidate), ctypes.byref(p),
                                           ctypes.byref(rb), _ptr(attr_count), _stream(stream)))


NOALLOC_MAX_PIXELS = 1 << 20


def accumulate_error_stats_noalloc(ctx, width, height, err, err_minmax, dom, gt, view_id, is_candidate, params,
                                   regions, attr_count, stream=None):
    """as_accumulate_error_stats_noalloc: the same call with the library's
    static scratch (views up to NOALLOC_MAX_PIXELS pixels)."""
    p = params.struct()
    rb = regions.struct()
    addr = lambda x: ctypes.c_void_p(x) if isinstance(x, int) else _ptr(x)
    _check(lib().as_accumulate_error_stats_noalloc(ctx.handle, ctypes.c_int32(width), ctypes.c_int32(height),
                                                   addr(err), addr(err_minmax), addr(dom), _ptr(gt),
                                                   ctypes.c_int32(view_id), ctypes.c_int64(is_candidate.shape[0]),
                                                   _ptr(is_candidate), ctypes.byref(p), ctypes.byref(rb),
                                                   _ptr(attr_count), _stream(stream)))


def split_rows_per_candidate(params):
    """Rows the split appends per candidate at most (the output bound is
    n + n_cand times this): fixed_n for the fixed-N split, else
    max(2, N_max + 1)."""
    return params.fixed_n if params.variant == VARIANT_FIXED_N else max(2, params.n_max + 1)


def adaptive_split(ctx, g, cand, regions, views, attr_count, params, noise, out=None, mode=None, count=None,
                   offset=None, n_out=None, n_cand_dev=None, stream=None):
    """as_adaptive_split.  Returns (out Gaussians with capacity rows, mode,
    count, offset, n_out tensor); outputs not passed are allocated here.
    n_cand_dev: optional device count of the candidates in use (cand's length
    is then a capacity)."""
    nc = int(cand.shape[0])
    if out is None:
        cap = g.n + nc * split_rows_per_candidate(params)
        out = Gaussians.empty(max(cap, 1), g.sh_degree)
    if mode is None:
        mode = torch.zeros(max(nc, 1), dtype=torch.uint8, device="cuda")
    if count is None:
        count = torch.zeros(max(nc, 1), dtype=torch.int32, device="cuda")
    if offset is None:
        offset = torch.zeros(max(nc, 1), dtype=torch.int64, device="cuda")
    if n_out is None:
        n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    cams = (_Camera * max(len(views), 1))(*[camera_struct(v) for v in views])
    gs = g.struct()
    p = params.struct()
    rb = regions.struct()
    om = _GaussiansMut.of(out)
    _check(lib().as_adaptive_split(ctx.handle, ctypes.byref(gs), _ptr(cand) if nc else None, ctypes.c_int64(nc),
                                   ctypes.byref(rb), cams, ctypes.c_int32(len(views)), _ptr(attr_count), ctypes.byref(p),
                                   _ptr(noise) if nc else None, ctypes.byref(om), _ptr(mode) if nc else None,
                                   _ptr(count) if nc else None, _ptr(offset) if nc else None, _ptr(n_out), _ptr(n_cand_dev),
                                   _stream(stream)))
    return out, mode[:nc], count[:nc], offset[:nc], n_out


# ---- optimisation loop -----------------------------------------------------------

class _AdamParams(ctypes.Structure):
    _fields_ = [(f, ctypes.c_float) for f in ("lr_means", "lr_log_scales", "lr_quats", "lr_opacity", "lr_sh_dc",
                                              "lr_sh_rest", "beta1", "beta2", "eps")]


class AdamParams:
    """Adam with 3DGS's per-group learning rates (means 1.6e-4 times the scene
    extent, decayed by the caller; log scales 5e-3; quaternions 1e-3;
    opacity 5e-2; SH DC 2.5e-3, higher SH 2.5e-3 / 20; eps 1e-15)."""

    def __init__(self, lr_means=1.6e-4, lr_log_scales=5e-3, lr_quats=1e-3, lr_opacity=5e-2, lr_sh_dc=2.5e-3,
                 lr_sh_rest=2.5e-3 / 20, beta1=0.9, beta2=0.999, eps=1e-15):
        self.lr_means, self.lr_log_scales, self.lr_quats, self.lr_opacity = lr_means, lr_log_scales, lr_quats, lr_opacity
        self.lr_sh_dc, self.lr_sh_rest, self.beta1, self.beta2, self.eps = lr_sh_dc, lr_sh_rest, beta1, beta2, eps

    def struct(self):
        return _AdamParams(self.lr_means, self.lr_log_scales, self.lr_quats, self.lr_opacity, self.lr_sh_dc,
                           self.lr_sh_rest, self.beta1, self.beta2, self.eps)


def adam_step(ctx, params, grads, m, v, hp, step, stream=None):
    """as_adam_step: params, m, v updated in place."""
    pm, mm, vm = _GaussiansMut.of(params), _GaussiansMut.of(m), _GaussiansMut.of(v)
    gs = grads.struct()
    h = hp.struct()
    _check(lib().as_adam_step(ctx.handle, ctypes.byref(pm), ctypes.byref(gs), ctypes.byref(mm), ctypes.byref(vm),
                              ctypes.byref(h), ctypes.c_int32(step), _stream(stream)))


def l1_loss(ctx, image, gt, dL=None, sums=None, want_grad=True, stream=None):
    """as_l1_loss: returns (dL or None, sums[2] = (sum |d|, sum d^2)) on the device."""
    H, W = image.shape[1], image.shape[2]
    if want_grad and dL is None:
        dL = torch.empty_like(image)
    if sums is None:
        sums = torch.empty(2, dtype=torch.float64, device="cuda")
    _check(lib().as_l1_loss(ctx.handle, ctypes.c_int32(W), ctypes.c_int32(H), _ptr(image), _ptr(gt),
                            _ptr(dL) if want_grad else None, _ptr(sums), _stream(stream)))
    return (dL if want_grad else None), sums


def densify_select(ctx, g, g2d_accum, vis_count, grad_threshold, size_threshold, out=None, stream=None):
    """as_densify_select: (clone_mask u8 [n], is_candidate u8 [n], cand i32 [n] (first n_cand valid), n_cand);
    out: optional preallocated (clone, is_cand, cand, n_cand) of those shapes."""
    n = g.n
    if out is None:
        clone = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
        is_cand = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
        cand = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        n_cand = torch.empty(1, dtype=torch.int64, device="cuda")
    else:
        clone, is_cand, cand, n_cand = out
    gs = g.struct()
    _check(lib().as_densify_select(ctx.handle, ctypes.byref(gs), _ptr(g2d_accum), _ptr(vis_count),
                                   ctypes.c_double(grad_threshold), ctypes.c_double(size_threshold), _ptr(clone),
                                   _ptr(is_cand), _ptr(cand), _ptr(n_cand), _stream(stream)))
    return clone[:n], is_cand[:n], cand, n_cand


def split_row_map(ctx, n, cand, mode, capacity, state_in=None, n_dev=None, n_cand_dev=None, row_src=None,
                  stream=None):
    """as_split_row_map: row_src i32 [capacity] (n_dev, n_cand_dev: optional
    device counts, n and len(cand) then being capacities)."""
    nc = int(cand.shape[0])
    if row_src is None:
        row_src = torch.empty(max(capacity, 1), dtype=torch.int32, device="cuda")
    _check(lib().as_split_row_map(ctx.handle, ctypes.c_int64(n), _ptr(cand) if nc else None, ctypes.c_int64(nc),
                                  _ptr(mode) if nc else None, _ptr(state_in), _ptr(row_src), ctypes.c_int64(capacity),
                                  _ptr(n_dev), _ptr(n_cand_dev), _stream(stream)))
    return row_src[:capacity]


def clone_prune(ctx, g, clone_mask, state_in, min_opacity, max_scale, out=None, state_src=None, n_out=None,
                stream=None):
    """as_clone_prune: (out Gaussians with 2 n rows of capacity (n without a
    clone mask), state_src i32, n_out device tensor).  g may carry a device row
    count (g.counted)."""
    n = g.n
    if out is None:
        out = Gaussians.empty(max(2 * n if clone_mask is not None else n, 1), g.sh_degree)
    if state_src is None:
        state_src = torch.empty(max(out.n, 1), dtype=torch.int32, device="cuda")
    if n_out is None:
        n_out = torch.empty(1, dtype=torch.int64, device="cuda")
    gs = g.struct()
    om = _GaussiansMut.of(out)
    _check(lib().as_clone_prune(ctx.handle, ctypes.byref(gs), _ptr(clone_mask), _ptr(state_in),
                                ctypes.c_double(min_opacity), ctypes.c_double(max_scale), ctypes.byref(om),
                                _ptr(state_src), _ptr(n_out), _stream(stream)))
    return out, state_src, n_out


def gather_rows(ctx, src, row_map, n_rows, dst=None, n_rows_dev=None, stream=None):
    """as_gather_rows: dst row r = src row map[r] (zeros for -1); n_rows_dev:
    optional device count of the rows to write (n_rows then a capacity)."""
    if dst is None:
        dst = Gaussians.empty(max(n_rows, 1), src.sh_degree)
    ss = src.struct()
    dm = _GaussiansMut.of(dst)
    _check(lib().as_gather_rows(ctx.handle, ctypes.byref(ss), _ptr(row_map) if n_rows else None,
                                ctypes.c_int64(n_rows), ctypes.byref(dm), _ptr(n_rows_dev), _stream(stream)))
    return dst


def reset_opacity(ctx, g, max_opacity, m_op=None, v_op=None, stream=None):
    """as_reset_opacity: in place."""
    gm = _GaussiansMut.of(g)
    _check(lib().as_reset_opacity(ctx.handle, ctypes.byref(gm), ctypes.c_double(max_opacity), _ptr(m_op), _ptr(v_op),
                                  _stream(stream)))


class _Tuning(ctypes.Structure):
    _fields_ = [("lds_batch", ctypes.c_int32), ("longest_first", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("radix_bits", ctypes.c_int32), ("block_cull", ctypes.c_int32), ("single_pass_sort", ctypes.c_int32),
                ("bin_tile", ctypes.c_int32)]


def set_tuning(ctx, lds_batch=256, longest_first=True, persistent=False, radix_bits=8, block_cull=True,
               single_pass_sort=0, bin_tile=16):
    """as_set_tuning (single_pass_sort: bit 0 the depth sort, bit 1 the pair
    sort take one launch per digit; bin_tile: 16 or 32 pixel squares for
    the pair binning)."""
    t = _Tuning(lds_batch, 1 if longest_first else 0, 1 if persistent else 0, radix_bits, 1 if block_cull else 0,
                int(single_pass_sort), int(bin_tile))
    _check(lib().as_set_tuning(ctx.handle, ctypes.byref(t)))


def get_tuning(ctx):
    t = _Tuning()
    _check(lib().as_get_tuning(ctx.handle, ctypes.byref(t)))
    return dict(lds_batch=t.lds_batch, longest_first=bool(t.longest_first), persistent=bool(t.persistent),
                radix_bits=t.radix_bits, block_cull=bool(t.block_cull), single_pass_sort=t.single_pass_sort,
                bin_tile=t.bin_tile)


def timing_enable(ctx, on=True):
    _check(lib().as_timing_enable(ctx.handle, ctypes.c_int32(1 if on else 0)))


def timing_read(ctx):
    """{stage: (total ms, runs)} since the last read."""
    ms = (ctypes.c_double * len(STAGES))()
    runs = (ctypes.c_int64 * len(STAGES))()
    _check(lib().as_timing_read(ctx.handle, ms, runs))
    return {name: (ms[k], runs[k]) for k, name in enumerate(STAGES)}


def debug_sort_pairs(ctx, keys, vals, key_bits, stream=None):
    _check(lib().as_debug_sort_pairs(ctx.handle, _ptr(keys), _ptr(vals), ctypes.c_int64(keys.shape[0]),
                                     ctypes.c_int32(key_bits), _stream(stream)))


def debug_sort_u32(ctx, keys, vals, lo_bit, hi_bit, radix_bits=8, single_pass=True, gather_src=None,
                   gather_dst=None, stream=None):
    """as_debug_sort_u32 (in place; int32 tensors holding the u32 bits)."""
    _check(lib().as_debug_sort_u32(ctx.handle, _ptr(keys), _ptr(vals), ctypes.c_int64(keys.numel()),
                                   ctypes.c_int32(lo_bit), ctypes.c_int32(hi_bit), ctypes.c_int32(radix_bits),
                                   ctypes.c_int32(1 if single_pass else 0), _ptr(gather_src), _ptr(gather_dst),
                                   _stream(stream)))


def debug_fp64_ops(ctx, a, b, stream=None):
    out = torch.empty(4, a.shape[0], dtype=torch.float64, device="cuda")
    _check(lib().as_debug_fp64_ops(ctx.handle, _ptr(a), _ptr(b), ctypes.c_int64(a.shape[0]), _ptr(out),
                                   _stream(stream)))
    return out


def debug_row_addressing(ctx, force_64bit):
    """as_debug_row_addressing: SH rows by 64-bit addresses (True) or the
    default buffer addressing (False) in the context's projection kernels."""
    _check(lib().as_debug_row_addressing(ctx.handle, ctypes.c_int32(1 if force_64bit else 0)))


def debug_blend_alpha(frame, pix, gauss, stream=None):
    """as_debug_blend_alpha: the blend's FP32 unclamped alpha o G for (pixel,
    Gaussian) pairs of the frame's last render (view 0).  pix: int32 [n, 2]
    (x, y); gauss: int32 [n] visible Gaussian ids.  Returns float32 [n]."""
    n = int(pix.shape[0])
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(lib().as_debug_blend_alpha(frame.handle, ctypes.c_int32(0), ctypes.c_int64(n), _ptr(pix), _ptr(gauss),
                                      _ptr(out), _stream(stream)))
    return out
