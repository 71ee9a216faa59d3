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
                ("sh_degree", ctypes.c_int32)]


class _SplitParams(ctypes.Structure):
    _fields_ = [("tau_l1", ctypes.c_double), ("r_erode", ctypes.c_int32), ("m_min", ctypes.c_int32),
                ("L", ctypes.c_int32), ("n_max", ctypes.c_int32), ("gamma_d", ctypes.c_double),
                ("gamma_c", ctypes.c_double), ("eps", ctypes.c_double), ("eta", ctypes.c_double)]


class _RegionBuf(ctypes.Structure):
    _fields_ = [("records", ctypes.c_void_p), ("capacity", ctypes.c_int64), ("count", ctypes.c_void_p)]


class _FrameView(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("n_cap", ctypes.c_int64), ("key_cap", ctypes.c_int64)] + [
        (nm, ctypes.c_void_p) for nm in ("n_keys", "keys", "vals", "ranges", "depth_key", "box", "ntiles", "rec",
                                         "t_final", "last", "n_contrib", "dom", "err", "err_minmax", "grad2d")]


REGION_DTYPE = np.dtype([
    ("cand", "<i4"), ("view", "<i4"), ("label", "<i4"), ("area", "<i4"), ("band", "<i4"), ("pad0", "<i4"),
    ("sx", "<i8"), ("sy", "<i8"), ("sxx", "<i8"), ("sxy", "<i8"), ("syy", "<i8"),
    ("cx", "<f8"), ("cy", "<f8"), ("cov", "<f8", (3,)), ("e1", "<f8", (2,)), ("sigma1", "<f8"), ("sigma2", "<f8"),
    ("rgb", "<f4", (3,)), ("pad1", "<f4")])
assert REGION_DTYPE.itemsize == 152

EXPORTED = ("as_ctx_create", "as_ctx_destroy", "as_last_error", "as_version", "as_frame_create", "as_frame_destroy",
            "as_frame_get_view", "as_render", "as_render_backward", "as_error_map", "as_accumulate_error_stats",
            "as_adaptive_split", "as_timing_enable", "as_timing_read", "as_debug_sort_pairs", "as_debug_fp64_ops")

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
            if name not in ("as_last_error", "as_version", "as_ctx_destroy", "as_frame_destroy"):
                getattr(L, name).restype = ctypes.c_int
        L.as_ctx_destroy.restype = None
        L.as_frame_destroy.restype = None
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


class SplitParams:
    """AdpSplit hyper-parameters; defaults from Sec. 5 (tau_l1 0.1, r_erode 2,
    m_min 5, L 3, N_max 19, gamma_d 2.0, gamma_c 0.15), eps 1e-8, eta 0.8."""

    def __init__(self, tau_l1=0.1, r_erode=2, m_min=5, L=3, n_max=19, gamma_d=2.0, gamma_c=0.15, eps=1e-8, eta=0.8):
        self.tau_l1, self.r_erode, self.m_min, self.L, self.n_max = tau_l1, r_erode, m_min, L, n_max
        self.gamma_d, self.gamma_c, self.eps, self.eta = gamma_d, gamma_c, eps, eta

    def struct(self):
        return _SplitParams(self.tau_l1, self.r_erode, self.m_min, self.L, self.n_max, self.gamma_d, self.gamma_c,
                            self.eps, self.eta)


class Gaussians:
    """Device-resident Gaussians (torch tensors in the library layout)."""

    FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree):
        self.means, self.log_scales, self.quats = means, log_scales, quats
        self.opacity_logits, self.sh, self.sh_degree = opacity_logits, sh, int(sh_degree)

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
                          _ptr(self.sh), self.n, self.sh_degree)

    def rows(self, n):
        """First n rows (views with the full row stride are not contiguous, so copy)."""
        return Gaussians(self.means[:, :n].contiguous(), self.log_scales[:, :n].contiguous(),
                         self.quats[:, :n].contiguous(), self.opacity_logits[:n].contiguous(),
                         self.sh[:, :, :n].contiguous(), self.sh_degree)


class Context:
    """An as_ctx bound to one device."""

    def __init__(self, device=0):
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().as_ctx_create(ctypes.c_int(device), ctypes.byref(h)))
        self.handle = h

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
    """Per-view rasterizer state (as_frame)."""

    def __init__(self, ctx, n_cap, width, height, key_cap=None, auto_grow=True):
        if key_cap is None:
            key_cap = max(1 << 16, 8 * n_cap)
        h = ctypes.c_void_p()
        _check(lib().as_frame_create(ctx.handle, ctypes.c_int64(n_cap), ctypes.c_int32(width), ctypes.c_int32(height),
                                     ctypes.c_int64(key_cap), ctypes.c_int32(1 if auto_grow else 0), ctypes.byref(h)))
        self.ctx, self.handle, self.width, self.height, self.n_cap = ctx, h, width, height, n_cap

    def view(self):
        v = _FrameView()
        _check(lib().as_frame_get_view(self.handle, ctypes.byref(v)))
        return v

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
        v = self.view()
        return int(self._dev(v.n_keys, 4).view(np.uint32)[0])

    def host_state(self, n):
        """Keys, values, ranges, per-Gaussian and per-pixel state as numpy arrays."""
        v = self.view()
        K = min(self.n_keys(), v.key_cap)
        P = self.width * self.height
        T = v.tiles_x * v.tiles_y
        return dict(
            n_keys=self.n_keys(), keys=self._dev(v.keys, 8 * K).view(np.uint64), vals=self._dev(v.vals, 4 * K).view(np.uint32),
            ranges=self._dev(v.ranges, 8 * T).view(np.uint32).reshape(T, 2),
            depth_key=self._dev(v.depth_key, 4 * n).view(np.uint32), box=self._dev(v.box, 8 * n).view(np.int16).reshape(n, 4),
            ntiles=self._dev(v.ntiles, 4 * n).view(np.uint32), rec=self._dev(v.rec, 48 * n).view(np.float32).reshape(n, 12),
            t_final=self._dev(v.t_final, 4 * P).view(np.float32).reshape(self.height, self.width),
            last=self._dev(v.last, 4 * P).view(np.uint32).reshape(self.height, self.width),
            n_contrib=self._dev(v.n_contrib, 4 * P).view(np.uint32).reshape(self.height, self.width),
            dom=self._dev(v.dom, 4 * P).view(np.int32).reshape(self.height, self.width),
            err=self._dev(v.err, 8 * P).view(np.float64).reshape(self.height, self.width),
            err_minmax=self._dev(v.err_minmax, 16).view(np.uint64),
            tiles_x=v.tiles_x, tiles_y=v.tiles_y)

    def device_maps(self):
        """Device addresses of the per-pixel maps (for accumulate_error_stats)."""
        v = self.view()
        return dict(err=v.err, err_minmax=v.err_minmax, dom=v.dom, t_final=v.t_final)


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
    _check(lib().as_render(ctx.handle, ctypes.byref(gs), ctypes.byref(c), frame.handle, _ptr(gt), _ptr(image),
                           _stream(stream)))
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


class _GaussiansMut(_Gaussians):
    @staticmethod
    def of(g):
        m = _GaussiansMut()
        m.means, m.log_scales, m.quats = _ptr(g.means), _ptr(g.log_scales), _ptr(g.quats)
        m.opacity_logits, m.sh = _ptr(g.opacity_logits), _ptr(g.sh)
        m.n, m.sh_degree = int(g.means.shape[1]), g.sh_degree
        return m


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


def adaptive_split(ctx, g, cand, regions, views, attr_count, params, noise, out=None, stream=None):
    """as_adaptive_split.  Returns (out Gaussians with capacity rows, mode,
    count, offset, n_out tensor)."""
    nc = int(cand.shape[0])
    if out is None:
        cap = g.n + nc * max(2, params.n_max + 1)
        out = Gaussians.empty(max(cap, 1), g.sh_degree)
    mode = torch.zeros(max(nc, 1), dtype=torch.uint8, device="cuda")
    count = torch.zeros(max(nc, 1), dtype=torch.int32, device="cuda")
    offset = torch.zeros(max(nc, 1), dtype=torch.int64, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    cams = (_Camera * max(len(views), 1))(*[camera_struct(v) for v in views])
    gs = g.struct()
    p = params.struct()
    rb = regions.struct()
    om = _GaussiansMut.of(out)
    _check(lib().as_adaptive_split(ctx.handle, ctypes.byref(gs), _ptr(cand) if nc else None, ctypes.c_int64(nc),
                                   ctypes.byref(rb), cams, ctypes.c_int32(len(views)), _ptr(attr_count), ctypes.byref(p),
                                   _ptr(noise) if nc else None, ctypes.byref(om), _ptr(mode) if nc else None,
                                   _ptr(count) if nc else None, _ptr(offset) if nc else None, _ptr(n_out),
                                   _stream(stream)))
    return out, mode[:nc], count[:nc], offset[:nc], n_out


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


def debug_fp64_ops(ctx, a, b, stream=None):
    out = torch.empty(4, a.shape[0], dtype=torch.float64, device="cuda")
    _check(lib().as_debug_fp64_ops(ctx.handle, _ptr(a), _ptr(b), ctypes.c_int64(a.shape[0]), _ptr(out),
                                   _stream(stream)))
    return out
