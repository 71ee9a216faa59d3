"""CPU FP64 oracle for the Gaussian rasterizer and the AdpSplit adaptive split.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call this package; the product path never does.  It shares no
code with the HIP path; both sides only receive the same seeded inputs.

The arithmetic lives in ``oracle.c`` (plain loops, FP64, built with
-ffp-contract=off).  This module only marshals numpy arrays through ctypes.

Scenes and cameras are duck-typed: a scene has ``means`` [3,n], ``log_scales``
[3,n], ``quats`` [4,n] (w,x,y,z), ``opacity_logits`` [n], ``sh`` [(d+1)^2,3,n]
(all float32) and ``sh_degree``; a camera has ``R`` (3x3 world->camera),
``t`` (3,), ``fx, fy, cx, cy, width, height`` and ``bg`` (3,).

Parity status per function (what pins it, see tests/test_oracle_*.py):
  project                 pinned (closed forms, FD Jacobian, brute-force box)
  bin                     pinned (brute-force enumeration + independent sort)
  render_pixels           pinned (single-Gaussian closed form, two-layer closed
                          form, invariants on transmittance and weights)
  render_backward_pixels  pinned (central finite differences in FP64)
  project_backward        pinned (central finite differences in FP64)
  error_stats             pinned (hand-built maps, brute-force counts, BFS
                          against scipy.ndimage labelling, rectangle moments)
  adaptive_split          pinned per stage (closed-form t*, axis-aligned child
                          shape, merge identities, closed-form merged mean,
                          colour, axes and scales of Eq. (merge_cov) via
                          merge_group, hand-built mode counts);
                          whole-method fidelity to the authors' unreleased
                          code is "parity unpinned" (no code or worked example
                          exists to compare against)
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

REGION_DTYPE = np.dtype(
    [
        ("cand", "<i4"), ("view", "<i4"), ("label", "<i4"), ("area", "<i4"), ("band", "<i4"),
        ("sx", "<i8"), ("sy", "<i8"), ("sxx", "<i8"), ("sxy", "<i8"), ("syy", "<i8"),
        ("cx", "<f8"), ("cy", "<f8"), ("cov", "<f8", (3,)), ("e1", "<f8", (2,)),
        ("sigma1", "<f8"), ("sigma2", "<f8"), ("rgb", "<f8", (3,)),
    ],
    align=True,
)

MODE_VANILLA, MODE_RESET, MODE_ADAPTIVE = 0, 1, 2


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_bin.restype = ctypes.c_int64
        L.orc_error_stats.restype = ctypes.c_int64
        L.orc_adaptive_split.restype = ctypes.c_int64
        L.orc_region_size.restype = ctypes.c_int64
        L.orc_child_proposal.restype = ctypes.c_int
        assert L.orc_region_size() == REGION_DTYPE.itemsize, "oracle region layout mismatch"
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def pack_camera(cam):
    """21 doubles: R[9], t[3], fx, fy, cx, cy, W, H, bg[3] (float32 values widened)."""
    R = np.asarray(cam.R, dtype=np.float32).reshape(9).astype(np.float64)
    t = np.asarray(cam.t, dtype=np.float32).reshape(3).astype(np.float64)
    intr = np.array([cam.fx, cam.fy, cam.cx, cam.cy], dtype=np.float32).astype(np.float64)
    bg = np.asarray(cam.bg, dtype=np.float32).reshape(3).astype(np.float64)
    return np.concatenate([R, t, intr, np.array([cam.width, cam.height], np.float64), bg])


def _scene_arrays(sc):
    return (_c(sc.means, np.float32), _c(sc.log_scales, np.float32), _c(sc.quats, np.float32),
            _c(sc.opacity_logits, np.float32), _c(sc.sh, np.float32))


class Projected:
    """Per-Gaussian projection rows (FP64) of one view."""

    def __init__(self, n):
        self.n = n
        self.valid = np.zeros(n, np.int32)
        self.mean2d = np.zeros((n, 2))
        self.cov2d = np.zeros((n, 3))
        self.conic = np.zeros((n, 3))
        self.rgb = np.zeros((n, 3))
        self.opacity = np.zeros(n)
        self.tview = np.zeros((n, 3))
        self.depth_key = np.zeros(n, np.uint32)
        self.box = np.zeros((n, 4), np.int32)
        # culling / box-edge decisions within transcendental rounding of a threshold
        self.box_flag = np.zeros(n, np.uint8)


def project(scene, cam):
    """Sec. 3 projection: EWA covariance, conic, mean, colour, depth key, box."""
    n = scene.means.shape[1]
    m, s, q, o, sh = _scene_arrays(scene)
    pr = Projected(n)
    pc = pack_camera(cam)
    lib().orc_project(ctypes.c_int64(n), ctypes.c_int(scene.sh_degree), _p(m), _p(s), _p(q), _p(o), _p(sh),
                      _p(pc), _p(pr.valid), _p(pr.mean2d), _p(pr.cov2d), _p(pr.conic), _p(pr.rgb),
                      _p(pr.opacity), _p(pr.tview), _p(pr.depth_key), _p(pr.box), _p(pr.box_flag))
    pr.width, pr.height = int(cam.width), int(cam.height)
    pr.bg = np.asarray(cam.bg, np.float32).astype(np.float64)
    return pr


def bin_tiles(pr, tile_w=16, tile_h=16):
    """Brute-force (tile | depth) keys, their stable sort and per-tile ranges."""
    n = pr.n
    cap = 0
    v = pr.valid.astype(bool)
    b = pr.box[v]
    cap = int((((b[:, 2] // tile_w) - (b[:, 0] // tile_w) + 1) * ((b[:, 3] // tile_h) - (b[:, 1] // tile_h) + 1)).sum())
    keys = np.zeros(max(cap, 1), np.uint64)
    vals = np.zeros(max(cap, 1), np.uint32)
    ntx = (pr.width + tile_w - 1) // tile_w
    nty = (pr.height + tile_h - 1) // tile_h
    ranges = np.zeros((ntx * nty, 2), np.uint32)
    K = lib().orc_bin(ctypes.c_int64(n), _p(pr.valid), _p(pr.box), _p(pr.depth_key), ctypes.c_int(pr.width),
                      ctypes.c_int(pr.height), ctypes.c_int(tile_w), ctypes.c_int(tile_h), _p(keys), _p(vals),
                      _p(ranges), ctypes.c_int64(cap))
    assert K == cap
    return keys[:K], vals[:K], ranges


def all_pixels(width, height):
    ys, xs = np.mgrid[0:height, 0:width]
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)


def render_pixels(pr, pix):
    """Eq. (rendering) + Eq. (dominant-map) at the listed pixels [npix, 2] (x, y)."""
    pix = _c(pix, np.int32)
    npix = pix.shape[0]
    out = dict(color=np.zeros((npix, 3)), T=np.zeros(npix), ncontrib=np.zeros(npix, np.int32),
               dom=np.zeros(npix, np.int64), last=np.zeros(npix, np.int64), flag=np.zeros(npix, np.uint8),
               pairs=np.zeros(npix, np.int64))
    lib().orc_render_pixels(ctypes.c_int64(pr.n), _p(pr.valid), _p(pr.mean2d), _p(pr.conic), _p(pr.rgb),
                            _p(pr.opacity), _p(pr.depth_key), _p(pr.box), _p(_c(pr.bg, np.float64)),
                            ctypes.c_int64(npix), _p(pix), _p(out["color"]), _p(out["T"]), _p(out["ncontrib"]),
                            _p(out["dom"]), _p(out["last"]), _p(out["flag"]), _p(out["pairs"]))
    return out


def alpha_pairs(pr, pix, ids, with_bound=False):
    """Unclamped alpha o G (FP64) of Gaussian ids[k] at pixel pix[k] = (x, y);
    with_bound=True also returns the relative error bound the near-threshold
    flags assume for the blend's FP32 evaluation of that alpha."""
    pix = _c(pix, np.int32)
    ids = _c(ids, np.int64)
    out = np.zeros(len(ids))
    bound = np.zeros(len(ids)) if with_bound else None
    lib().orc_alpha_pairs(_p(pr.mean2d), _p(pr.conic), _p(pr.opacity), ctypes.c_int64(len(ids)), _p(pix), _p(ids),
                          _p(out), _p(bound) if with_bound else None)
    return (out, bound) if with_bound else out


def render_image(pr):
    """Full image: colour [3,H,W] and per-pixel maps [H,W]."""
    W, H = pr.width, pr.height
    r = render_pixels(pr, all_pixels(W, H))
    img = r["color"].reshape(H, W, 3).transpose(2, 0, 1).copy()
    maps = {k: r[k].reshape(H, W) for k in ("T", "ncontrib", "dom", "last", "flag", "pairs")}
    return img, maps


def render_backward_pixels(pr, pix, dL_dcolor):
    """Reverse pass of Eq. (rendering): per-Gaussian gradients of the 2D rows."""
    pix = _c(pix, np.int32)
    npix = pix.shape[0]
    g = _c(dL_dcolor, np.float64).reshape(npix, 3)
    n = pr.n
    out = dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), opacity=np.zeros(n), rgb=np.zeros((n, 3)))
    lib().orc_render_backward_pixels(ctypes.c_int64(n), _p(pr.valid), _p(pr.mean2d), _p(pr.conic), _p(pr.rgb),
                                     _p(pr.opacity), _p(pr.depth_key), _p(pr.box), _p(_c(pr.bg, np.float64)),
                                     ctypes.c_int64(npix), _p(pix), _p(g), _p(out["mean2d"]), _p(out["conic"]),
                                     _p(out["opacity"]), _p(out["rgb"]))
    return out


def project_backward(scene, cam, g2d):
    """Chain rule from the 2D gradients to the stored parameters (SoA layout)."""
    n = scene.means.shape[1]
    m, s, q, o, sh = _scene_arrays(scene)
    nk = (scene.sh_degree + 1) ** 2
    out = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
               opacity_logits=np.zeros(n), sh=np.zeros((nk, 3, n)))
    pc = pack_camera(cam)
    lib().orc_project_backward(ctypes.c_int64(n), ctypes.c_int(scene.sh_degree), _p(m), _p(s), _p(q), _p(o),
                               _p(sh), _p(pc), _p(_c(g2d["mean2d"], np.float64)), _p(_c(g2d["conic"], np.float64)),
                               _p(_c(g2d["opacity"], np.float64)), _p(_c(g2d["rgb"], np.float64)),
                               _p(out["means"]), _p(out["log_scales"]), _p(out["quats"]),
                               _p(out["opacity_logits"]), _p(out["sh"]))
    return out


VARIANT_ADPSPLIT, VARIANT_FIXED_N, VARIANT_ADAPTIVE_N, VARIANT_CHILD_INIT = 0, 1, 2, 3
FLAG_ERODE_SIDE, FLAG_CROSS_VIEW, FLAG_EXTENT_MAX, FLAG_SHARE_OPACITY = 1, 2, 4, 8


class SplitParams:
    """Sec. 5 defaults: tau_l1 0.1, r_erode 2, m_min 5, L 3, N_max 19,
    gamma_d 2.0, gamma_c 0.15; eps 1e-8 [A15]; eta 0.8 [A24].  variant: the
    full method (0) or a step of the Table 2 ablation / the fixed-N random
    split (1 fixed N, 2 adaptive N with random placement, 3 child
    initialisation without merging); flags: alternative readings (1 erosion
    square of side r+1 [A11], 2 cross-view merging only [A18], 4 extent =
    largest scale [A22], 8 shared opacity o/(N+1) [A23]); noise_n: normals
    per candidate in the noise input (0 = 2)."""

    def __init__(self, tau_l1=0.1, r_erode=2, m_min=5, L=3, n_max=19, gamma_d=2.0, gamma_c=0.15, eps=1e-8,
                 eta=0.8, variant=0, flags=0, fixed_n=2, noise_n=0):
        self.tau_l1, self.r_erode, self.m_min, self.L, self.n_max = tau_l1, r_erode, m_min, L, n_max
        self.gamma_d, self.gamma_c, self.eps, self.eta = gamma_d, gamma_c, eps, eta
        self.variant, self.flags, self.fixed_n, self.noise_n = variant, flags, fixed_n, noise_n


def error_stats(img, gt, dom, is_cand, view, params, attr, cap=None, want_maps=False):
    """Sec. 4.1 for one view.  img, gt: [3,H,W] float32; dom: [H,W] int32;
    is_cand: [n] uint8; attr: [n] int32, accumulated in place.
    Returns (regions structured array, maps dict or None)."""
    img = _c(img, np.float32)
    gt = _c(gt, np.float32)
    dom = _c(dom, np.int32)
    is_cand = _c(is_cand, np.uint8)
    assert attr.dtype == np.int32 and attr.flags.c_contiguous
    H, W = dom.shape
    P = H * W
    if cap is None:
        cap = P // max(params.m_min, 1) + 1
    regs = np.zeros(cap, REGION_DTYPE)
    maps = None
    ptrs = [None] * 5
    if want_maps:
        maps = dict(E=np.zeros((H, W)), M=np.zeros((H, W), np.uint8), Mp=np.zeros((H, W), np.uint8),
                    B=np.zeros((H, W), np.uint8), label=np.zeros((H, W), np.int32))
        ptrs = [_p(maps[k]) for k in ("E", "M", "Mp", "B", "label")]
    r = lib().orc_error_stats(ctypes.c_int(W), ctypes.c_int(H), _p(img), _p(gt), _p(dom),
                              ctypes.c_int64(is_cand.shape[0]), _p(is_cand), ctypes.c_int(view),
                              ctypes.c_double(params.tau_l1), ctypes.c_int(params.r_erode),
                              ctypes.c_int(params.m_min), ctypes.c_int(params.L),
                              ctypes.c_int(1 if params.flags & FLAG_ERODE_SIDE else 0), _p(attr), _p(regs),
                              ctypes.c_int64(cap), *ptrs)
    if r < 0:
        raise RuntimeError("oracle region capacity exceeded: need %d" % (-r - 1))
    return regs[:r].copy(), maps


def adaptive_split(scene, cand, regions, cams, attr, params, noise, out_cap=None):
    """Sec. 4.2-4.3 and the implementation details of Sec. 5."""
    n = scene.means.shape[1]
    m, s, q, o, sh = _scene_arrays(scene)
    cand = _c(cand, np.int32)
    nc = cand.shape[0]
    regions = np.ascontiguousarray(regions, dtype=REGION_DTYPE)
    camp = np.ascontiguousarray(np.stack([pack_camera(c) for c in cams]) if len(cams) else np.zeros((1, 21)))
    attr = _c(attr, np.int32)
    nz = params.noise_n if params.noise_n > 0 else 2
    noise = _c(noise, np.float32).reshape(nc * nz * 3) if nc else np.zeros(3 * nz, np.float32)
    prm = np.array([params.gamma_d, params.gamma_c, params.eps, params.eta, params.n_max, params.variant,
                    params.flags, params.fixed_n, params.noise_n], np.float64)
    nk = (scene.sh_degree + 1) ** 2
    if out_cap is None:
        out_cap = n + nc * max(2, params.n_max + 1, params.fixed_n if params.variant == VARIANT_FIXED_N else 0)
    mode = np.zeros(max(nc, 1), np.uint8)
    count = np.zeros(max(nc, 1), np.int32)
    offset = np.zeros(max(nc, 1), np.int64)
    om = np.zeros((3, out_cap), np.float32)
    osc = np.zeros((3, out_cap), np.float32)
    oq = np.zeros((4, out_cap), np.float32)
    oo = np.zeros(out_cap, np.float32)
    osh = np.zeros((nk, 3, out_cap), np.float32)
    nout = lib().orc_adaptive_split(ctypes.c_int64(n), ctypes.c_int(scene.sh_degree), _p(m), _p(s), _p(q), _p(o),
                                    _p(sh), _p(cand), ctypes.c_int64(nc), _p(regions),
                                    ctypes.c_int64(regions.shape[0]), _p(camp), ctypes.c_int(len(cams)), _p(attr),
                                    _p(prm), _p(noise), _p(mode), _p(count), _p(offset), _p(om), _p(osc), _p(oq),
                                    _p(oo), _p(osh), ctypes.c_int64(out_cap))
    if nout < 0:
        raise RuntimeError("oracle split output capacity exceeded: need %d" % (-nout - 1))
    return dict(mode=mode[:nc], count=count[:nc], offset=offset[:nc], n_out=int(nout),
                means=om[:, :nout], log_scales=osc[:, :nout], quats=oq[:, :nout], opacity_logits=oo[:nout],
                sh=osh[:, :, :nout])


def sh_basis(x, y, z):
    Y = np.zeros(16)
    lib().orc_sh_basis(ctypes.c_double(x), ctypes.c_double(y), ctypes.c_double(z), _p(Y))
    return Y


def jacobi3(A):
    A = _c(A, np.float64).reshape(9)
    V = np.zeros(9)
    lam = np.zeros(3)
    lib().orc_jacobi3(_p(A), _p(V), _p(lam))
    return V.reshape(3, 3), lam


def merge_group(mu, R, s, rgb):
    """Eq. (merge_cov) for M proposals given directly: mu [M,3], R [M,3,3],
    s [M,3], rgb [M,3].  Returns (mean, colour, E [3,3] with the axes as
    columns, scales sqrt(lambda) [3]); the split merges with the same code."""
    mu = _c(mu, np.float64).reshape(-1, 3)
    M = mu.shape[0]
    R = _c(R, np.float64).reshape(M, 9)
    s = _c(s, np.float64).reshape(M, 3)
    rgb = _c(rgb, np.float64).reshape(M, 3)
    mo, co, Ro, so = np.zeros(3), np.zeros(3), np.zeros(9), np.zeros(3)
    lib().orc_merge_group(ctypes.c_int64(M), _p(mu), _p(R), _p(s), _p(rgb), _p(mo), _p(co), _p(Ro), _p(so))
    return mo, co, Ro.reshape(3, 3), so


def child_proposal(parent, region, cam, eps=1e-8):
    """Child (mu, R, s) of one region for a single-Gaussian parent scene."""
    m, s, q, o, _ = _scene_arrays(parent)
    reg = np.ascontiguousarray(np.asarray(region, dtype=REGION_DTYPE).reshape(1))
    mu = np.zeros(3)
    R = np.zeros(9)
    sc = np.zeros(3)
    ok = lib().orc_child_proposal(_p(m), _p(s), _p(q), _p(o), _p(reg), _p(pack_camera(cam)), ctypes.c_double(eps),
                                  _p(mu), _p(R), _p(sc))
    return bool(ok), mu, R.reshape(3, 3), sc


def render_rows(pr, y0=0, y1=None, dL_dcolor=None, margins=False, grad_abs=False):
    """Eq. (rendering) for every pixel of rows [y0, y1) (same arithmetic as
    render_pixels, gathered per row).  With dL_dcolor [(y1-y0)*W, 3] the
    reverse pass runs too and the 2D gradients are returned under "grad".

    margins=True adds "margins" [npix, 4]: for each decision (alpha vs 1/255,
    T(1 - alpha) vs 1e-4, the dominant weight's lead over the runner-up, o G
    vs the 0.99 clamp) the smallest ratio of its relative distance to the
    threshold over its FP32 error bound plus 1e-6 (inf where the decision
    never arises); the pixel is flagged when any ratio is at most 1.  It also
    adds "t_bound" [npix]: the relative error bound those flags assume for an
    FP32 evaluation of the final transmittance.  grad_abs=True (with dL_dcolor) adds
    grad["abs"] [n, 9]: per Gaussian the summed magnitudes of the products
    that make up each 2D gradient (mean x, y; conic a, b, c; opacity; colour
    r, g, b), the scale of its floating-point rounding error."""
    W = pr.width
    y1 = pr.height if y1 is None else y1
    npix = (y1 - y0) * W
    out = dict(color=np.zeros((npix, 3)), T=np.zeros(npix), ncontrib=np.zeros(npix, np.int32),
               dom=np.zeros(npix, np.int64), last=np.zeros(npix, np.int64), flag=np.zeros(npix, np.uint8),
               pairs=np.zeros(npix, np.int64))
    n = pr.n
    gp = [None] * 4
    gC = None
    if dL_dcolor is not None:
        gC = _c(dL_dcolor, np.float64).reshape(npix, 3)
        out["grad"] = dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), opacity=np.zeros(n), rgb=np.zeros((n, 3)))
        gp = [_p(out["grad"][k]) for k in ("mean2d", "conic", "opacity", "rgb")]
    mp = ga = tb = None
    if margins:
        out["margins"] = np.zeros((npix, 4))
        out["t_bound"] = np.zeros(npix)
        mp = _p(out["margins"])
        tb = _p(out["t_bound"])
    if grad_abs:
        assert dL_dcolor is not None, "grad_abs needs dL_dcolor"
        out["grad"]["abs"] = np.zeros((n, 9))
        ga = _p(out["grad"]["abs"])
    lib().orc_render_rows(ctypes.c_int64(n), _p(pr.valid), _p(pr.mean2d), _p(pr.conic), _p(pr.rgb), _p(pr.opacity),
                          _p(pr.depth_key), _p(pr.box), _p(_c(pr.bg, np.float64)), ctypes.c_int(W), ctypes.c_int(y0),
                          ctypes.c_int(y1), _p(out["color"]), _p(out["T"]), _p(out["ncontrib"]), _p(out["dom"]),
                          _p(out["last"]), _p(out["flag"]), _p(out["pairs"]), _p(gC) if gC is not None else None,
                          *gp, mp, ga, tb)
    return out
