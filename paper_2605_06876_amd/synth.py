"""Seeded synthetic inputs: scenes, cameras, target images, error-map fixtures.

This module draws random numbers and builds camera poses; it holds none of the
rasterizer's or the split's arithmetic, so both the HIP path and the CPU
oracle can be fed from it.  The paper's datasets (MipNeRF360, Deep-Blending,
Tanks&Temples) are not available; these generators stand in for them with
the shapes the benchmark configurations name.
"""
import math

import numpy as np


class Camera:
    """Pinhole camera.  ``R`` (3x3, float32) maps world to camera coordinates
    with x right, y down, z forward; ``t`` is the translation
    (x_cam = R x_world + t).  Intrinsics in pixels; ``bg`` is the background."""

    def __init__(self, R, t, fx, fy, cx, cy, width, height, bg=(0.0, 0.0, 0.0)):
        self.R = np.asarray(R, np.float32).reshape(3, 3)
        self.t = np.asarray(t, np.float32).reshape(3)
        self.fx, self.fy, self.cx, self.cy = float(np.float32(fx)), float(np.float32(fy)), float(np.float32(cx)), float(np.float32(cy))
        self.width, self.height = int(width), int(height)
        self.bg = np.asarray(bg, np.float32).reshape(3)

    def __repr__(self):
        return "Camera(%dx%d, f=%.2f)" % (self.width, self.height, self.fx)


class Scene:
    """Gaussians in struct-of-arrays float32 layout.

    means [3,n], log_scales [3,n], quats [4,n] (w,x,y,z, not necessarily
    normalised), opacity_logits [n], sh [(deg+1)^2, 3, n]."""

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree):
        self.means = np.ascontiguousarray(means, np.float32)
        self.log_scales = np.ascontiguousarray(log_scales, np.float32)
        self.quats = np.ascontiguousarray(quats, np.float32)
        self.opacity_logits = np.ascontiguousarray(opacity_logits, np.float32)
        self.sh = np.ascontiguousarray(sh, np.float32)
        self.sh_degree = int(sh_degree)

    @property
    def n(self):
        return self.means.shape[1]

    def subset(self, idx):
        idx = np.asarray(idx)
        return Scene(self.means[:, idx], self.log_scales[:, idx], self.quats[:, idx], self.opacity_logits[idx],
                     self.sh[:, :, idx], self.sh_degree)

    def nbytes(self):
        return sum(a.nbytes for a in (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh))


def look_at(eye, target, width, height, fov_x_deg=60.0, down=(0.0, 1.0, 0.0), bg=(0.0, 0.0, 0.0)):
    """Camera at ``eye`` looking at ``target``; ``down`` is the world vector
    that should appear pointing down the image.  Horizontal field of view."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    d = np.asarray(down, np.float64)
    r = np.cross(d, f)
    if np.linalg.norm(r) < 1e-6:
        r = np.cross(np.array([0.0, 0.0, 1.0]), f)
    r /= np.linalg.norm(r)
    dn = np.cross(f, r)
    R = np.stack([r, dn, f])
    t = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R, t, fx, fx, width / 2.0, height / 2.0, width, height, bg)


def sphere_cameras(k, radius, sizes, seed=0, fov_x_deg=60.0):
    """k cameras on a sphere (Fibonacci points) looking at the origin, world
    up = -y.  ``sizes`` is a list of (W, H), cycled."""
    rng = np.random.default_rng(seed)
    golden = math.pi * (3.0 - math.sqrt(5.0))
    off = rng.uniform(0, 2 * math.pi)
    cams = []
    for i in range(k):
        y = 1.0 - 2.0 * (i + 0.5) / k
        rr = math.sqrt(max(0.0, 1.0 - y * y))
        th = golden * i + off
        eye = radius * np.array([math.cos(th) * rr, y, math.sin(th) * rr])
        W, H = sizes[i % len(sizes)]
        cams.append(look_at(eye, (0, 0, 0), W, H, fov_x_deg))
    return cams


def random_pose_camera(rng, radius, W, H, fov_x_deg=60.0):
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    return look_at(radius * v, (0, 0, 0), W, H, fov_x_deg)


def _random_quats(rng, n):
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def scene_uniform_sh0(n, seed, log_scale_mu=-3.5, log_scale_sd=0.5):
    """Means U[-1,1]^3; log-scales N(mu, sd); quaternions uniform on S^3;
    opacity logits N(0,1); SH degree 0 with colours U[0,1].  The DC
    coefficient is drawn directly over U(-sqrt(pi), sqrt(pi)), the range that
    the degree-0 basis maps onto colours [0, 1]."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(3, n))
    log_scales = rng.normal(log_scale_mu, log_scale_sd, size=(3, n))
    quats = _random_quats(rng, n)
    opac = rng.normal(0.0, 1.0, size=n)
    root_pi = math.sqrt(math.pi)
    sh = rng.uniform(-root_pi, root_pi, size=(1, 3, n))
    return Scene(means, log_scales, quats, opac, sh, 0)


def scene_clusters(n, seed, sh_degree=3, n_clusters=64, background=0.10, log_scale_mu=-4.5, log_scale_sd=0.8):
    """Mixture of anisotropic clusters plus a uniform background: cluster
    centres U[-0.8,0.8]^3, per-axis std U(0.03,0.25), random rotation, equal
    weights; background U[-1,1]^3.  Log-scales N(mu, sd); quaternions uniform
    on S^3; opacity logits N(0,1); DC coefficients U(0,1); higher-order
    coefficients N(0, 0.1)."""
    rng = np.random.default_rng(seed)
    nb = int(round(n * background))
    nc = n - nb
    centres = rng.uniform(-0.8, 0.8, size=(n_clusters, 3))
    stds = rng.uniform(0.03, 0.25, size=(n_clusters, 3))
    rots = []
    for _ in range(n_clusters):
        Q, Rr = np.linalg.qr(rng.normal(size=(3, 3)))
        rots.append(Q * np.sign(np.diag(Rr)))
    lab = rng.integers(0, n_clusters, size=nc)
    local = rng.normal(size=(nc, 3)) * stds[lab]
    pts = np.einsum("nij,nj->ni", np.stack(rots)[lab], local) + centres[lab]
    bgp = rng.uniform(-1.0, 1.0, size=(nb, 3))
    means = np.concatenate([pts, bgp], axis=0).T
    perm = rng.permutation(n)
    means = means[:, perm]
    log_scales = rng.normal(log_scale_mu, log_scale_sd, size=(3, n))
    quats = _random_quats(rng, n)
    opac = rng.normal(0.0, 1.0, size=n)
    nk = (sh_degree + 1) ** 2
    sh = np.empty((nk, 3, n))
    sh[0] = rng.uniform(0.0, 1.0, size=(3, n))
    if nk > 1:
        sh[1:] = rng.normal(0.0, 0.1, size=(nk - 1, 3, n))
    return Scene(means, log_scales, quats, opac, sh, sh_degree)


def noise_image(H, W, seed):
    """Seeded uniform-noise RGB target [3,H,W]."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(3, H, W)).astype(np.float32)


def smooth_image(H, W, seed, cells=24, noise=0.02):
    """Spatially coherent RGB target [3,H,W] in [0,1]: a coarse random grid
    upsampled bilinearly, plus a little pixel noise."""
    rng = np.random.default_rng(seed)
    gh, gw = max(2, H // cells + 2), max(2, W // cells + 2)
    grid = rng.uniform(0.0, 1.0, size=(3, gh, gw))
    ys = np.linspace(0, gh - 1.001, H)
    xs = np.linspace(0, gw - 1.001, W)
    y0 = np.floor(ys).astype(int)
    x0 = np.floor(xs).astype(int)
    fy = (ys - y0)[:, None]
    fx = (xs - x0)[None, :]
    g00 = grid[:, y0][:, :, x0]
    g01 = grid[:, y0][:, :, x0 + 1]
    g10 = grid[:, y0 + 1][:, :, x0]
    g11 = grid[:, y0 + 1][:, :, x0 + 1]
    img = (g00 * (1 - fy) * (1 - fx) + g01 * (1 - fy) * fx + g10 * fy * (1 - fx) + g11 * fy * fx)
    img = img + rng.normal(0.0, noise, size=img.shape)
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def error_map_fixture(H, W, n, seed, n_sites=400, cand_frac=0.5, empty_frac=0.05, n_blobs=60):
    """Inputs for the error-statistics stage in isolation: a dominant map made
    of Voronoi cells (each cell one Gaussian id, some cells empty = -1), a
    candidate mask over n Gaussians, a smooth target and a rendered image that
    differs from it by noise plus a number of high-error blobs.
    Returns (img [3,H,W], gt [3,H,W], dom [H,W] int32, is_cand [n] uint8)."""
    rng = np.random.default_rng(seed)
    gt = smooth_image(H, W, seed + 7)
    sx = rng.uniform(0, W, n_sites)
    sy = rng.uniform(0, H, n_sites)
    ids = rng.integers(0, n, size=n_sites).astype(np.int32)
    ids[rng.uniform(size=n_sites) < empty_frac] = -1
    yy, xx = np.mgrid[0:H, 0:W]
    best = np.full((H, W), np.inf)
    dom = np.full((H, W), -1, np.int32)
    for k in range(n_sites):
        d = (xx - sx[k]) ** 2 + (yy - sy[k]) ** 2
        m = d < best
        best[m] = d[m]
        dom[m] = ids[k]
    is_cand = (rng.uniform(size=n) < cand_frac).astype(np.uint8)
    err = rng.normal(0.0, 0.03, size=(3, H, W))
    for _ in range(n_blobs):
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        rx, ry = rng.uniform(1.5, 12.0), rng.uniform(1.5, 12.0)
        amp = rng.uniform(0.2, 1.0) * rng.choice([-1.0, 1.0], size=(3, 1, 1))
        prof = np.exp(-0.5 * (((xx - cx) / rx) ** 2 + ((yy - cy) / ry) ** 2))
        err = err + amp * prof[None]
    img = (gt + err).astype(np.float32)
    return img, gt, dom, is_cand


def vanilla_noise(n_cand, seed, per=2):
    """Standard normals for the random children of the split, [n_cand, per, 3]."""
    return np.random.default_rng(seed).normal(size=(n_cand, per, 3)).astype(np.float32)


def c1_inputs(seed=1001):
    """2,000 Gaussians, SH degree 0, one 128x128 view at z=-4, fov 60 deg,
    uniform-noise target."""
    scene = scene_uniform_sh0(2000, seed)
    cam = look_at((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), 128, 128, 60.0)
    gt = noise_image(128, 128, seed + 1)
    return scene, cam, gt


def c2_inputs(seed=1002, n=1_000_000):
    """1,000,000 clustered Gaussians, SH degree 3, one 1256x828 view at z=-4,
    fov 60 deg, smooth synthetic target."""
    scene = scene_clusters(n, seed, 3)
    cam = look_at((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), 1256, 828, 60.0)
    gt = smooth_image(828, 1256, seed + 1)
    return scene, cam, gt
