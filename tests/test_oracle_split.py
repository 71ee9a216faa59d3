"""Pins of the CPU oracle's AdpSplit half (Sec. 4.1-4.3, App. A, Sec. 5
implementation details) against closed forms, library routines and brute
force (no GPU)."""
import math

import numpy as np
import pytest
from scipy import ndimage, optimize
from scipy.spatial.transform import Rotation

import oracle
from paper_2605_06876_amd import synth

P = oracle.SplitParams()


def maps_from_error(E, dom, n=None, cand=None):
    """Image/GT pair whose min-max normalised L1 error equals E (E in [0,1],
    min 0 and max 1 present): gt = 0, img channel 0 = E."""
    H, W = E.shape
    img = np.zeros((3, H, W), np.float32)
    img[0] = E.astype(np.float32)
    gt = np.zeros((3, H, W), np.float32)
    n = n if n is not None else int(dom.max()) + 1
    is_cand = np.ones(n, np.uint8) if cand is None else cand
    return img, gt, dom.astype(np.int32), is_cand


# ---- Eq. (l1map), metric map, attribution ----------------------------------------

def test_normalisation_and_attribution_brute_force():
    img, gt, dom, is_cand = synth.error_map_fixture(96, 128, 50, seed=5)
    attr = np.zeros(50, np.int32)
    regs, maps = oracle.error_stats(img, gt, dom, is_cand, 0, P, attr, want_maps=True)
    E = maps["E"]
    assert E.min() == 0.0 and E.max() == 1.0
    e = np.abs(img.astype(np.float64) - gt.astype(np.float64)).sum(0)
    np.testing.assert_allclose(E, (e - e.min()) / (e.max() - e.min()), rtol=1e-15, atol=1e-16)
    M = E > P.tau_l1
    np.testing.assert_array_equal(maps["M"], M)
    want = np.zeros(50, np.int64)
    for d in range(50):
        if is_cand[d]:
            want[d] = (M & (dom == d)).sum()
    np.testing.assert_array_equal(attr, want)


def test_constant_error_gives_no_high_error_pixels():
    dom = np.zeros((16, 16), np.int32)
    img = np.full((3, 16, 16), 0.5, np.float32)
    gt = np.zeros_like(img)
    attr = np.zeros(1, np.int32)
    regs, maps = oracle.error_stats(img, gt, dom, np.ones(1, np.uint8), 0, P, attr, want_maps=True)
    assert (maps["E"] == 0).all() and len(regs) == 0 and attr[0] == 0


# ---- erosion [A11] -----------------------------------------------------------------

@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_erosion_matches_scipy(r):
    img, gt, dom, is_cand = synth.error_map_fixture(64, 80, 20, seed=6)
    prm = oracle.SplitParams(r_erode=r)
    regs, maps = oracle.error_stats(img, gt, dom, is_cand, 0, prm, np.zeros(20, np.int32), want_maps=True)
    want = ndimage.binary_erosion(maps["M"].astype(bool), structure=np.ones((2 * r + 1, 2 * r + 1), bool),
                                  border_value=1) if r > 0 else maps["M"].astype(bool)
    np.testing.assert_array_equal(maps["Mp"].astype(bool), want)


def test_erosion_of_block():
    E = np.zeros((40, 50))
    E[10:22, 5:20] = 1.0
    img, gt, dom, is_cand = maps_from_error(E, np.zeros((40, 50), np.int32))
    regs, maps = oracle.error_stats(img, gt, dom, is_cand, 0, P, np.zeros(1, np.int32), want_maps=True)
    want = np.zeros((40, 50), bool)
    want[12:20, 7:18] = True
    np.testing.assert_array_equal(maps["Mp"].astype(bool), want)


# ---- bands [A10] --------------------------------------------------------------------

def test_bands_uniform_over_tau_to_one():
    E = np.linspace(0, 1, 1001).reshape(1, 1001)
    E = np.repeat(E, 3, axis=0)
    img, gt, dom, is_cand = maps_from_error(E, np.zeros(E.shape, np.int32))
    prm = oracle.SplitParams(r_erode=0, L=3)
    _, maps = oracle.error_stats(img, gt, dom, is_cand, 0, prm, np.zeros(1, np.int32), want_maps=True)
    Ev = maps["E"][1]
    B = maps["B"][1]
    hi = Ev > 0.1
    assert (B[~hi] == 0).all()
    b = B[hi]
    assert (np.diff(b.astype(int)) >= 0).all() and b[0] == 0 and b[-1] == 2
    # each band covers an equal share of (tau, 1]: the edges sit at 0.4 and 0.7
    first1 = Ev[hi][np.argmax(b == 1)]
    first2 = Ev[hi][np.argmax(b == 2)]
    assert abs(first1 - 0.4) <= 1e-3 and abs(first2 - 0.7) <= 1e-3


# ---- Eq. (error-region): 8-connected components on (D, B) -----------------------------

def test_regions_match_scipy_labelling_per_class():
    img, gt, dom, is_cand = synth.error_map_fixture(120, 160, 40, seed=8, n_blobs=120)
    prm = oracle.SplitParams(m_min=1)
    regs, maps = oracle.error_stats(img, gt, dom, is_cand, 3, prm, np.zeros(40, np.int32), want_maps=True)
    lab = maps["label"]
    active = maps["Mp"].astype(bool) & (dom >= 0) & (is_cand[np.maximum(dom, 0)] == 1)
    assert ((lab >= 0) == active).all()
    # partition equality against scipy, class by class
    n_comp = 0
    for d in np.unique(dom[active]):
        for b in np.unique(maps["B"][active & (dom == d)]):
            cls = active & (dom == d) & (maps["B"] == b)
            sl, k = ndimage.label(cls, structure=np.ones((3, 3)))
            n_comp += k
            for c in range(1, k + 1):
                pix = np.flatnonzero(sl == c)
                labels = lab.reshape(-1)[pix]
                assert (labels == labels[0]).all() and labels[0] == pix.min()
    assert n_comp == len(np.unique(lab[lab >= 0]))
    assert len(regs) == n_comp and (regs["view"] == 3).all()
    assert (np.diff(regs["label"]) > 0).all()


def test_diagonal_chain_is_one_region_and_band_splits():
    E = np.zeros((20, 20))
    for k in range(12):
        E[4 + k, 3 + k] = 1.0
    dom = np.zeros((20, 20), np.int32)
    img, gt, dom, is_cand = maps_from_error(E, dom)
    prm = oracle.SplitParams(r_erode=0, m_min=1)
    regs, _ = oracle.error_stats(img, gt, dom, is_cand, 0, prm, np.zeros(1, np.int32))
    assert len(regs) == 1 and regs["area"][0] == 12
    E2 = E.copy()
    E2[10:, :] *= 0.5   # second half of the chain drops to a lower band
    E2[0, 0] = 1.0      # keep the maximum at 1
    img, gt, dom, is_cand = maps_from_error(E2, np.zeros((20, 20), np.int32))
    regs, _ = oracle.error_stats(img, gt, dom, is_cand, 0, prm, np.zeros(1, np.int32))
    assert sorted(regs["area"].tolist()) == [1, 6, 6]


def test_k_separated_squares_and_min_area():
    E = np.zeros((60, 60))
    dom = np.zeros((60, 60), np.int32)
    for k in range(5):
        E[5 + 10 * k:8 + 10 * k, 5:8] = 1.0        # 3x3 = 9 px
        E[5 + 10 * k:7 + 10 * k, 30:32] = 1.0      # 2x2 = 4 px < m_min
    img, gt, dom, is_cand = maps_from_error(E, dom)
    prm = oracle.SplitParams(r_erode=0, m_min=5)
    regs, _ = oracle.error_stats(img, gt, dom, is_cand, 0, prm, np.zeros(1, np.int32))
    assert len(regs) == 5 and (regs["area"] == 9).all()


# ---- region statistics -------------------------------------------------------------------

@pytest.mark.parametrize("w,h", [(9, 5), (4, 11), (7, 7)])
def test_rectangle_statistics(w, h):
    E = np.zeros((40, 40))
    x0, y0 = 6, 13
    E[y0:y0 + h, x0:x0 + w] = 1.0
    img, gt, dom, is_cand = maps_from_error(E, np.zeros((40, 40), np.int32))
    gt[1] = np.arange(1600, dtype=np.float32).reshape(40, 40) / 1600
    img[1] = gt[1]   # keep the error map unchanged
    prm = oracle.SplitParams(r_erode=0, m_min=1)
    regs, _ = oracle.error_stats(img, gt, dom, is_cand, 0, prm, np.zeros(1, np.int32))
    r = regs[0]
    assert r["area"] == w * h
    np.testing.assert_allclose([r["cx"], r["cy"]], [x0 + w / 2, y0 + h / 2], rtol=1e-15)
    # exact second moment of a union of unit squares: w^2/12 and h^2/12
    np.testing.assert_allclose(r["cov"], [w * w / 12, 0.0, h * h / 12], rtol=1e-14, atol=1e-15)
    if w > h:
        np.testing.assert_allclose(r["e1"], [1, 0]); np.testing.assert_allclose([r["sigma1"], r["sigma2"]], [w / math.sqrt(12), h / math.sqrt(12)])
    elif h > w:
        np.testing.assert_allclose(r["e1"], [0, 1]); np.testing.assert_allclose([r["sigma1"], r["sigma2"]], [h / math.sqrt(12), w / math.sqrt(12)])
    else:
        np.testing.assert_allclose(r["e1"], [1, 0])
    gx, gy = int(math.floor(r["cx"])), int(math.floor(r["cy"]))
    assert r["rgb"][1] == np.float64(gt[1, gy, gx])


def test_pca_direction_matches_eigh():
    rng = np.random.default_rng(9)
    for _ in range(20):
        H = W = 64
        yy, xx = np.mgrid[0:H, 0:W]
        th = rng.uniform(0, np.pi)
        a, b = rng.uniform(3, 12), rng.uniform(1, 3)
        u = (xx - 32) * math.cos(th) + (yy - 32) * math.sin(th)
        v = -(xx - 32) * math.sin(th) + (yy - 32) * math.cos(th)
        E = ((u / a) ** 2 + (v / b) ** 2 <= 1).astype(float)
        E[0, 0] = 0
        img, gt, dom, is_cand = maps_from_error(E, np.zeros((H, W), np.int32))
        regs, _ = oracle.error_stats(img, gt, dom, is_cand, 0, oracle.SplitParams(r_erode=0, m_min=1),
                                     np.zeros(1, np.int32))
        r = regs[np.argmax(regs["area"])]
        ys, xs = np.nonzero(E > 0.5)
        C = np.cov(np.stack([xs, ys]), bias=True) + np.eye(2) / 12
        lam, V = np.linalg.eigh(C)
        v1 = V[:, 1] * np.sign(V[0, 1] if V[0, 1] != 0 else V[1, 1])
        np.testing.assert_allclose(r["e1"], v1, atol=1e-9)
        np.testing.assert_allclose([r["sigma1"], r["sigma2"]], np.sqrt(lam[::-1]), rtol=1e-9)


# ---- Sec. 4.2 / App. A: child centre and shape -----------------------------------------

def region_record(cand, view, label, cx, cy, e1, s1, s2, rgb, area=10):
    r = np.zeros(1, oracle.REGION_DTYPE)
    r["cand"], r["view"], r["label"], r["area"] = cand, view, label, area
    r["cx"], r["cy"] = cx, cy
    r["e1"] = e1
    r["sigma1"], r["sigma2"] = s1, s2
    r["rgb"] = rgb
    return r


def parent(mu, log_s, q=(1, 0, 0, 0), logit=0.5, deg=0):
    nk = (deg + 1) ** 2
    return synth.Scene(np.array(mu, np.float32).reshape(3, 1), np.array(log_s, np.float32).reshape(3, 1),
                       np.array(q, np.float32).reshape(4, 1), np.array([logit], np.float32),
                       np.zeros((nk, 3, 1), np.float32), deg)


def test_tstar_is_the_minimiser_of_the_mahalanobis_quadratic():
    """Eq. (tstar) against a numerical 1-D minimisation along the ray."""
    rng = np.random.default_rng(10)
    cam = synth.look_at((0.3, -0.2, -4.0), (0, 0, 0), 200, 160, 60.0)
    Rw = cam.R.astype(np.float64)
    ov = -Rw.T @ cam.t.astype(np.float64)
    for _ in range(20):
        mu = rng.uniform(-0.5, 0.5, 3)
        ls = rng.normal(-2.0, 0.6, 3)
        q = rng.normal(size=4)
        par = parent(mu, ls, q)
        cx, cy = rng.uniform(20, 180), rng.uniform(20, 140)
        reg = region_record(0, 0, 0, cx, cy, (1, 0), 3.0, 2.0, (0.5, 0.5, 0.5))
        ok, muc, R, s = oracle.child_proposal(par, reg, cam)
        dcam = np.array([(cx - cam.cx) / cam.fx, (cy - cam.cy) / cam.fy, 1.0])
        d = Rw.T @ dcam
        d /= np.linalg.norm(d)
        qd = par.quats[:, 0].astype(np.float64)
        Rg = Rotation.from_quat([qd[1], qd[2], qd[3], qd[0]]).as_matrix()
        A = Rg @ np.diag(np.exp(-2 * par.log_scales[:, 0].astype(np.float64))) @ Rg.T
        m = par.means[:, 0].astype(np.float64)
        f = lambda t: (ov + t * d - m) @ A @ (ov + t * d - m)
        t = optimize.minimize_scalar(f, bracket=(0.0, 10.0), tol=1e-14).x
        np.testing.assert_allclose(muc, ov + t * d, rtol=1e-6, atol=1e-7)


def test_isotropic_parent_gives_euclidean_closest_point_and_ray_through_mean():
    cam = synth.Camera(np.eye(3), (0, 0, 4), 100.0, 100.0, 64, 48, 128, 96)
    par = parent((0.2, -0.1, 0.5), [math.log(0.1)] * 3)
    m = par.means[:, 0].astype(np.float64)
    ov = np.array([0, 0, -4.0])
    cx, cy = 90.3, 30.7
    reg = region_record(0, 0, 0, cx, cy, (1, 0), 2.0, 1.0, (0.2, 0.3, 0.4))
    ok, muc, _, _ = oracle.child_proposal(par, reg, cam, eps=0.0)
    d = np.array([(cx - 64) / 100, (cy - 48) / 100, 1.0])
    d /= np.linalg.norm(d)
    want = ov + ((m - ov) @ d) * d
    np.testing.assert_allclose(muc, want, rtol=1e-12)
    # centroid exactly on the projection of the mean: the child sits on the mean
    t = m - ov
    cx2, cy2 = 100 * t[0] / t[2] + 64, 100 * t[1] / t[2] + 48
    reg2 = region_record(0, 0, 0, cx2, cy2, (1, 0), 2.0, 1.0, (0.2, 0.3, 0.4))
    ok, muc2, _, _ = oracle.child_proposal(par, reg2, cam, eps=0.0)
    np.testing.assert_allclose(muc2, m, rtol=1e-12, atol=1e-14)


def test_axis_aligned_child_shape():
    """Identity camera rotation, e1 = x: s1 = min(sigma1 t_z / f, s_max),
    s2 = s3 = min(sigma2 t_z / f, s_max), R = I."""
    f = 100.0
    cam = synth.Camera(np.eye(3), (0, 0, 4), f, f, 64, 48, 128, 96)
    par = parent((0.0, 0.0, 0.0), [math.log(0.2), math.log(0.05), math.log(0.1)])
    smax = math.exp(float(np.float32(math.log(0.2))))
    for s1, s2 in ((3.0, 1.5), (40.0, 2.0), (90.0, 70.0)):
        reg = region_record(0, 0, 0, 64.0, 48.0, (1, 0), s1, s2, (0.2, 0.3, 0.4))
        ok, muc, R, s = oracle.child_proposal(par, reg, cam, eps=0.0)
        tz = muc[2] + 4.0
        np.testing.assert_allclose(tz, 4.0, rtol=1e-12)
        np.testing.assert_allclose(s, [min(s1 * tz / f, smax), min(s2 * tz / f, smax), min(s2 * tz / f, smax)],
                                   rtol=1e-12)
        np.testing.assert_allclose(R, np.eye(3), atol=1e-15)


def test_child_rotation_is_proper_orthonormal():
    rng = np.random.default_rng(11)
    cam = synth.look_at((1.0, 2.0, -3.0), (0, 0, 0), 160, 120, 70.0)
    for _ in range(50):
        par = parent(rng.uniform(-0.3, 0.3, 3), rng.normal(-2, 0.5, 3), rng.normal(size=4))
        th = rng.uniform(0, 2 * np.pi)
        e1 = np.array([abs(math.cos(th)), math.sin(th)])
        reg = region_record(0, 0, 0, rng.uniform(10, 150), rng.uniform(10, 110), e1, rng.uniform(1, 9),
                            rng.uniform(0.3, 1.0), (0.5, 0.5, 0.5))
        ok, muc, R, s = oracle.child_proposal(par, reg, cam)
        if not ok:
            continue
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=2e-7)   # z_v is float32-rounded
        assert abs(np.linalg.det(R) - 1.0) < 1e-6
        assert s[1] == s[2] and s[0] > 0


def test_jacobi_against_eigh():
    rng = np.random.default_rng(12)
    for _ in range(100):
        X = rng.normal(size=(3, 3))
        A = X @ X.T + np.diag(rng.uniform(0, 1, 3))
        V, lam = oracle.jacobi3(A)
        np.testing.assert_allclose(lam, np.linalg.eigvalsh(A)[::-1], rtol=1e-12)
        np.testing.assert_allclose(V @ np.diag(lam) @ V.T, A, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(V.T @ V, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(V) - 1.0) < 1e-12


# ---- Eq. (merge_conditions), Eq. (merge_cov), cap, modes, append --------------------------

def split_one(par, regs, cams, attr_val=1, prm=P, noise=None):
    noise = np.zeros((1, 2, 3), np.float32) if noise is None else noise
    attr = np.array([attr_val], np.int32)
    regs = np.concatenate(regs) if len(regs) else np.zeros(0, oracle.REGION_DTYPE)
    return oracle.adaptive_split(par, np.array([0], np.int32), regs, cams, attr, prm, noise)


def cov_of(q, ls):
    q = np.asarray(q, np.float64)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    return R @ np.diag(np.exp(2 * np.asarray(ls, np.float64))) @ R.T


CAM = synth.Camera(np.eye(3), (0, 0, 4), 100.0, 100.0, 64, 48, 128, 96)
PAR = parent((0.0, 0.0, 0.0), [math.log(0.3)] * 3, logit=0.7)


def test_singleton_group_is_its_proposal():
    reg = region_record(0, 0, 17, 70.0, 40.0, (0.8, 0.6), 4.0, 1.5, (0.9, 0.1, 0.2))
    out = split_one(PAR, [reg], [CAM])
    ok, muc, R, s = oracle.child_proposal(PAR, reg, CAM)
    assert out["mode"][0] == oracle.MODE_ADAPTIVE and out["count"][0] == 2 and out["n_out"] == 2
    np.testing.assert_allclose(out["means"][:, 0], muc, rtol=1e-6)
    np.testing.assert_allclose(cov_of(out["quats"][:, 0], out["log_scales"][:, 0]), R @ np.diag(s ** 2) @ R.T,
                               rtol=2e-6, atol=1e-9)
    C0 = 1 / (2 * math.sqrt(math.pi))
    np.testing.assert_allclose(out["sh"][0, :, 0] * C0 + 0.5, [0.9, 0.1, 0.2], rtol=1e-6)
    assert out["opacity_logits"][0] == PAR.opacity_logits[0]
    # parent copy: unchanged apart from opacity o / (N + 1)
    np.testing.assert_array_equal(out["means"][:, 1], PAR.means[:, 0])
    o = 1 / (1 + math.exp(-float(PAR.opacity_logits[0])))
    np.testing.assert_allclose(1 / (1 + math.exp(-float(out["opacity_logits"][1]))), o / 2, rtol=1e-6)


def test_identical_proposals_merge_to_one():
    reg_a = region_record(0, 0, 17, 70.0, 40.0, (0.8, 0.6), 4.0, 1.5, (0.9, 0.1, 0.2))
    reg_b = region_record(0, 1, 5, 70.0, 40.0, (0.8, 0.6), 4.0, 1.5, (0.9, 0.1, 0.2))
    out = split_one(PAR, [reg_a, reg_b], [CAM, CAM])
    single = split_one(PAR, [reg_a], [CAM])
    assert out["count"][0] == 2
    np.testing.assert_allclose(out["means"][:, 0], single["means"][:, 0], rtol=1e-6)
    np.testing.assert_allclose(cov_of(out["quats"][:, 0], out["log_scales"][:, 0]),
                               cov_of(single["quats"][:, 0], single["log_scales"][:, 0]), rtol=1e-5, atol=1e-9)


def _gap_pair(dx_px):
    a = region_record(0, 0, 1, 64.0, 48.0, (1, 0), 2.0, 2.0, (0.5, 0.5, 0.5))
    b = region_record(0, 0, 2, 64.0 + dx_px, 48.0, (1, 0), 2.0, 2.0, (0.5, 0.5, 0.5))
    return a, b


def test_merge_threshold_just_below_and_above_gamma_d():
    """Two isotropic-in-plane children offset along x: the symmetric
    Mahalanobis sum is 2 * dx / s1, so the link flips at dx = s1."""
    a, b = _gap_pair(0.0)
    ok, mua, Ra, sa = oracle.child_proposal(PAR, a, CAM)
    s1 = sa[0]
    fx, tz = 100.0, 4.0
    for frac, linked in ((0.999, True), (1.001, False)):
        dx_px = frac * s1 * fx / tz
        a, b = _gap_pair(dx_px)
        out = split_one(PAR, [a, b], [CAM])
        assert out["count"][0] == (2 if linked else 3), frac


def test_chain_is_transitive_and_colour_gate():
    # sigma = 2 px at t_z = 4, f = 100: links need an offset below 2 px
    a = region_record(0, 0, 1, 60.0, 48.0, (1, 0), 2.0, 2.0, (0.5, 0.5, 0.5))
    b = region_record(0, 0, 2, 61.8, 48.0, (1, 0), 2.0, 2.0, (0.5, 0.5, 0.5))
    c = region_record(0, 0, 3, 63.6, 48.0, (1, 0), 2.0, 2.0, (0.5, 0.5, 0.5))
    out = split_one(PAR, [a, b, c], [CAM])
    out_ac = split_one(PAR, [a, c], [CAM])
    assert out_ac["count"][0] == 3        # A and C alone do not link
    assert out["count"][0] == 2           # A-B-C chain is one group
    c2 = region_record(0, 0, 3, 63.6, 48.0, (1, 0), 2.0, 2.0, (0.5, 0.5, 0.66))
    out = split_one(PAR, [a, b, c2], [CAM])
    assert out["count"][0] == 3           # colour difference 0.16 > 0.15 cuts B-C


def test_merged_group_encloses_members():
    """Eq. (merge_cov): the merged ellipsoid's reach along its own axes covers
    every member's 1-sigma reach (support-function containment)."""
    a = region_record(0, 0, 1, 60.0, 48.0, (1, 0), 3.0, 1.0, (0.5, 0.5, 0.5))
    b = region_record(0, 1, 2, 60.5, 48.2, (0.6, 0.8), 2.0, 1.2, (0.52, 0.5, 0.5))
    out = split_one(PAR, [a, b], [CAM, CAM])
    assert out["count"][0] == 2
    Sm = cov_of(out["quats"][:, 0], out["log_scales"][:, 0])
    lam, E = np.linalg.eigh(Sm)
    mum = out["means"][:, 0].astype(np.float64)
    for reg in (a, b):
        ok, mu, R, s = oracle.child_proposal(PAR, reg, CAM)
        S = R @ np.diag(s ** 2) @ R.T
        for r in range(3):
            e = E[:, r]
            assert abs(e @ (mu - mum)) + math.sqrt(e @ S @ e) <= math.sqrt(lam[r]) * (1 + 1e-5)


# Closed forms of Eq. (merge_cov).  For axis-aligned members whose mean
# covariance has distinct eigenvalues, the merged axes are the coordinate axes
# (descending variance) and the merged scale along each axis is the largest
# member reach along it: offset from the merged mean plus the member's own
# scale on that axis.

def _axis_members(offsets, scales, colours, Q=None, centre=(0.0, 0.0, 0.0)):
    Q = np.eye(3) if Q is None else Q
    mu = np.array([centre]) + (Q @ np.asarray(offsets, np.float64).T).T
    R = np.repeat(Q[None], len(offsets), axis=0)
    return mu, R, np.asarray(scales, np.float64), np.asarray(colours, np.float64)


def _axes_match(E, Q):
    """E's columns equal Q's up to sign, and det E = +1 [A21]."""
    np.testing.assert_allclose(np.abs(E.T @ Q), np.eye(3), atol=1e-12)
    assert abs(np.linalg.det(E) - 1.0) < 1e-12


def test_merge_pair_closed_form():
    """Two members of scales (s1, s2, s3), s1 > s2 > s3, offset by d along x
    with different colours: mean = midpoint, colour = average, axes = x, y,
    z, scales (d/2 + s1, s2, s3)."""
    d, sc = 0.4, (0.3, 0.2, 0.1)
    c = (0.25, -0.5, 1.5)
    mu, R, s, rgb = _axis_members([(-d / 2, 0, 0), (d / 2, 0, 0)], [sc, sc],
                                  [(0.9, 0.2, 0.4), (0.7, 0.6, 0.0)], centre=c)
    m, col, E, sm = oracle.merge_group(mu, R, s, rgb)
    np.testing.assert_allclose(m, c, rtol=0, atol=1e-15)
    np.testing.assert_allclose(col, [0.8, 0.4, 0.2], rtol=0, atol=1e-15)
    _axes_match(E, np.eye(3))
    np.testing.assert_allclose(sm ** 2, [(d / 2 + sc[0]) ** 2, sc[1] ** 2, sc[2] ** 2], rtol=1e-12)


def test_merge_pair_rotated_closed_form():
    """The same pair rotated by Q about an arbitrary centre: the axes rotate
    with it and the scales do not change."""
    d, sc = 0.4, (0.3, 0.2, 0.1)
    for seed in range(5):
        Q = Rotation.random(random_state=seed).as_matrix()
        mu, R, s, rgb = _axis_members([(-d / 2, 0, 0), (d / 2, 0, 0)], [sc, sc],
                                      [(0.9, 0.2, 0.4), (0.7, 0.6, 0.0)], Q=Q, centre=(1.0, 2.0, -3.0))
        m, col, E, sm = oracle.merge_group(mu, R, s, rgb)
        np.testing.assert_allclose(m, (1.0, 2.0, -3.0), rtol=0, atol=1e-14)
        np.testing.assert_allclose(col, [0.8, 0.4, 0.2], rtol=0, atol=1e-15)
        _axes_match(E, Q)
        np.testing.assert_allclose(sm, [d / 2 + sc[0], sc[1], sc[2]], rtol=1e-12)


def test_merge_three_members_takes_the_max_reach():
    """Three members of unequal shape at uneven x offsets: each merged scale
    is the largest member reach on that axis, which differs from the sum over
    members and from the first member's reach."""
    offs = [(-0.5, 0.0, 0.0), (0.1, 0.0, 0.0), (0.7, 0.0, 0.0)]
    scs = [(0.30, 0.12, 0.05), (0.25, 0.21, 0.04), (0.35, 0.15, 0.08)]
    cols = [(0.1, 0.2, 0.3), (0.4, 0.5, 0.6), (0.7, 0.8, 0.3)]
    mu, R, s, rgb = _axis_members(offs, scs, cols)
    m, col, E, sm = oracle.merge_group(mu, R, s, rgb)
    xbar = (-0.5 + 0.1 + 0.7) / 3
    np.testing.assert_allclose(m, [xbar, 0, 0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(col, np.mean(cols, axis=0), rtol=0, atol=1e-15)
    # mean covariance diag(mean s_x^2, mean s_y^2, mean s_z^2) is already
    # ordered x > y > z here, so the axes are x, y, z
    sq = np.square(scs).mean(0)
    assert sq[0] > sq[1] > sq[2]
    _axes_match(E, np.eye(3))
    want = [max(abs(o[0] - xbar) + t[0] for o, t in zip(offs, scs)),
            max(t[1] for t in scs), max(t[2] for t in scs)]
    np.testing.assert_allclose(sm, want, rtol=1e-12)
    # the max is not the sum, nor the first member's reach, nor the last's
    assert abs(sm[1] - sum(t[1] for t in scs)) > 0.1
    assert abs(sm[1] - scs[0][1]) > 0.05 and abs(sm[0] - (abs(offs[0][0] - xbar) + scs[0][0])) > 0.05


def test_merge_axes_follow_the_mean_covariance_order():
    """When the members' variance is largest along z, the first merged axis
    is z: the axes come from the mean covariance, in descending order."""
    mu, R, s, rgb = _axis_members([(0, 0, -0.1), (0, 0, 0.1)], [(0.1, 0.2, 0.5), (0.1, 0.2, 0.5)],
                                  [(0.5, 0.5, 0.5)] * 2)
    m, col, E, sm = oracle.merge_group(mu, R, s, rgb)
    P = np.array([[0, 0, 1], [0, 1, 0], [1, 0, 0]], np.float64)   # columns z, y, x
    _axes_match(E, P)
    np.testing.assert_allclose(sm, [0.1 + 0.5, 0.2, 0.1], rtol=1e-12)


def test_split_writes_the_merged_child():
    """Through the whole split: two regions in two views whose proposals
    merge.  The child's mean, colour (read back from the SH DC) and
    covariance are the merge of the two proposals, and the colour is the
    average of two different region colours."""
    a = region_record(0, 0, 1, 60.0, 48.0, (1, 0), 3.0, 1.0, (0.50, 0.40, 0.30))
    b = region_record(0, 1, 2, 60.6, 48.3, (0.6, 0.8), 2.0, 1.2, (0.60, 0.30, 0.40))
    out = split_one(PAR, [a, b], [CAM, CAM])
    assert out["mode"][0] == oracle.MODE_ADAPTIVE and out["count"][0] == 2
    props = [oracle.child_proposal(PAR, r, CAM) for r in (a, b)]
    assert all(p[0] for p in props)
    mu = np.stack([p[1] for p in props])
    R = np.stack([p[2] for p in props])
    sc = np.stack([p[3] for p in props])
    m, col, E, sm = oracle.merge_group(mu, R, sc, [(0.50, 0.40, 0.30), (0.60, 0.30, 0.40)])
    np.testing.assert_allclose(m, mu.mean(0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(col, [0.55, 0.35, 0.35], rtol=0, atol=1e-15)
    np.testing.assert_allclose(out["means"][:, 0], m, rtol=1e-6)
    C0 = 1 / (2 * math.sqrt(math.pi))
    np.testing.assert_allclose(out["sh"][0, :, 0].astype(np.float64) * C0 + 0.5, [0.55, 0.35, 0.35], rtol=1e-6)
    np.testing.assert_allclose(cov_of(out["quats"][:, 0], out["log_scales"][:, 0]), E @ np.diag(sm ** 2) @ E.T,
                               rtol=1e-5, atol=1e-9)


def test_vanilla_fallback_without_attribution():
    noise = synth.vanilla_noise(1, 3)
    out = split_one(PAR, [], [CAM], attr_val=0, noise=noise)
    assert out["mode"][0] == oracle.MODE_VANILLA and out["count"][0] == 2 and out["n_out"] == 2
    q = PAR.quats[:, 0].astype(np.float64)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    s = np.exp(PAR.log_scales[:, 0].astype(np.float64))
    for c in range(2):
        want = PAR.means[:, 0] + R @ (s * noise[0, c].astype(np.float64))
        np.testing.assert_allclose(out["means"][:, c], want, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(np.exp(out["log_scales"][:, c].astype(np.float64)), s / (0.8 * 2), rtol=1e-6)
        np.testing.assert_array_equal(out["quats"][:, c], PAR.quats[:, 0])
        assert out["opacity_logits"][c] == PAR.opacity_logits[0]


def test_reset_when_attributed_but_no_region_survives():
    reg = region_record(0, 0, 1, 70.0, 40.0, (1, 0), 2.0, 1.0, (0.5, 0.5, 0.5))
    out = split_one(PAR, [], [CAM], attr_val=4)
    assert out["mode"][0] == oracle.MODE_RESET and out["count"][0] == 0 and out["n_out"] == 1
    np.testing.assert_array_equal(out["means"][:, 0], PAR.means[:, 0])
    del reg


def _separated_regions(k, view=0):
    regs = []
    for j in range(k):
        cx = 8.0 + 12.0 * (j % 10)
        cy = 10.0 + 14.0 * (j // 10)
        regs.append(region_record(0, view, 100 + j, cx, cy, (1, 0), 1.5, 1.0, (0.1 + 0.03 * j, 0.5, 0.5)))
    return regs


@pytest.mark.parametrize("k,want", [(1, 2), (3, 4), (7, 8), (25, 20)])
def test_k_separated_regions_give_k_plus_one_rows_capped(k, want):
    par = parent((0.0, 0.0, 0.0), [math.log(0.02)] * 3, logit=0.7)
    out = split_one(par, _separated_regions(k), [CAM])
    assert out["count"][0] == want and out["n_out"] == want


def test_cap_keeps_largest_extents_in_order():
    par = parent((0.0, 0.0, 0.0), [math.log(0.5)] * 3, logit=0.7)
    regs = []
    for j in range(25):
        cx = 8.0 + 12.0 * (j % 10)
        cy = 10.0 + 14.0 * (j // 10)
        regs.append(region_record(0, 0, 100 + j, cx, cy, (1, 0), 1.0 + 0.1 * j, 0.5, (0.03 * j, 0.5, 0.5)))
    out = split_one(par, regs, [CAM], prm=oracle.SplitParams(gamma_d=1e-9))
    ext = np.exp(out["log_scales"][:, :19].astype(np.float64).sum(0))
    assert (np.diff(ext) <= 1e-12 * ext[:-1]).all()
    assert out["count"][0] == 20


def test_append_order_and_offsets():
    scene = synth.scene_uniform_sh0(10, seed=4)
    cams = [CAM]
    cand = np.array([2, 5, 7], np.int32)
    attr = np.zeros(10, np.int32)
    attr[5] = 3   # 5 -> reset, 2 and 7 -> vanilla
    noise = synth.vanilla_noise(3, 1)
    out = oracle.adaptive_split(scene, cand, np.zeros(0, oracle.REGION_DTYPE), cams, attr, P, noise)
    np.testing.assert_array_equal(out["mode"], [0, 1, 0])
    np.testing.assert_array_equal(out["count"], [2, 0, 2])
    np.testing.assert_array_equal(out["offset"], [0, 2, 2])
    surv = [i for i in range(10) if i not in (2, 7)]
    assert out["n_out"] == 8 + 4
    np.testing.assert_array_equal(out["opacity_logits"][:8], scene.opacity_logits[surv])
    np.testing.assert_array_equal(out["quats"][:, 8:10], np.repeat(scene.quats[:, 2:3], 2, 1))
    np.testing.assert_array_equal(out["quats"][:, 10:12], np.repeat(scene.quats[:, 7:8], 2, 1))


def test_end_to_end_maps_to_counts():
    """Hand-built maps through both stages: a candidate with two separated
    regions in one view and the same two regions in a second view ends with
    2 merged children + parent copy; a candidate with only tiny regions is
    reset; a candidate never dominant falls back to the vanilla split."""
    H, W = 64, 96
    E = np.zeros((H, W))
    dom = np.full((H, W), -1, np.int32)
    dom[:, :48] = 0
    dom[:, 48:] = 1
    E[10:17, 10:17] = 1.0     # candidate 0, region A
    E[40:47, 20:27] = 1.0     # candidate 0, region B
    E[10:12, 60:62] = 1.0     # candidate 1: 2x2 only
    img, gt, dom, _ = maps_from_error(E, dom)
    gt[:] = 0.25
    img[0] = E.astype(np.float32) + 0.25
    is_cand = np.array([1, 1, 1], np.uint8)
    prm = oracle.SplitParams(r_erode=1)
    attr = np.zeros(3, np.int32)
    regs0, _ = oracle.error_stats(img, gt, dom, is_cand, 0, prm, attr)
    regs1, _ = oracle.error_stats(img, gt, dom, is_cand, 1, prm, attr)
    regs = np.concatenate([regs0, regs1])
    assert len(regs) == 4 and attr.tolist() == [2 * 98, 2 * 4, 0]
    scene = synth.scene_uniform_sh0(3, seed=9)
    scene.means[:] = 0.0
    scene.log_scales[:] = math.log(0.3)
    cam = synth.Camera(np.eye(3), (0, 0, 4), 100.0, 100.0, 48, 32, W, H)
    out = oracle.adaptive_split(scene, np.array([0, 1, 2], np.int32), regs, [cam, cam], attr, prm,
                                synth.vanilla_noise(3, 0))
    np.testing.assert_array_equal(out["mode"], [2, 1, 0])
    np.testing.assert_array_equal(out["count"], [3, 0, 2])
    assert out["n_out"] == 1 + 5


# ---- Table 2 ablation variants, the fixed-N random split, alternative readings ------------

def test_fixed_n_random_split_statistics():
    """Fixed N = 5 random children (the five-child split of Sec. 1): N rows per
    candidate whatever the regions say, scales shrunk by eta * N, and the
    offsets of the children from the parent centre have the parent's
    covariance (checked statistically over many candidates)."""
    n = 400
    rng = np.random.default_rng(3)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    ls = np.log([0.3, 0.1, 0.05])
    scene = synth.Scene(np.zeros((3, n), np.float32), np.repeat(ls[:, None], n, 1).astype(np.float32),
                        np.repeat(q[:, None], n, 1).astype(np.float32), np.full(n, 0.4, np.float32),
                        np.zeros((1, 3, n), np.float32), 0)
    N = 5
    prm = oracle.SplitParams(variant=oracle.VARIANT_FIXED_N, fixed_n=N, noise_n=N)
    noise = rng.normal(size=(n, N, 3)).astype(np.float32)
    reg = region_record(0, 0, 1, 70.0, 40.0, (1, 0), 2.0, 1.0, (0.5, 0.5, 0.5))
    out = oracle.adaptive_split(scene, np.arange(n, dtype=np.int32), reg, [CAM], np.ones(n, np.int32), prm, noise)
    assert (out["mode"] == 3).all() and (out["count"] == N).all() and out["n_out"] == n * N
    np.testing.assert_allclose(np.exp(out["log_scales"][:, 0].astype(np.float64)), np.exp(ls) / (0.8 * N), rtol=1e-6)
    off = out["means"][:, : n * N].astype(np.float64)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    S = R @ np.diag(np.exp(2 * ls)) @ R.T
    emp = off @ off.T / off.shape[1]
    assert np.abs(emp - S).max() <= 0.1 * np.abs(S).max()


def test_ablation_steps_on_one_region_seen_twice():
    """The same region in two views: AdpSplit merges the two proposals (one
    child + parent copy), child initialisation without merging keeps both
    (two children + parent copy), adaptive N places two random children."""
    reg_a = region_record(0, 0, 17, 70.0, 40.0, (0.8, 0.6), 4.0, 1.5, (0.9, 0.1, 0.2))
    reg_b = region_record(0, 1, 5, 70.0, 40.0, (0.8, 0.6), 4.0, 1.5, (0.9, 0.1, 0.2))
    noise = np.zeros((1, 19, 3), np.float32)
    full = split_one(PAR, [reg_a, reg_b], [CAM, CAM])
    ci = split_one(PAR, [reg_a, reg_b], [CAM, CAM], prm=oracle.SplitParams(variant=oracle.VARIANT_CHILD_INIT))
    an = split_one(PAR, [reg_a, reg_b], [CAM, CAM], noise=noise,
                   prm=oracle.SplitParams(variant=oracle.VARIANT_ADAPTIVE_N, noise_n=19))
    assert (full["mode"][0], full["count"][0]) == (oracle.MODE_ADAPTIVE, 2)
    assert (ci["mode"][0], ci["count"][0]) == (oracle.MODE_ADAPTIVE, 3)
    assert (an["mode"][0], an["count"][0]) == (3, 2)
    # child initialisation: each child is its region's proposal
    ok, muc, R, s = oracle.child_proposal(PAR, reg_a, CAM)
    for c in range(2):
        np.testing.assert_allclose(ci["means"][:, c], muc, rtol=1e-6)
    # adaptive N with zero noise: children sit on the parent, scales / (eta * 2)
    for c in range(2):
        np.testing.assert_array_equal(an["means"][:, c], PAR.means[:, 0])
        np.testing.assert_allclose(np.exp(an["log_scales"][:, c].astype(np.float64)),
                                   np.exp(PAR.log_scales[:, 0].astype(np.float64)) / 1.6, rtol=1e-6)
    assert an["n_out"] == 2   # parent removed, no copy


@pytest.mark.parametrize("variant", [oracle.VARIANT_ADAPTIVE_N, oracle.VARIANT_CHILD_INIT])
def test_ablation_counts_track_regions(variant):
    par = parent((0.0, 0.0, 0.0), [math.log(0.02)] * 3, logit=0.7)
    for k in (1, 4, 25):
        out = split_one(par, _separated_regions(k), [CAM], noise=np.zeros((1, 19, 3), np.float32),
                        prm=oracle.SplitParams(variant=variant, noise_n=19))
        nk = min(k, 19)
        assert out["count"][0] == (nk if variant == oracle.VARIANT_ADAPTIVE_N else nk + 1)


def test_cross_view_flag_keeps_same_view_pairs_apart():
    a = region_record(0, 0, 1, 60.0, 48.0, (1, 0), 2.0, 2.0, (0.5, 0.5, 0.5))
    b = region_record(0, 0, 2, 60.5, 48.0, (1, 0), 2.0, 2.0, (0.5, 0.5, 0.5))
    b2 = region_record(0, 1, 2, 60.5, 48.0, (1, 0), 2.0, 2.0, (0.5, 0.5, 0.5))
    fl = oracle.SplitParams(flags=oracle.FLAG_CROSS_VIEW)
    assert split_one(PAR, [a, b], [CAM])["count"][0] == 2           # default: any pair links
    assert split_one(PAR, [a, b], [CAM], prm=fl)["count"][0] == 3   # same view: not merged
    assert split_one(PAR, [a, b2], [CAM, CAM], prm=fl)["count"][0] == 2


def test_extent_flag_changes_which_child_the_cap_keeps():
    """Two separated children, N_max = 1: one is long and thin (larger
    maximum scale), the other round (larger s1 s2 s3)."""
    par = parent((0.0, 0.0, 0.0), [math.log(0.5)] * 3, logit=0.7)
    thin = region_record(0, 0, 1, 30.0, 30.0, (1, 0), 6.0, 0.3, (0.1, 0.5, 0.5))
    round_ = region_record(0, 0, 2, 90.0, 60.0, (1, 0), 3.0, 3.0, (0.9, 0.5, 0.5))
    C0 = 1 / (2 * math.sqrt(math.pi))
    prod = split_one(par, [thin, round_], [CAM], prm=oracle.SplitParams(n_max=1))
    mx = split_one(par, [thin, round_], [CAM], prm=oracle.SplitParams(n_max=1, flags=oracle.FLAG_EXTENT_MAX))
    assert prod["sh"][0, 0, 0] * C0 + 0.5 == pytest.approx(0.9, abs=1e-6)   # round: larger product
    assert mx["sh"][0, 0, 0] * C0 + 0.5 == pytest.approx(0.1, abs=1e-6)     # thin: larger maximum


def test_shared_opacity_flag():
    par = parent((0.0, 0.0, 0.0), [math.log(0.02)] * 3, logit=0.7)
    out = split_one(par, _separated_regions(3), [CAM], prm=oracle.SplitParams(flags=oracle.FLAG_SHARE_OPACITY))
    o = 1 / (1 + math.exp(-0.7))
    got = 1 / (1 + np.exp(-out["opacity_logits"][:4].astype(np.float64)))
    np.testing.assert_allclose(got, o / 4, rtol=1e-6)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_erosion_side_flag_on_a_block(r):
    """A square element of side r+1 (offsets -floor(r/2) .. r - floor(r/2))
    erodes a w x h block away from the borders to (w - r) x (h - r), shifted
    by the element's asymmetry."""
    H, W = 40, 50
    E = np.zeros((H, W))
    E[10:30, 12:40] = 1.0
    dom = np.zeros((H, W), np.int32)
    img, gt, dom, is_cand = maps_from_error(E, dom)
    prm = oracle.SplitParams(r_erode=r, flags=oracle.FLAG_ERODE_SIDE, m_min=1)
    regs, maps = oracle.error_stats(img, gt, dom, is_cand, 0, prm, np.zeros(1, np.int32), want_maps=True)
    lo, hi = r // 2, r - r // 2
    want = np.zeros((H, W), bool)
    want[10 + lo:30 - hi, 12 + lo:40 - hi] = True
    np.testing.assert_array_equal(maps["Mp"].astype(bool), want)
