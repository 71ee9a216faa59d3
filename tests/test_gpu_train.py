"""GPU parity of the optimisation-loop entry points against the CPU oracle
(oracle/train.py) on seeded inputs spanning several blocks with ragged tails:
Adam (FP32 against FP64, bounds derived from FP32 rounding: the first moment
within 4 ulp of its terms' magnitude (they may cancel), the second within
8 ulp, parameters within 4 ulp plus 16 ulp of the step plus the first
moment's error carried through the step), the L1 gradient (bit-exact) and sums
(1e-6 relative), and bit-exact selections, row maps, clone + prune and
gathers."""
import math
import sys

import numpy as np
import pytest

from oracle import train as otrain

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_06876_amd import api  # noqa: E402

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    # scratch for the largest Gaussian set of the loop calls below
    return api.Context(0, max_gaussians=1 << 17, max_candidates=1 << 12, max_regions=1 << 10, max_views=4)


def rand_set(n, deg, rng, ls_mu=-3.0):
    nk = (deg + 1) ** 2
    f = np.float32
    return dict(means=rng.normal(0, 1, (3, n)).astype(f), log_scales=rng.normal(ls_mu, 0.7, (3, n)).astype(f),
                quats=rng.normal(0, 1, (4, n)).astype(f), opacity_logits=rng.normal(0, 3, n).astype(f),
                sh=rng.normal(0, 0.3, (nk, 3, n)).astype(f))


def to_dev(d, deg):
    t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).cuda() for k in FIELDS}
    return api.Gaussians(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], t["sh"], deg)


def to_host(g, n=None):
    return {k: getattr(g, k).cpu().numpy()[..., :n] if n is not None else getattr(g, k).cpu().numpy() for k in FIELDS}


HP = api.AdamParams(lr_means=1.6e-3)
# the library takes its hyper-parameters as FP32: the oracle gets the same rounded values
HPD = {k: float(np.float32(getattr(HP, k))) for k in ("lr_means", "lr_log_scales", "lr_quats", "lr_opacity", "lr_sh_dc",
                                                       "lr_sh_rest", "beta1", "beta2", "eps")}


@pytest.mark.parametrize("n,deg,step", [(1000, 0, 1), (70001, 3, 7), (257, 1, 2)])
def test_adam_step_matches_oracle(ctx, n, deg, step):
    say("adam n=%d deg=%d step=%d" % (n, deg, step))
    rng = np.random.default_rng(n + step)
    p, g = rand_set(n, deg, rng), rand_set(n, deg, rng)
    m = {k: (0.01 * rng.normal(size=a.shape)).astype(np.float32) for k, a in p.items()}
    v = {k: (1e-3 * rng.random(size=a.shape)).astype(np.float32) for k, a in p.items()}
    P, G, M, V = to_dev(p, deg), to_dev(g, deg), to_dev(m, deg), to_dev(v, deg)
    api.adam_step(ctx, P, G, M, V, HP, step)
    torch.cuda.synchronize()
    wp, wm, wv = otrain.adam_step(p, g, m, v, HPD, step)
    gp, gm, gv = to_host(P), to_host(M), to_host(V)
    u = 2.0 ** -24
    b1 = HPD["beta1"]
    bc1, bc2 = 1 - b1 ** step, 1 - HPD["beta2"] ** step
    lr = dict(means=HPD["lr_means"], log_scales=HPD["lr_log_scales"], quats=HPD["lr_quats"],
              opacity_logits=HPD["lr_opacity"])
    for k in FIELDS:
        # FP32 rounding of b1 m + (1 - b1) g is relative to the terms, which may cancel
        terms_m = np.abs(b1 * m[k].astype(np.float64)) + np.abs((1 - b1) * g[k].astype(np.float64))
        tol_m = 4 * u * terms_m + 1e-30
        assert (np.abs(gm[k] - wm[k]) <= tol_m).all(), k
        np.testing.assert_allclose(gv[k], wv[k], rtol=8 * u, atol=1e-30, err_msg=k)
        if k == "sh":
            rate = np.full(p[k].shape, HPD["lr_sh_rest"])
            rate[0] = HPD["lr_sh_dc"]
        else:
            rate = lr[k]
        denom = np.sqrt(wv[k] / bc2) + HPD["eps"]
        step_size = np.abs(wp[k] - p[k].astype(np.float64))
        # parameter: its own rounding, the step's relative rounding, and the moment's error carried by the step
        tol = 4 * np.spacing(np.abs(wp[k]).astype(np.float32)).astype(np.float64) + 16 * u * step_size + \
            rate / bc1 * tol_m / denom
        assert (np.abs(gp[k] - wp[k]) <= tol).all(), k


def test_adam_rejects_bad_arguments(ctx):
    rng = np.random.default_rng(0)
    p = to_dev(rand_set(10, 0, rng), 0)
    with pytest.raises(api.AdpSplitError):
        api.adam_step(ctx, p, p, p, p, HP, 0)
    q = to_dev(rand_set(11, 0, rng), 0)
    with pytest.raises(api.AdpSplitError):
        api.adam_step(ctx, p, q, p, p, HP, 1)


@pytest.mark.parametrize("W,H", [(1, 1), (37, 53), (640, 480)])
def test_l1_loss_matches_oracle(ctx, W, H):
    say("l1 %dx%d" % (W, H))
    rng = np.random.default_rng(W * H)
    img = rng.random((3, H, W)).astype(np.float32)
    gt = rng.random((3, H, W)).astype(np.float32)
    eq = rng.random((3, H, W)) < 0.1
    gt[eq] = img[eq]                                   # sign(0) = 0
    it, gtt = torch.from_numpy(img).cuda(), torch.from_numpy(gt).cuda()
    dL, sums = api.l1_loss(ctx, it, gtt)
    _, sums2 = api.l1_loss(ctx, it, gtt, want_grad=False)
    torch.cuda.synchronize()
    wd, (s1, s2) = otrain.l1_loss(img, gt)
    np.testing.assert_array_equal(dL.cpu().numpy(), wd.astype(np.float32))
    got = sums.cpu().numpy()
    assert got[0] == pytest.approx(s1, rel=1e-6) and got[1] == pytest.approx(s2, rel=1e-6)
    np.testing.assert_array_equal(sums2.cpu().numpy(), got)


@pytest.mark.parametrize("n", [1, 999, 50001])
def test_densify_select_matches_oracle(ctx, n):
    say("select n=%d" % n)
    rng = np.random.default_rng(n)
    g = rand_set(n, 0, rng)
    accum = rng.exponential(0.2, n).astype(np.float32)
    vis = rng.integers(0, 5, n).astype(np.int32)
    thr, size_thr = 0.1, math.exp(-2.5)
    clone, is_cand, cand, n_cand = api.densify_select(ctx, to_dev(g, 0), torch.from_numpy(accum).cuda(),
                                                      torch.from_numpy(vis).cuda(), thr, size_thr)
    torch.cuda.synchronize()
    wc, wk, wids = otrain.densify_select(g, accum, vis, thr, size_thr)
    np.testing.assert_array_equal(clone.cpu().numpy().astype(bool), wc)
    np.testing.assert_array_equal(is_cand.cpu().numpy().astype(bool), wk)
    nc = int(n_cand.item())
    assert nc == len(wids)
    np.testing.assert_array_equal(cand[:nc].cpu().numpy(), wids)


def test_densify_select_empty_set(ctx):
    z = torch.zeros
    g = api.Gaussians(z(3, 0, device="cuda"), z(3, 0, device="cuda"), z(4, 0, device="cuda"), z(0, device="cuda"),
                      z(1, 3, 0, device="cuda"), 0)
    _, _, _, n_cand = api.densify_select(ctx, g, z(0, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"),
                                         0.1, 0.1)
    assert int(n_cand.item()) == 0


@pytest.mark.parametrize("n,k,compose", [(10, 3, False), (40001, 5003, True), (300, 0, False)])
def test_split_row_map_matches_oracle(ctx, n, k, compose):
    rng = np.random.default_rng(n + k)
    cand = np.sort(rng.choice(n, k, replace=False)).astype(np.int32)
    mode = rng.integers(0, 4, k).astype(np.uint8)
    state = rng.integers(-1, 2 * n, n).astype(np.int32) if compose else None
    cap = n + 3 * k + 7
    rs = api.split_row_map(ctx, n, torch.from_numpy(cand).cuda(), torch.from_numpy(mode).cuda(), cap,
                           state_in=torch.from_numpy(state).cuda() if compose else None)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(rs.cpu().numpy(), otrain.split_row_map(n, cand, mode, cap, state))


def test_split_row_map_against_a_gpu_split(ctx):
    """The survivors of a fixed-N random split on the GPU are exactly the input
    rows the map names."""
    from paper_2605_06876_amd import synth
    rng = np.random.default_rng(21)
    n = 5000
    g = to_dev(rand_set(n, 1, rng), 1)
    cand = np.sort(rng.choice(n, 300, replace=False)).astype(np.int32)
    prm = api.SplitParams(variant=api.VARIANT_FIXED_N, fixed_n=2)
    regions = api.RegionBuffer(16)
    attr = torch.zeros(n, dtype=torch.int32, device="cuda")
    cam = synth.sphere_cameras(1, 4.0, [(64, 48)], seed=1)[0]
    noise = torch.from_numpy(synth.vanilla_noise(len(cand), 7)).cuda()
    out, mode, count, offset, n_out = api.adaptive_split(ctx, g, torch.from_numpy(cand).cuda(), regions, [cam], attr,
                                                         prm, noise)
    rs = api.split_row_map(ctx, n, torch.from_numpy(cand).cuda(), mode, out.n)
    torch.cuda.synchronize()
    r = rs.cpu().numpy()
    n_surv = int((r >= 0).sum())
    assert n_surv == n - len(cand) and int(n_out.item()) == n_surv + int(count.sum().item())
    src, dst = to_host(g), to_host(out)
    for f in FIELDS:
        np.testing.assert_array_equal(dst[f][..., :n_surv], src[f][..., r[:n_surv]])


@pytest.mark.parametrize("n,deg,max_scale,with_state", [(7, 0, 0.0, False), (30001, 3, 0.2, True),
                                                        (1024, 2, 0.0, True)])
def test_clone_prune_matches_oracle(ctx, n, deg, max_scale, with_state):
    say("clone_prune n=%d deg=%d" % (n, deg))
    rng = np.random.default_rng(n + deg)
    g = rand_set(n, deg, rng, ls_mu=-2.0)
    g["opacity_logits"] = rng.normal(-4.5, 2.0, n).astype(np.float32)   # many below sigmoid^-1(0.005)
    clone = (rng.random(n) < 0.3).astype(np.uint8)
    state = rng.integers(-1, 3 * n, n).astype(np.int32) if with_state else None
    out, st, n_out = api.clone_prune(ctx, to_dev(g, deg), torch.from_numpy(clone).cuda(),
                                     torch.from_numpy(state).cuda() if with_state else None, 0.005, max_scale)
    torch.cuda.synchronize()
    want, wst = otrain.clone_prune(g, clone.astype(bool), state, 0.005, max_scale)
    k = int(n_out.item())
    assert k == len(wst)
    np.testing.assert_array_equal(st.cpu().numpy()[:k], wst)
    got = to_host(out, k)
    for f in FIELDS:
        np.testing.assert_array_equal(got[f], want[f], err_msg=f)


def test_clone_prune_capacity_and_aliasing(ctx):
    rng = np.random.default_rng(2)
    g = to_dev(rand_set(100, 0, rng), 0)
    small = api.Gaussians.empty(150, 0)
    clone = torch.ones(100, dtype=torch.uint8, device="cuda")
    # with a clone mask every row may be cloned: 2 n rows; without, n
    with pytest.raises(api.AdpSplitError) as e:
        api.clone_prune(ctx, g, clone, None, 0.005, 0.0, out=small)
    assert e.value.status == api.AS_ERR_CAPACITY
    with pytest.raises(api.AdpSplitError) as e:
        api.clone_prune(ctx, g, None, None, 0.005, 0.0, out=api.Gaussians.empty(99, 0))
    assert e.value.status == api.AS_ERR_CAPACITY
    api.clone_prune(ctx, g, None, None, 0.005, 0.0, out=small)


@pytest.mark.parametrize("n_src,n_rows", [(100, 130), (60001, 60001)])
def test_gather_rows_matches_oracle(ctx, n_src, n_rows):
    rng = np.random.default_rng(n_src)
    src = rand_set(n_src, 3, rng)
    row_map = rng.integers(-1, n_src, n_rows).astype(np.int32)
    dst = api.gather_rows(ctx, to_dev(src, 3), torch.from_numpy(row_map).cuda(), n_rows)
    torch.cuda.synchronize()
    want = otrain.gather_rows(src, row_map)
    got = to_host(dst, n_rows)
    for f in FIELDS:
        np.testing.assert_array_equal(got[f], want[f].astype(np.float32), err_msg=f)


def test_reset_opacity_matches_oracle(ctx):
    rng = np.random.default_rng(4)
    g = rand_set(3001, 0, rng)
    G = to_dev(g, 0)
    m = torch.ones(3001, device="cuda")
    v = torch.ones(3001, device="cuda")
    api.reset_opacity(ctx, G, 0.01, m, v)
    torch.cuda.synchronize()
    want = otrain.reset_opacity(g["opacity_logits"], 0.01)
    got = G.opacity_logits.cpu().numpy()
    cap = np.float32(math.log(0.01 / 0.99))
    np.testing.assert_array_equal(got, np.minimum(g["opacity_logits"], cap))
    np.testing.assert_allclose(got, want, atol=1e-6)
    assert float(m.abs().sum()) == 0.0 and float(v.abs().sum()) == 0.0
