"""Pins of the CPU oracle of the optimisation loop (no GPU): Adam against
torch.optim.Adam in FP64 and its first-step closed form, the L1 loss on
hand-computed values, the density-control selection, clone and prune on
hand-built sets, and the split's row map against the split oracle's own
output rows."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import train as otrain
from paper_2605_06876_amd import synth

HP = dict(lr_means=1.6e-3, lr_log_scales=5e-3, lr_quats=1e-3, lr_opacity=5e-2, lr_sh_dc=2.5e-3,
          lr_sh_rest=2.5e-3 / 20, beta1=0.9, beta2=0.999, eps=1e-15)


def rand_set(n, deg, rng):
    nk = (deg + 1) ** 2
    return dict(means=rng.normal(0, 1, (3, n)), log_scales=rng.normal(-3, 0.5, (3, n)), quats=rng.normal(0, 1, (4, n)),
                opacity_logits=rng.normal(0, 1, n), sh=rng.normal(0, 0.3, (nk, 3, n)))


def test_adam_matches_torch_adam_over_steps():
    rng = np.random.default_rng(1)
    n, deg = 37, 2
    p = rand_set(n, deg, rng)
    zero = {k: np.zeros_like(v) for k, v in p.items()}
    m, v = dict(zero), dict(zero)
    tens = {k: torch.tensor(p[k], dtype=torch.float64, requires_grad=True) for k in ("means", "log_scales", "quats",
                                                                                   "opacity_logits")}
    sh_dc = torch.tensor(p["sh"][:1], dtype=torch.float64, requires_grad=True)
    sh_rest = torch.tensor(p["sh"][1:], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([
        dict(params=[tens["means"]], lr=HP["lr_means"]), dict(params=[tens["log_scales"]], lr=HP["lr_log_scales"]),
        dict(params=[tens["quats"]], lr=HP["lr_quats"]), dict(params=[tens["opacity_logits"]], lr=HP["lr_opacity"]),
        dict(params=[sh_dc], lr=HP["lr_sh_dc"]), dict(params=[sh_rest], lr=HP["lr_sh_rest"])],
        betas=(HP["beta1"], HP["beta2"]), eps=HP["eps"])
    for step in range(1, 5):
        g = rand_set(n, deg, rng)
        for k in tens:
            tens[k].grad = torch.tensor(g[k])
        sh_dc.grad = torch.tensor(g["sh"][:1])
        sh_rest.grad = torch.tensor(g["sh"][1:])
        opt.step()
        p, m, v = otrain.adam_step(p, g, m, v, HP, step)
    for k in tens:
        np.testing.assert_allclose(p[k], tens[k].detach().numpy(), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(p["sh"][:1], sh_dc.detach().numpy(), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(p["sh"][1:], sh_rest.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(2)
    p = rand_set(5, 0, rng)
    g = rand_set(5, 0, rng)
    z = {k: np.zeros_like(a) for k, a in p.items()}
    out, m, v = otrain.adam_step(p, g, z, z, dict(HP, eps=0.0), 1)
    # m-hat = g and v-hat = g^2, so the step is -lr sign(g)
    np.testing.assert_allclose(out["means"] - p["means"], -HP["lr_means"] * np.sign(g["means"]), rtol=1e-12)
    np.testing.assert_allclose(out["sh"][0] - p["sh"][0], -HP["lr_sh_dc"] * np.sign(g["sh"][0]), rtol=1e-12)
    np.testing.assert_allclose(m["quats"], 0.1 * g["quats"], rtol=1e-15)
    np.testing.assert_allclose(v["quats"], 0.001 * g["quats"] ** 2, rtol=1e-12)


def test_l1_loss_hand_values():
    img = np.zeros((3, 1, 2), np.float32)
    gt = np.zeros((3, 1, 2), np.float32)
    img[0, 0, 0], gt[0, 0, 0] = 0.75, 0.25     # d = +0.5
    img[1, 0, 1], gt[1, 0, 1] = 0.0, 0.25      # d = -0.25
    dL, (s1, s2) = otrain.l1_loss(img, gt)
    assert s1 == pytest.approx(0.75) and s2 == pytest.approx(0.3125)
    assert dL[0, 0, 0] == pytest.approx(1 / 6) and dL[1, 0, 1] == pytest.approx(-1 / 6)
    assert (dL[2] == 0).all() and dL[0, 0, 1] == 0.0   # sign(0) = 0


def test_densify_select_hand_cases():
    ls = np.log(np.array([[0.01, 0.01, 0.5, 0.5, 0.01, 0.5], [0.01] * 6, [0.01] * 6]))
    g = dict(log_scales=ls)
    accum = np.array([0.3, 0.1, 0.3, 0.1, 0.0, 0.5], np.float32)
    vis = np.array([1, 1, 1, 1, 0, 2], np.int32)
    clone, cand, ids = otrain.densify_select(g, accum, vis, 0.2, 0.1)
    # averages 0.3, 0.1, 0.3, 0.1, 0.0, 0.25; large scale at rows 2, 3, 5
    assert clone.tolist() == [True, False, False, False, False, False]
    assert cand.tolist() == [False, False, True, False, False, True]
    assert ids.tolist() == [2, 5]


def test_split_row_map_matches_the_split_oracle_rows():
    CAM = synth.Camera(np.eye(3), (0, 0, 4), 100.0, 100.0, 64, 48, 128, 96)
    P = oracle.SplitParams()
    scene = synth.scene_uniform_sh0(10, seed=4)
    cand = np.array([2, 5, 7], np.int32)
    attr = np.zeros(10, np.int32)
    attr[5] = 3   # modes: vanilla, reset, vanilla
    out = oracle.adaptive_split(scene, cand, np.zeros(0, oracle.REGION_DTYPE), [CAM], attr, P,
                                synth.vanilla_noise(3, 1))
    rm = otrain.split_row_map(10, cand, out["mode"], 14)
    n_surv = int((rm >= 0).sum())
    assert n_surv == out["n_out"] - int(out["count"].sum())
    for f in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        np.testing.assert_array_equal(np.asarray(out[f])[..., :n_surv], np.asarray(getattr(scene, f))[..., rm[:n_surv]])
    assert (rm[n_surv:] == -1).all()


def test_split_row_map_hand_case():
    rm = otrain.split_row_map(6, np.array([1, 3, 4]), np.array([0, 1, 2]), 9)
    assert rm.tolist() == [0, 2, 3, 5, -1, -1, -1, -1, -1]
    rm = otrain.split_row_map(6, np.array([1, 3, 4]), np.array([0, 1, 2]), 5, state_in=[7, 8, -1, 9, 10, 11])
    assert rm.tolist() == [7, -1, 9, 11, -1]


def test_clone_prune_hand_case():
    rng = np.random.default_rng(3)
    g = rand_set(6, 1, rng)
    logit = lambda p: math.log(p / (1 - p))
    g["opacity_logits"][:] = [logit(0.5), logit(0.001), logit(0.5), logit(0.2), logit(0.004), logit(0.9)]
    g["log_scales"][:] = np.log(0.05)
    g["log_scales"][1, 3] = np.log(2.0)        # too large: pruned when max_scale = 1
    clone = np.array([1, 1, 0, 0, 0, 1], bool)
    state_in = np.array([10, 11, -1, 13, 14, 15])
    out, st = otrain.clone_prune(g, clone, state_in, 0.005, 1.0)
    # kept: 0, 2, 5 (1 and 4 transparent, 3 too large); clones of kept: 0, 5
    np.testing.assert_array_equal(out["means"], g["means"][:, [0, 2, 5, 0, 5]])
    assert st.tolist() == [10, -1, 15, -1, -1]
    out2, st2 = otrain.clone_prune(g, None, None, 0.005, 0.0)
    assert st2.tolist() == [0, 2, 3, 5]


def test_gather_rows_and_reset_opacity():
    rng = np.random.default_rng(5)
    g = rand_set(4, 0, rng)
    out = otrain.gather_rows(g, [3, -1, 0])
    np.testing.assert_array_equal(out["quats"], np.stack([g["quats"][:, 3], np.zeros(4), g["quats"][:, 0]], 1))
    o = otrain.reset_opacity(np.array([-10.0, 0.0, 5.0]), 0.01)
    cap = math.log(0.01 / 0.99)
    assert o.tolist() == pytest.approx([-10.0, cap, cap])
    assert 1 / (1 + math.exp(-cap)) == pytest.approx(0.01)
