"""The densification training loop on the GPU (a short synthetic schedule):
every row that keeps optimiser state after a densification step (clone,
split, prune) is a bit-exact copy of the pre-step row it names, rows without
state are exactly the clones and the split's new rows, the Adam moments follow
their rows, and training improves the held-out PSNR for both split methods."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_06876_amd import api, train  # noqa: E402

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    ctx = api.Context(0)
    pb = train.Problem(ctx, n_teacher=20_000, n_train=16, n_eval=4, size=(160, 120), seed=3)
    return ctx, pb


def host(g):
    return {k: getattr(g, k).cpu().numpy() for k in FIELDS}


@pytest.mark.parametrize("method", ["adpsplit", "vanilla"])
def test_densify_step_keeps_rows_and_moments(setup, method):
    ctx, pb = setup
    cfg = train.TrainConfig(method=method, iters=400, densify_from=100, densify_until=300, views_per_split=8, seed=5)
    tr = train.Trainer(ctx, pb, cfg, n_init=3000)
    for it in range(1, 151):
        tr.step(it)
    torch.cuda.synchronize()
    before, m_before = host(tr.g), host(tr.m)
    info = tr.densify(150)
    torch.cuda.synchronize()
    say("%s: %s" % (method, info))
    st = tr.last_state_map.cpu().numpy()
    after, m_after = host(tr.g), host(tr.m)
    assert len(st) == tr.g.n == info["n_after"]
    assert info["candidates"] > 0 and info["n_after"] != info["n_before"]
    kept = st >= 0
    assert len(np.unique(st[kept])) == kept.sum()           # a state row is carried at most once
    for k in FIELDS:
        np.testing.assert_array_equal(after[k][..., kept], before[k][..., st[kept]], err_msg=k)
        np.testing.assert_array_equal(m_after[k][..., kept], m_before[k][..., st[kept]], err_msg=k)
        assert (m_after[k][..., ~kept] == 0).all()
    # new rows: the clones plus the split's rows, less any pruned
    assert (~kept).sum() <= info["clones"] + 19 * info["candidates"] + 2 * info["candidates"]


@pytest.mark.parametrize("method", ["adpsplit", "vanilla"])
def test_short_training_improves_psnr(setup, method):
    ctx, pb = setup
    cfg = train.TrainConfig(method=method, iters=400, densify_from=100, densify_until=300, views_per_split=8,
                            eval_every=200, seed=6)
    tr = train.Trainer(ctx, pb, cfg, n_init=3000)
    res = tr.run()
    say("%s: %s" % (method, {k: v for k, v in res.items() if k != "history"}))
    h = res["history"]
    assert h[-1]["psnr"] > h[0]["psnr"] + 1.0
    assert res["final_n"] > 3000 and res["densify_calls"] == 3
