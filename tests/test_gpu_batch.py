"""GPU checks of the batched graph launch (ig_filter_batch): every item
matches the FP64 oracle, equals the single-cube run bitwise, graph replays give
the same bytes, and per-item statistics and latencies are filled."""
import numpy as np
import pytest

import igsynth

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_03782_amd as ig
    ig.lib()
    return torch.device("cuda:0")


SHAPES = [(7, 9, 11), (33, 32, 32), (20, 45, 70), (12, 90, 130), (5, 17, 256), (40, 3, 64), (1, 1, 1),
          (16, 64, 40)]


def _items(dev, seed=0):
    import torch
    rng = np.random.default_rng(seed)
    cubes, items = [], []
    for k, shape in enumerate(SHAPES):
        c = igsynth.random_cube(shape, seed=100 + k + seed, scale=1.5)
        c.flat[rng.integers(c.size)] = 9.0
        n_iter = int(rng.integers(0, 10))
        K = float(rng.uniform(1.5, 3.0))
        x = torch.from_numpy(c).to(dev)
        inplace = (k % 3 == 2)
        out = x if inplace else torch.empty_like(x)
        cubes.append((c, n_iter, K, inplace))
        items.append((x, out, dict(K=K, tau=1 / 16, n_iter=n_iter, C=(1.0, 1.0, 1.0), cond="pm_exp")))
    return cubes, items


@pytest.mark.parametrize("t_block,waves,zchunk", [(0, 16, 32), (1, 8, 7), (2, 16, 64), (3, 8, 13), (4, 16, 32),
                                                  (2, 12, 5)])
def test_batch_matches_oracle_and_single_runs(dev, oracle_lib, t_block, waves, zchunk):
    import torch
    import paper_1609_03782_amd as ig
    ig.batch_set_schedule(t_block, waves, zchunk)
    try:
        cubes, items = _items(dev)
        res = ig.batch(items, want_stats=True, want_latency=True)
        torch.cuda.synchronize()
        for (c, n_iter, K, inplace), (x, out, kw), st, lat in zip(cubes, items, res["stats"], res["latency_ms"]):
            ref, rho = oracle_lib.run(c, "pm_exp", K=K, tau=1 / 16, n_iter=n_iter)
            y = out.cpu().numpy()
            err = float(np.abs(y.astype(np.float64) - ref).max())
            assert err <= TOL * rho, (c.shape, n_iter, err / rho)
            assert st.rms_used == pytest.approx(rho, rel=1e-12)
            assert st.sum_out == pytest.approx(float(y.astype(np.float64).sum()), rel=1e-9, abs=1e-6)
            assert lat >= 0.0
            single = ig.Filter(c.shape, K=K, tau=1 / 16, n_iter=n_iter, cond="pm_exp")
            single.set_schedule("naive")
            ys = single.run(torch.from_numpy(c).to(dev))
            torch.cuda.synchronize()
            assert np.array_equal(ys.cpu().numpy(), y), (c.shape, n_iter)
    finally:
        ig.batch_set_schedule(0, 16, 32)
        ig.batch_cache_clear()


def test_batch_graph_replay_bitwise(dev):
    import torch
    import paper_1609_03782_amd as ig
    _, items = _items(dev, seed=5)
    items = [(x, out, kw) for (x, out, kw) in items if out.data_ptr() != x.data_ptr()]
    ig.batch(items)
    torch.cuda.synchronize()
    first = [out.clone() for _, out, _ in items]
    for _, out, _ in items:
        out.fill_(-1.0)
    for _ in range(3):
        ig.batch(items)                   # cached plan: graph replay
    torch.cuda.synchronize()
    for a, (_, out, _) in zip(first, items):
        assert torch.equal(a, out)
    ig.batch_cache_clear()


def test_batch_nonfinite_item(dev):
    import torch
    import paper_1609_03782_amd as ig
    a = igsynth.random_cube((8, 8, 8), seed=1)
    b = igsynth.random_cube((8, 9, 10), seed=2)
    b[2, 3, 4] = np.nan
    xa, xb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    oa, ob = torch.empty_like(xa), torch.full_like(xb, 3.0)
    kw = dict(K=2.0, tau=1 / 16, n_iter=4)
    with pytest.raises(ig.IgError) as ei:
        ig.batch([(xa, oa, kw), (xb, ob, kw)], want_stats=True)
    assert ei.value.status == ig.IG_ERR_NONFINITE
    torch.cuda.synchronize()
    assert bool((ob == 3.0).all())
    ref = ig.Filter(a.shape, **kw).run(xa)
    torch.cuda.synchronize()
    assert torch.equal(ref, oa)
    ig.batch_cache_clear()
