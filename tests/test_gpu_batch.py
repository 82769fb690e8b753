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
    assert bool(torch.isnan(ob).all())
    ref = ig.Filter(a.shape, **kw).run(xa)
    torch.cuda.synchronize()
    assert torch.equal(ref, oa)
    # without statistics the call does not wait; the NaN output carries the failure
    oa2, ob2 = torch.empty_like(xa), torch.zeros_like(xb)
    ig.batch([(xa, oa2, kw), (xb, ob2, kw)])
    torch.cuda.synchronize()
    assert bool(torch.isnan(ob2).all()) and torch.equal(oa2, ref)
    ig.batch_cache_clear()


# --- LDS-resident cubes -------------------------------------------------------
RES_SHAPES = [(32, 32, 32), (33, 32, 32), (1, 1, 40), (40, 1, 1), (1, 1, 1), (3, 1, 200), (17, 23, 29),
              (8, 128, 32), (2, 2, 256)]


@pytest.mark.parametrize("cond", ["pm_exp", "pm_rational", "intensity"])
def test_resident_bitwise_equal_to_streamed(dev, oracle_lib, cond):
    """A batch of small cubes gives the same bits with the LDS-resident path
    as with the streamed passes; the oracle agrees; stats say which ran."""
    import torch
    import paper_1609_03782_amd as ig
    rng = np.random.default_rng(7)
    cubes, items = [], []
    for k, shape in enumerate(RES_SHAPES):
        c = igsynth.random_cube(shape, seed=300 + k, scale=1.5)
        c.flat[rng.integers(c.size)] = 8.0
        n_iter = int(rng.integers(1, 13))
        K = float(rng.uniform(1.5, 3.0))
        x = torch.from_numpy(c).to(dev)
        kw = dict(K=K, tau=1 / 16 if cond != "intensity" else 0.0325, n_iter=n_iter,
                  C=(1.0, 1.0, 1.0) if cond != "intensity" else (5.0, 5.0, 5.0), cond=cond)
        cubes.append((c, kw))
        items.append((x, torch.empty_like(x), kw))
    outs = {}
    try:
        for lim in (32768, 0):
            ig.batch_set_resident(lim)
            assert ig.batch_get_resident() == lim
            res = ig.batch(items, want_stats=True, want_latency=True)
            torch.cuda.synchronize()
            outs[lim] = [o.clone() for _, o, _ in items]
            for (c, kw), st, lat in zip(cubes, res["stats"], res["latency_ms"]):
                resident = lim > 0 and c.size <= lim
                if resident:
                    assert st.passes == 1 and st.schedule["t_block"] == kw["n_iter"]
                    waves = 1
                    while waves < 16 and 64 * waves * 32 < c.size:
                        waves *= 2
                    assert st.schedule["waves"] == waves, (c.shape, st.schedule)
                assert lat > 0.0
    finally:
        ig.batch_set_resident(32768)
        ig.batch_cache_clear()
    for (c, kw), a, b in zip(cubes, outs[32768], outs[0]):
        assert torch.equal(a, b), (c.shape, kw["n_iter"])
        ref, rho = oracle_lib.run(c, cond, K=kw["K"], tau=kw["tau"], n_iter=kw["n_iter"], C=kw["C"])
        err = float(np.abs(a.cpu().numpy().astype(np.float64) - ref).max())
        assert err <= TOL * rho, (c.shape, err / rho)


def test_resident_in_place_and_mixed_batch(dev):
    """In-place resident cubes next to streamed ones of the same batch, against
    single-cube runs (bitwise); a zero-iteration small cube is copied."""
    import torch
    import paper_1609_03782_amd as ig
    shapes = [(16, 16, 16), (24, 70, 90), (30, 30, 30), (10, 10, 10)]
    cubes, items = [], []
    for k, shape in enumerate(shapes):
        c = igsynth.random_cube(shape, seed=400 + k, scale=1.5)
        x = torch.from_numpy(c).to(dev)
        n_iter = 0 if k == 3 else 9
        out = x if k == 0 else torch.empty_like(x)
        kw = dict(K=2.0, tau=1 / 16, n_iter=n_iter)
        cubes.append((c, kw))
        items.append((x, out, kw))
    res = ig.batch(items, want_stats=True)
    torch.cuda.synchronize()
    for (c, kw), (x, out, _), st in zip(cubes, items, res["stats"]):
        single = ig.Filter(c.shape, **kw)
        ys = single.run(torch.from_numpy(c).to(dev))
        torch.cuda.synchronize()
        assert torch.equal(ys, out), c.shape
        assert st.sum_out == pytest.approx(float(ys.double().sum()), rel=1e-9, abs=1e-6)
    assert res["stats"][0].passes == 1 and res["stats"][2].passes == 1
    assert res["stats"][1].passes > 1 and res["stats"][3].passes == 0
    ig.batch_cache_clear()


def test_resident_graph_replay_bitwise(dev):
    import torch
    import paper_1609_03782_amd as ig
    items = []
    for k in range(6):
        c = igsynth.random_cube((20 + k, 21, 22), seed=500 + k, scale=1.5)
        x = torch.from_numpy(c).to(dev)
        items.append((x, torch.empty_like(x), dict(K=2.0, tau=1 / 16, n_iter=15 + k)))
    ig.batch(items)
    torch.cuda.synchronize()
    first = [o.clone() for _, o, _ in items]
    for rep in range(3):
        for _, o, _ in items:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        ig.batch(items)
        torch.cuda.synchronize()
        for a, (_, o, _) in zip(first, items):
            assert torch.equal(a, o), rep
    ig.batch_cache_clear()


def test_batch_changed_parameters_or_settings_rebuild(dev):
    """Repeated calls with identical items reuse the last plan; a changed
    parameter or batch setting on the same tensors must not (each result is
    checked against single-cube runs)."""
    import torch
    import paper_1609_03782_amd as ig
    shapes = [(12, 13, 14), (40, 50, 60)]
    xs = [torch.from_numpy(igsynth.random_cube(s, seed=600 + k, scale=1.5)).to(dev) for k, s in enumerate(shapes)]
    outs = [torch.empty_like(x) for x in xs]
    try:
        for n_iter, K, res_lim, T in [(5, 2.0, 32768, 0), (5, 2.0, 32768, 0), (6, 2.0, 32768, 0),
                                      (6, 2.5, 32768, 0), (6, 2.5, 0, 0), (6, 2.5, 0, 3)]:
            ig.batch_set_resident(res_lim)
            ig.batch_set_schedule(T, 16, 32)
            kw = dict(K=K, tau=1 / 16, n_iter=n_iter)
            prep = ig.batch_prepare([(x, o, kw) for x, o in zip(xs, outs)])
            ig.batch(prep)
            ig.batch(prep)
            torch.cuda.synchronize()
            for x, o in zip(xs, outs):
                ref = ig.Filter(tuple(x.shape), **kw).run(x)
                torch.cuda.synchronize()
                assert torch.equal(ref, o), (tuple(x.shape), n_iter, K, res_lim, T)
    finally:
        ig.batch_set_resident(32768)
        ig.batch_set_schedule(0, 16, 32)
        ig.batch_cache_clear()


def test_batch_fresh_buffers_reuse_plan_and_cache_stays_bounded(dev):
    """A serving loop that hands in new output (and input) tensors on every
    call reuses the plan of that shape signature, with its buffer table
    rewritten; results stay bitwise those of single-cube runs, and the cache
    never holds more than 8 plans however many signatures pass through."""
    import torch
    import paper_1609_03782_amd as ig
    ig.batch_cache_clear()
    shapes = [(10, 21, 33), (24, 40, 72)]
    kw = dict(K=2.0, tau=1 / 16, n_iter=5)
    cubes = [igsynth.random_cube(s, seed=700 + k, scale=1.5) for k, s in enumerate(shapes)]
    refs = [ig.Filter(c.shape, **kw).run(torch.from_numpy(c).to(dev)) for c in cubes]
    torch.cuda.synchronize()
    keep = []
    for call in range(6):
        xs = [torch.from_numpy(c).to(dev) for c in cubes]     # fresh input and output tensors
        outs = [torch.full_like(x, float(call)) for x in xs]
        keep.append((xs, outs))                                # distinct addresses every call
        ig.batch([(x, o, kw) for x, o in zip(xs, outs)])
        assert ig.batch_cache_size() == 1
    torch.cuda.synchronize()
    for xs, outs in keep:
        for o, r in zip(outs, refs):
            assert torch.equal(o, r)
    # eleven signatures (n_iter 1..11) through an 8-plan cache
    ig.batch_cache_clear()
    x = torch.from_numpy(cubes[0]).to(dev)
    for n in range(1, 12):
        o = torch.empty_like(x)
        ig.batch([(x, o, dict(K=2.0, tau=1 / 16, n_iter=n))])
        assert ig.batch_cache_size() == min(n, 8)
        torch.cuda.synchronize()
        assert torch.equal(o, ig.Filter(tuple(x.shape), K=2.0, tau=1 / 16, n_iter=n).run(x)), n
    ig.batch_cache_clear()
    assert ig.batch_cache_size() == 0


# --- persistent launch ----------------------------------------------------------
@pytest.mark.parametrize("t_block,waves,zchunk", [(1, 8, 16), (2, 16, 7), (3, 12, 32)])
def test_persistent_launch_bitwise_equal_to_rounds(dev, t_block, waves, zchunk):
    """One persistent launch (workgroups take items from a device counter and
    wait for the cube's previous pass) gives bitwise the output of one launch
    per round, for in-place and out-of-place items, with latencies and
    statistics filled and graph replays repeating the bytes."""
    import torch
    import paper_1609_03782_amd as ig
    ig.batch_set_schedule(t_block, waves, zchunk)
    ig.batch_set_resident(0)
    try:
        outs = {}
        for persistent in (False, True):
            ig.batch_set_launch(persistent)
            assert ig.batch_get_launch() == persistent
            cubes, items = _items(dev, seed=7)
            res = ig.batch(items, want_stats=True, want_latency=True)
            torch.cuda.synchronize()
            outs[persistent] = [out.clone() for _, out, _ in items]
            assert all(lat >= 0.0 for lat in res["latency_ms"])
            for (c, n_iter, K, inplace), st in zip(cubes, res["stats"]):
                assert st.nonfinite == 0
            if persistent:   # graph replays on fresh buffers (in-place items: fresh inputs each time)
                for _ in range(2):
                    _, items2 = _items(dev, seed=7)
                    for x, out, _ in items2:
                        if out.data_ptr() != x.data_ptr():
                            out.fill_(-1.0)
                    ig.batch(items2)
                    torch.cuda.synchronize()
                    for a, (_, out, _) in zip(outs[True], items2):
                        assert torch.equal(a, out)
        for a, b in zip(outs[False], outs[True]):
            assert torch.equal(a, b)
    finally:
        ig.batch_set_launch(False)
        ig.batch_set_schedule(0, 16, 32)
        ig.batch_set_resident(32768)
        ig.batch_cache_clear()


def test_persistent_launch_nonfinite_item(dev):
    """A cube with a NaN voxel under the persistent launch: its pieces run
    nothing but are counted, so the other cubes' passes still complete."""
    import torch
    import paper_1609_03782_amd as ig
    ig.batch_set_launch(True)
    ig.batch_set_resident(0)
    try:
        a = igsynth.random_cube((8, 30, 40), seed=1)
        b = igsynth.random_cube((9, 20, 30), seed=2)
        b[2, 3, 4] = np.nan
        xa, xb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
        oa, ob = torch.empty_like(xa), torch.full_like(xb, 3.0)
        kw = dict(K=2.0, tau=1 / 16, n_iter=9)
        with pytest.raises(ig.IgError) as ei:
            ig.batch([(xb, ob, kw), (xa, oa, kw)], want_stats=True)
        assert ei.value.status == ig.IG_ERR_NONFINITE
        torch.cuda.synchronize()
        assert bool(torch.isnan(ob).all())
        ref = ig.Filter(a.shape, **kw).run(xa)
        torch.cuda.synchronize()
        assert torch.equal(ref, oa)
    finally:
        ig.batch_set_launch(False)
        ig.batch_set_resident(32768)
        ig.batch_cache_clear()
