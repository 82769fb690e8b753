"""Host-only checks of the work split of the streaming kernel: for many
shapes and schedules the pieces of a pass cover every output voxel exactly
once, stay inside the cube, and (balanced split) come in whole rounds of
nearly equal work."""
import numpy as np
import pytest

import paper_1609_03782_amd as ig

SHAPES = [(512, 512, 512), (32, 64, 64), (13, 37, 70), (5, 3, 300), (1, 1, 1), (160, 256, 256), (7, 600, 33),
          (40, 2, 3), (97, 1, 1031)]
SCHEDS = [dict(t_block=2, waves=16), dict(t_block=1, waves=16), dict(t_block=2, waves=16, rounds=3),
          dict(t_block=3, waves=9), dict(t_block=2, waves=8, zchunk=7), dict(t_block=4, waves=10, vec=1),
          dict(t_block=1, waves=3, vec=2, zchunk=1)]


def tile_rows(g, ny, k):
    """Rows [y0, y1) that y tile k outputs (the even split the header states)."""
    return k * ny // g["nty"], (k + 1) * ny // g["nty"]


def tile_cols(g, nx, k):
    """Columns [x0, x1) that x tile k outputs: starts at k nx / ntx rounded
    up to whole lane chunks, the last tile ends at nx."""
    q = g["ntx"] * g["V"]
    start = lambda i: nx if i == g["ntx"] else g["V"] * -(-(i * nx) // q)
    return start(k), start(k + 1)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("sched", SCHEDS)
def test_pieces_cover_every_output_once(shape, sched):
    nz, ny, nx = shape
    for T in range(1, sched["t_block"] + 1):
        why = ig.schedule_check(shape, dict(kind="blocked", **sched), n_iter=sched["t_block"])
        if why is not None:
            continue
        g, pcs = ig.schedule_plan(shape, dict(kind="blocked", **sched), T)
        assert g["pieces"] == len(pcs) > 0
        # the x and y tiles partition the columns and rows ...
        for part, n in (([tile_cols(g, nx, k) for k in range(g["ntx"])], nx),
                        ([tile_rows(g, ny, k) for k in range(g["nty"])], ny)):
            assert part[0][0] == 0 and part[-1][1] == n and all(a[1] == b[0] for a, b in zip(part, part[1:]))
        # ... and each tile's pieces partition its planes
        zs = {}
        for tx, ty, z0, z1 in pcs:
            assert 0 <= tx < g["ntx"] and 0 <= ty < g["nty"] and 0 <= z0 < z1 <= nz
            (x0, x1), (y0, y1) = tile_cols(g, nx, tx), tile_rows(g, ny, ty)
            assert 0 <= x0 < x1 <= nx and x1 - x0 <= g["ox"] and x0 % g["V"] == 0
            assert 0 <= y0 < y1 <= ny and y1 - y0 <= g["oy"]
            zs.setdefault((int(tx), int(ty)), []).append((int(z0), int(z1)))
        assert len(zs) == g["ntx"] * g["nty"], (shape, sched, T)
        for iv in zs.values():
            iv.sort()
            assert iv[0][0] == 0 and iv[-1][1] == nz and all(a[1] == b[0] for a, b in zip(iv, iv[1:])), \
                (shape, sched, T)
        if nz * ny * nx <= 1 << 22:   # the same by counting every voxel
            cover = np.zeros(shape, np.int32)
            for tx, ty, z0, z1 in pcs:
                (x0, x1), (y0, y1) = tile_cols(g, nx, tx), tile_rows(g, ny, ty)
                cover[z0:z1, y0:y1, x0:x1] += 1
            assert cover.min() == 1 and cover.max() == 1, (shape, sched, T)
        if g["ntx"] == 1:
            assert 64 // g["rows"] * g["V"] >= nx
        if g["nty"] == 1:
            assert g["waves"] * g["rows"] >= ny


def test_balanced_split_whole_rounds():
    g, pcs = ig.schedule_plan((512, 512, 512), dict(kind="blocked", t_block=2, waves=12), 2, ncu=256)
    assert len(pcs) % 256 == 0
    vol = []
    for tx, ty, z0, z1 in pcs:
        y0, y1 = tile_rows(g, 512, ty)
        vol.append((y1 - y0) * (z1 - z0))
    vol = np.array(vol)
    assert vol.max() <= 1.1 * vol.mean()          # equal work per piece (within 10 %)
    # each eighth of the table (one XCD) is a contiguous band of z
    per = len(pcs) // 8
    for j in range(8):
        zs = pcs[j::8][:, 2]
        assert zs.max() - zs.min() < 512 // 2


def test_vec_never_exceeds_nx():
    """A lane's chunk never reaches past the row: explicit vec > nx is
    rejected, the automatic layout takes 1 or 2 voxels per lane below nx = 4."""
    for nx, want in [(1, 1), (2, 2), (3, 2), (4, 4), (5, 4)]:
        g, _ = ig.schedule_plan((3, 5, nx), dict(kind="blocked", t_block=1, waves=4), 1)
        assert g["V"] == want, (nx, g)
    assert ig.schedule_check((3, 5, 3), dict(kind="blocked", t_block=1, waves=4, vec=4), n_iter=1) is not None
    assert ig.schedule_check((3, 5, 8), dict(kind="blocked", t_block=1, waves=4, vec=8), n_iter=1) is None


def test_x_tiles_start_at_whole_lane_chunks():
    """Cubes wider than one tile: tile origins (output start minus the halo)
    are multiples of vec, the halo covers t_block, and vector I/O is used
    exactly when nx is a multiple of vec."""
    for nx in (600, 1037, 1040, 2048):
        for V in (2, 4, 8):
            for T in (1, 2, 3, 4):
                s = dict(kind="blocked", t_block=T, waves=12, vec=V)
                if ig.schedule_check((2, 30, nx), s, n_iter=T) is not None:
                    continue
                g, _ = ig.schedule_plan((2, 30, nx), s, T)
                if g["ntx"] == 1:
                    continue
                hx = (64 * V - g["ox"]) // 2
                assert hx >= T and hx % V == 0 and g["ox"] % V == 0, (nx, V, T, g)
                assert g["vec_io"] == (1 if nx % V == 0 else 0), (nx, V, T, g)


def test_automatic_layout_by_width():
    for nx, want in [(200, 4), (300, 8), (512, 8), (513, 4), (1024, 4), (4096, 4)]:
        g, _ = ig.schedule_plan((2, 30, nx), dict(kind="blocked", t_block=2, waves=12), 2)
        assert g["V"] == want, (nx, g)


def test_rows_too_long_for_blocked_schedule():
    # a tile's rows of one plane must stay below 2^30 bytes (32-bit offsets)
    why = ig.schedule_check((1, 1, 1 << 24), dict(kind="blocked", t_block=1, waves=16, vec=8), n_iter=1)
    assert why is not None and "too long" in why


def test_even_tile_split():
    """Tiles share the rows and columns evenly: y tiles differ by at most one
    row, x tiles by at most one lane chunk (the last may be shorter by the
    row's ragged end), none exceeds the tile's output extent, and together
    they cover the row once; near-worst cases (n just below a multiple of the
    extent) included."""
    for nx in (600, 991, 992, 993, 1037, 1480, 1489, 2048, 4095):
        for V in (2, 4, 8):
            for T in (1, 2, 4):
                s = dict(kind="blocked", t_block=T, waves=12, vec=V)
                if ig.schedule_check((2, 30, nx), s, n_iter=T) is not None:
                    continue
                g, _ = ig.schedule_plan((2, 30, nx), s, T)
                w = [tile_cols(g, nx, i) for i in range(g["ntx"])]
                assert w[0][0] == 0 and w[-1][1] == nx
                assert all(a[1] == b[0] for a, b in zip(w, w[1:]))
                widths = [b - a for a, b in w]
                assert max(widths) <= g["ox"] and min(widths) > 0, (nx, V, T, g)
                assert max(widths[:-1] or widths) - min(widths[:-1] or widths) <= V
    for ny in (13, 100, 499, 500, 511, 512, 513, 1000):
        for waves, T in ((12, 2), (14, 2), (10, 2), (16, 1), (9, 3)):
            s = dict(kind="blocked", t_block=T, waves=waves)
            if ig.schedule_check((2, ny, 64), s, n_iter=T) is not None:
                continue
            g, _ = ig.schedule_plan((2, ny, 64), s, T)
            h = [tile_rows(g, ny, j) for j in range(g["nty"])]
            assert h[0][0] == 0 and h[-1][1] == ny and all(a[1] == b[0] for a, b in zip(h, h[1:]))
            rows = [b - a for a, b in h]
            assert max(rows) <= g["oy"] and max(rows) - min(rows) <= 1, (ny, waves, T, g)


def _wg_costs(shape, sched):
    """Steps each workgroup of the pass runs: per piece its planes plus the
    3 t_block of the pipeline refill."""
    T = sched["t_block"]
    sd = dict(kind="blocked", **sched)
    g, pcs = ig.schedule_plan(shape, sd, T, ncu=256)
    first = ig.schedule_plan_groups(shape, sd, T, ncu=256)
    if first is None:
        first = np.arange(len(pcs) + 1)
    cost = np.array([sum(int(z1 - z0) + 3 * T for _, _, z0, z1 in pcs[first[b]:first[b + 1]])
                     for b in range(len(first) - 1)])
    return g, pcs, first, cost


def test_ragged_shapes_balance_in_one_round():
    """Whole rounds of workgroups, and no workgroup much longer than the average:
    a thin last tile used to get a single piece of all nz planes that
    outlasted every other piece, and tile counts that do not divide the
    workgroups (43 tiles of 16-wave workgroups over 256) left some tiles with
    fewer, longer pieces; workgroups now take equal shares of the
    (tile, plane) sequence in that case."""
    for shape, sched in [((512, 512, 512), dict(t_block=2, waves=14)), ((500, 500, 500), dict(t_block=2, waves=12)),
                         ((512, 512, 512), dict(t_block=1, waves=12)), ((512, 512, 512), dict(t_block=2, waves=10)),
                         ((512, 500, 512), dict(t_block=2, waves=16)), ((512, 512, 512), dict(t_block=2, waves=16))]:
        g, pcs, first, cost = _wg_costs(shape, sched)
        tiles = g["ntx"] * g["nty"]
        assert len(first) - 1 <= 256 * max(1, -(-tiles // 256)), (shape, sched)   # whole rounds
        T = sched["t_block"]
        assert cost.max() <= 1.08 * cost.mean() + 3 * T, (shape, sched, cost.max(), cost.mean())


def test_grouped_plan_partitions_the_sequence():
    """A grouped plan: the workgroups' ranges partition the piece list, each
    workgroup's pieces are consecutive in (tile, plane) order (at most one
    tile boundary inside a share at these sizes), and the shares cost the
    same to within one refill."""
    for shape, sched in [((512, 512, 512), dict(t_block=2, waves=16)), ((512, 512, 512), dict(t_block=1, waves=16)),
                         ((64, 512, 512), dict(t_block=2, waves=16))]:
        g, pcs, first, cost = _wg_costs(shape, sched)
        assert ig.schedule_plan_groups(shape, dict(kind="blocked", **sched), sched["t_block"]) is not None
        assert first[0] == 0 and first[-1] == len(pcs) and (np.diff(first) >= 1).all()
        nz = shape[0]
        spans = [((ty * g["ntx"] + tx) * nz + z0, (ty * g["ntx"] + tx) * nz + z1) for tx, ty, z0, z1 in pcs]
        assert all(a < b for a, b in spans)
        assert all(p[1] <= q[0] for p, q in zip(spans, spans[1:]))    # sequence order, no overlap
        assert (np.diff(first) <= 2).all()
        T = sched["t_block"]
        assert cost.max() - cost.min() <= 3 * T + 1, (shape, sched, cost.min(), cost.max())




def test_grouping_only_where_it_pays():
    """Grouped plans only for passes of depth 1 and 2 on cubes one tile wide,
    and only when the one-piece split is unbalanced: the 512^3 cube keeps one
    piece per workgroup with 12 wavefronts (64 tiles x 4) and wide cubes keep
    their one-piece split."""
    assert ig.schedule_plan_groups((512, 512, 512), dict(kind="blocked", t_block=2, waves=12), 2) is None
    assert ig.schedule_plan_groups((128, 1024, 1024), dict(kind="blocked", t_block=2, waves=12), 2) is None
    assert ig.schedule_plan_groups((512, 512, 512), dict(kind="blocked", t_block=3, waves=10), 3) is None
    assert ig.schedule_plan_groups((512, 512, 512), dict(kind="blocked", t_block=2, waves=16), 2) is not None


def test_auto_schedule_takes_16_waves_for_fp32_only():
    """The default schedule of the 512^3 cube at T = 2: 16 wavefronts with a
    grouped plan for FP32 storage (its longest share is 93 plane steps of a
    16-wave workgroup against 134 of a 12-wave one), 12 wavefronts for 16-bit
    storage, where the 16-wave grouped pass measured slower."""
    assert ig.schedule_auto((512, 512, 512))["waves"] == 16
    for dt in ("bf16", "f16"):
        s = ig.schedule_auto((512, 512, 512), dtype=dt)
        assert s["waves"] == 12 and s["t_block"] == 2, (dt, s)
    # one step: no temporal blocking, no grouped 16-wave plan
    assert ig.schedule_auto((512, 512, 512), n_iter=1)["t_block"] == 1
