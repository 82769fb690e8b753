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
        cover = np.zeros(shape, np.int32)
        for tx, ty, z0, z1 in pcs:
            assert 0 <= tx < g["ntx"] and 0 <= ty < g["nty"] and 0 <= z0 < z1 <= nz
            x0, y0 = tx * g["ox"], ty * g["oy"]
            assert x0 < nx and y0 < ny
            cover[z0:z1, y0:y0 + g["oy"], x0:x0 + g["ox"]] += 1
        assert cover.min() == 1 and cover.max() == 1, (shape, sched, T)
        if g["ntx"] == 1:
            assert 64 // g["rows"] * g["V"] >= nx
        if g["nty"] == 1:
            assert g["waves"] * g["rows"] >= ny


def test_balanced_split_whole_rounds():
    g, pcs = ig.schedule_plan((512, 512, 512), dict(kind="blocked", t_block=2, waves=16), 2, ncu=256)
    assert len(pcs) % 256 == 0
    vol = []
    for tx, ty, z0, z1 in pcs:
        rows = min(g["oy"], 512 - ty * g["oy"])
        vol.append(rows * (z1 - z0))
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
