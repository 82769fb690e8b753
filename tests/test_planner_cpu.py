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
