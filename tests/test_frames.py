"""Host-side block-list marshalling: frame partitions to ta_block descriptors
(offsets, strides, log2 sizes, axis ids) and the rules the batched kernels
rely on (vector alignment of offsets and strides, axis ids in the table)."""

import numpy as np

import synth
import paper_2505_23618_amd as ta
from paper_2505_23618_amd.frames import SIZES, axis_id, descriptors


def small():
    return synth.frames_workload(nframes=2, width=448, height=200, seed=30)


def test_descriptors_address_each_block():
    frames, rows = small()
    nf, fh, fw = frames.shape
    d = descriptors(rows, fh, fw)
    assert d.dtype == ta.BLOCK_DTYPE and d.dtype.itemsize == 32 and len(d) == len(rows)
    for i in np.random.Generator(np.random.PCG64(1)).choice(len(rows), 50, replace=False):
        f, x, y, w, h, th, tv = (int(v) for v in rows[i])
        assert d["in_off"][i] == d["out_off"][i] == (f * fh + y) * fw + x
        assert d["in_stride"][i] == d["out_stride"][i] == fw
        assert (1 << int(d["log2w"][i]), 1 << int(d["log2h"][i])) == (w, h)
        assert d["axis_h"][i] == axis_id(th, w) and d["axis_v"][i] == axis_id(tv, h)
        # the block, read through the descriptor, is the frame's block
        flat = frames.reshape(-1)
        blk = np.stack([flat[d["in_off"][i] + r * fw: d["in_off"][i] + r * fw + w] for r in range(h)])
        assert (blk == frames[f, y:y + h, x:x + w]).all()


def test_descriptors_meet_the_vector_alignment_rule():
    frames, rows = small()
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    ch = np.where(d["log2w"] >= 3, 8, 4)
    assert (d["in_off"] % ch == 0).all() and (d["out_off"] % ch == 0).all()
    assert (d["in_stride"] % ch == 0).all() and (d["in_stride"] >= (1 << d["log2w"].astype(int))).all()


def test_workload_has_every_size_and_kind_mix():
    _, rows = small()
    assert len({(int(w), int(h)) for w, h in rows[:, 3:5]}) == 25
    assert set(np.unique(rows[:, 5:7])) == {0, 1, 2}


def test_axis_ids_are_distinct_and_inside_the_table():
    ids = {axis_id(t, n) for t in (0, 1, 2) for n in SIZES}
    assert len(ids) == 15 and max(ids) < 256 and min(ids) >= 0
