"""Pins of the block-list backward oracle (oracle/blockgrad.py): angle and
input gradients against FP64 central differences of L = sum_b <G_Y, Y_b>, a
set that no axis uses has a zero gradient, and two axes on one set add."""

import numpy as np
import pytest

from oracle import adjust as OA
from oracle import blockgrad as BG


def _workload(aset, seed, n_blocks=5):
    """Blocks of several sizes whose axes mix: the angle set (plain and
    flipped, rows and columns), a fixed band, and plain bases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = aset.n
    other = OA.band_matrix(8, 2, rng.uniform(-0.5, 0.5, OA.n_angles(8, 2)))
    use = BG.AxisUse("S3" if aset.kind == "band" else "C2", aset.kind, False, True)
    use_f = BG.AxisUse(use.base, aset.kind, True, True)
    shapes_axes = [
        ((n, n), (use, use_f)),                           # rows on the set, columns on its flip
        ((8, n), (use_f, BG.AxisUse("S3", "band", False, False, a=other))),
        ((4, n), (BG.AxisUse("C2"), use)),
        ((4, 8), (BG.AxisUse("S7"), BG.AxisUse("C8", flip=True))),   # no use of the set
        ((n, n), (BG.AxisUse("S2"), use_f)),
    ][:n_blocks]
    blocks, axes, gys = [], [], []
    for (w, h), ax in shapes_axes:
        blocks.append(rng.standard_normal((h, w)))
        gys.append(rng.standard_normal((h, w)))
        axes.append(ax)
    return blocks, axes, gys


def _loss(blocks, axes, gys, aset):
    return sum(float(np.sum(g * y)) for g, y in zip(gys, BG.forward(blocks, axes, aset)))


SETS = [
    BG.AngleSet("band", 8, np.random.Generator(np.random.PCG64(1)).uniform(-0.6, 0.6, OA.n_angles(8, 2)), taps=4),
    BG.AngleSet("band", 8, np.random.Generator(np.random.PCG64(2)).uniform(-0.6, 0.6, OA.n_angles(8, 3)), taps=6),
    BG.AngleSet("post", 8, np.random.Generator(np.random.PCG64(3)).uniform(-0.6, 0.6, 6), b=4,
                q0=OA.rotation_product(4, np.random.Generator(np.random.PCG64(4)).uniform(-1, 1, 6))),
]


@pytest.mark.parametrize("aset", SETS, ids=["band4", "band6", "post4"])
def test_angle_gradient_matches_central_differences(aset):
    blocks, axes, gys = _workload(aset, seed=10)
    _, g = BG.backward(blocks, axes, gys, aset)
    h = 1e-6
    fd = np.empty_like(aset.angles)
    for r in range(len(aset.angles)):
        up, dn = aset.angles.copy(), aset.angles.copy()
        up[r] += h
        dn[r] -= h
        fd[r] = (_loss(blocks, axes, gys, BG.AngleSet(**{**aset.__dict__, "angles": up})) -
                 _loss(blocks, axes, gys, BG.AngleSet(**{**aset.__dict__, "angles": dn}))) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


@pytest.mark.parametrize("aset", SETS[:1] + SETS[2:], ids=["band4", "post4"])
def test_input_gradient_matches_central_differences(aset):
    blocks, axes, gys = _workload(aset, seed=11)
    gxs, _ = BG.backward(blocks, axes, gys, aset)
    h = 1e-6
    for k, x in enumerate(blocks):
        for (i, j) in ((0, 0), (x.shape[0] - 1, x.shape[1] - 1), (x.shape[0] // 2, 1)):
            up = [b.copy() for b in blocks]
            dn = [b.copy() for b in blocks]
            up[k][i, j] += h
            dn[k][i, j] -= h
            fd = (_loss(up, axes, gys, aset) - _loss(dn, axes, gys, aset)) / (2 * h)
            assert abs(gxs[k][i, j] - fd) <= 1e-7 * max(1.0, abs(fd))


def test_unused_set_has_zero_gradient():
    aset = SETS[0]
    blocks, axes, gys = _workload(aset, seed=12)
    _, g = BG.backward(blocks[3:4], axes[3:4], gys[3:4], aset)
    assert np.all(g == 0.0)


def test_two_axes_on_one_set_add():
    aset = SETS[0]
    rng = np.random.Generator(np.random.PCG64(13))
    x, gy = rng.standard_normal((8, 8)), rng.standard_normal((8, 8))
    use = BG.AxisUse("S3", "band", False, True)
    fixed = BG.AxisUse("S3", "band", False, False, a=aset.matrix())
    _, both = BG.backward([x], [(use, use)], [gy], aset)
    _, rows = BG.backward([x], [(use, fixed)], [gy], aset)
    _, cols = BG.backward([x], [(fixed, use)], [gy], aset)
    assert np.allclose(both, rows + cols, rtol=0, atol=1e-12)
