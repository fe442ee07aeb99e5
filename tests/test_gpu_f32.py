"""GPU parity of the fp32 path against the FP64 oracle.

Tolerance (the reading of "within 1e-5 relative"): per block,
max |Y_gpu - Y_ref| <= 1e-5 * max |Y_ref|, with Y_ref the FP64 transform
computed from the same parameters; an all-zero reference requires exact
zeros.
"""

import numpy as np
import pytest

import synth
from oracle import fp as P
from tests.libcases import ALL_CASES, Registered

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32_CASES = ["cfg3_post16_64", "direct_dst7_64", "cfg2_dst7_k4", "cfg2_dct8_k4", "direct_dst7_32",
             "post8_32", "cfg1_dct2_band_16", "dst2_dct8_8x16"]
TOL = 1e-5


@pytest.fixture(scope="module")
def reg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Registered(0)


def _check(got, ref):
    err = np.abs(got.astype(np.float64) - ref).reshape(len(ref), -1).max(axis=1)
    scale = np.abs(ref).reshape(len(ref), -1).max(axis=1)
    zero = scale == 0
    assert (err[zero] == 0).all()
    rel = err[~zero] / scale[~zero]
    assert rel.max(initial=0.0) <= TOL, f"worst block rel err {rel.max():.3e}"
    return rel.max(initial=0.0)


@pytest.mark.parametrize("name", F32_CASES)
def test_f32_forward_inverse(reg, name):
    w, h = ALL_CASES[name][:2]
    ah, av = reg.axes[name]
    oh, ov = reg.oracle_axes(name)
    nb = 3 * (256 // max(w, h)) + 5
    print(f"f32 case {name} {w}x{h} nb={nb}", flush=True)
    rng = np.random.Generator(np.random.PCG64(31))
    sets = [synth.ar1_blocks(nb, h, w, 0.97, 12.0, seed=41).astype(np.float32),
            rng.standard_normal((nb, h, w)).astype(np.float32),
            np.zeros((2, h, w), np.float32)]
    for x in sets:
        xd = torch.from_numpy(x).cuda()
        y = reg.ctx.fwd(xd, ah, av)
        ref = P.fwd2d(x.astype(np.float64), oh, ov)
        _check(y.cpu().numpy(), ref)
        # inverse of the fp32 forward output
        yin = y.cpu().numpy()
        z = reg.ctx.inv(y, ah, av).cpu().numpy()
        _check(z, P.inv2d(yin.astype(np.float64), oh, ov))


def test_f32_full_size_sampled(reg):
    """64x64 sub-block workload at full size (65,536 blocks), sampled blocks."""
    x = synth.workload_blocks("cfg3_64x64").astype(np.float32)
    ah, av = reg.axes["cfg3_post16_64"]
    oh, ov = reg.oracle_axes("cfg3_post16_64")
    xd = torch.from_numpy(x).cuda()
    y = reg.ctx.fwd(xd, ah, av)
    z = reg.ctx.inv(y, ah, av)
    torch.cuda.synchronize()
    idx = np.concatenate([np.random.Generator(np.random.PCG64(5)).choice(len(x), 40, replace=False), [0, len(x) - 1]])
    it = torch.from_numpy(idx).cuda()
    ys = y[it].cpu().numpy()
    _check(ys, P.fwd2d(x[idx].astype(np.float64), oh, ov))
    _check(z[it].cpu().numpy(), P.inv2d(ys.astype(np.float64), oh, ov))
    # the roundtrip returns the input to fp32 precision
    assert np.abs(z[it].cpu().numpy() - x[idx]).max() < 1e-3
