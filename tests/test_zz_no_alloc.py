"""The allocation-free Givens backward (ta_givens_bwd_noalloc, for callers
that cannot allocate): called through the C ABI, its input gradient and
angle gradient equal those of ta_givens_bwd (caller's workspace) bit for
bit, on two calls in a row on the same device (the second with fewer
vectors, so it reads fewer of the static partial rows the first call left
behind), and both stay within the oracle tolerance (|dg|_inf <= 1e-4
|g|_inf against the FP64 gradient).  Sizes above the static capacity are
rejected before any launch."""

import ctypes

import numpy as np
import pytest

import synth
from oracle import refit as R

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402
from paper_2505_23618_amd import refit as RF  # noqa: E402


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _bwd(ctx, base, n, taps, th, x, gy, noalloc):
    m = x.shape[0]
    gx = torch.empty_like(x)
    gth = torch.empty_like(th)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = ta.lib()
    if noalloc:
        code = L.ta_givens_bwd_noalloc(ctx._h, base, n, taps, _p(th), m, _p(x), _p(gy), _p(gx), _p(gth), s)
    else:
        nbytes = ctypes.c_int64(0)
        assert L.ta_givens_workspace(m, ctypes.byref(nbytes)) == 0
        ws = torch.empty(max(nbytes.value, 4), dtype=torch.uint8, device=x.device)
        code = L.ta_givens_bwd(ctx._h, base, n, taps, _p(th), m, _p(x), _p(gy), _p(gx), _p(gth), _p(ws), s)
    assert code == 0, ta.lib().ta_last_error().decode()
    torch.cuda.synchronize()
    return gx, gth


@pytest.mark.parametrize("base,taps", [(ta.DCT2, 4), (ta.DST3, 6)])
def test_noalloc_backward_matches_workspace_backward(base, taps):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ta.Context(0)
    n = 32
    bname = {ta.DCT2: "C2", ta.DST3: "S3"}[base]
    rng = np.random.Generator(np.random.PCG64(31))
    th_np = rng.uniform(-0.5, 0.5, RF.n_angles(n, taps))
    th = torch.tensor(th_np, dtype=torch.float32, device="cuda")
    for m, seed in ((131072, 1), (5000 + 17, 2)):
        print(f"noalloc backward base {bname} taps {taps} vectors {m}", flush=True)
        x_np = synth.ar1_vectors(m, n, 0.85, 0.99, 1.0, seed=synth.SEED_BASE + 40 + seed)
        gy_np = np.random.Generator(np.random.PCG64(50 + seed)).standard_normal((m, n))
        x = torch.tensor(x_np, dtype=torch.float32, device="cuda")
        gy = torch.tensor(gy_np, dtype=torch.float32, device="cuda")
        gx_a, gth_a = _bwd(ctx, base, n, taps, th, x, gy, noalloc=True)
        gx_w, gth_w = _bwd(ctx, base, n, taps, th, x, gy, noalloc=False)
        assert torch.equal(gx_a, gx_w)
        assert torch.equal(gth_a, gth_w)
        dx, dth = R.backward(th_np, x_np, gy_np, base=bname, n=n, layers=taps // 2)
        assert np.abs(gx_a.cpu().numpy() - dx).max() <= 1e-4 * np.abs(dx).max()
        assert np.abs(gth_a.cpu().numpy() - dth).max() <= 1e-4 * np.abs(dth).max()


def test_noalloc_backward_rejects_too_many_vectors():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ta.Context(0)
    th = torch.zeros(31, dtype=torch.float32, device="cuda")
    x = torch.zeros((4, 32), dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = ta.lib().ta_givens_bwd_noalloc(ctx._h, ta.DCT2, 32, 4, _p(th), 4096 * 256 + 1, _p(x), _p(x), _p(x),
                                          _p(th), s)
    assert code == ta.TA_EINVAL
    assert "at most" in ta.lib().ta_last_error().decode()
