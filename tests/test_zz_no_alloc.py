"""distortion_bwd_noalloc (the allocation-free backward) against
distortion_bwd, through the C ABI: bit-identical gradients on two calls in a
row, the second with a smaller input, so the shared fixed scratch is reused
and must be cleared; an oversized request is rejected before any GPU work."""

import ctypes
import sys

import numpy as np
import pytest

from synth import distortion_batch

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_2412_02244_amd as ekm
    assert torch.cuda.is_available()
    return ekm.load_library()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(lib, xb, cb, g, dtype_code):
    import torch
    import paper_2412_02244_amd as ekm
    dev = torch.device("cuda:0")
    x = torch.from_numpy(xb).to(dev)
    c = torch.from_numpy(cb).to(dev)
    B, n, d = x.shape
    k = c.shape[1]
    a = torch.empty((B, n), dtype=torch.int32, device=dev)
    loss = torch.empty(B, dtype=torch.float64, device=dev)
    gl = torch.from_numpy(g).to(dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.distortion_fwd(_ptr(x), _ptr(c), dtype_code, B, n, k, d, _ptr(a), _ptr(loss), stream) == ekm.KM_OK
    gx_ref, gc_ref = torch.empty_like(x), torch.empty_like(c)
    assert lib.distortion_bwd(_ptr(x), _ptr(c), _ptr(a), _ptr(gl), dtype_code, B, n, k, d, _ptr(gx_ref),
                              _ptr(gc_ref), stream) == ekm.KM_OK, ekm.kmeans_last_error()
    gx, gc = torch.full_like(x, float("nan")), torch.full_like(c, float("nan"))
    st = lib.distortion_bwd_noalloc(_ptr(x), _ptr(c), _ptr(a), _ptr(gl), dtype_code, B, n, k, d, _ptr(gx),
                                    _ptr(gc), stream)
    assert st == ekm.KM_OK, ekm.kmeans_last_error()
    torch.cuda.synchronize()
    return (gx.cpu().numpy(), gc.cpu().numpy()), (gx_ref.cpu().numpy(), gc_ref.cpu().numpy()), a.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_matches_distortion_bwd_twice(lib, dtype):
    import oracle
    import paper_2412_02244_amd as ekm
    code = ekm.KM_F32 if dtype == "f32" else ekm.KM_F64
    cases = [(6, 3000, 64, 51), (2, 700, 16, 52)]  # second call: smaller B, n and k
    for B, n, k, seed in cases:
        _say(f"[noalloc] dtype={dtype} B={B} n={n} k={k} seed={seed}")
        xb, cb = distortion_batch(n_clouds=B, n=n, k=k, seed=seed)
        if dtype == "f64":
            xb, cb = xb.astype(np.float64), cb.astype(np.float64)
        g = np.linspace(0.5, 2.0, B)
        (gx, gc), (gx_ref, gc_ref), a = _both(lib, xb, cb, g, code)
        np.testing.assert_array_equal(gx, gx_ref)
        np.testing.assert_array_equal(gc, gc_ref)
        a_o, _ = oracle.distortion_fwd(xb, cb)
        np.testing.assert_array_equal(a, a_o)
        gx_o, gc_o = oracle.distortion_bwd(xb, cb, a_o, g)
        tol = dict(rtol=1e-6, atol=1e-6) if dtype == "f32" else dict(rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(gx, gx_o, **tol)
        np.testing.assert_allclose(gc, gc_o, **tol)


def test_noalloc_rejects_oversized_scratch(lib):
    import paper_2412_02244_amd as ekm
    p = ctypes.c_void_p(16)
    # B * k * (16 d + 4) = 512 * 1024 * 52 bytes > 8 MiB: rejected before any GPU work
    st = lib.distortion_bwd_noalloc(p, p, p, p, ekm.KM_F32, 512, 10, 1024, 3, None, p, None)
    assert st == ekm.KM_ERR_INVALID
    assert "scratch" in ekm.kmeans_last_error()
