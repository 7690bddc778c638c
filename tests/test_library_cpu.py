"""Host-side checks of the C-ABI library that need no GPU: it loads, it
exports every entry point include/ekm.h declares, argument errors come back
as status codes with a message before any GPU work, and the workspace model
is an upper bound that grows with n."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ekm.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2412_02244_amd as ekm
    if not os.path.exists(ekm.LIB_PATH):
        from paper_2412_02244_amd import build
        build.build(verbose=False)
    return ekm.load_library()


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"EKM_API\s+[\w\s\*]+?\b(\w+)\s*\(", src)))


def test_header_declares_the_abi():
    names = _declared()
    import paper_2412_02244_amd as ekm
    assert set(names) == set(ekm.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    import paper_2412_02244_amd as ekm
    out = subprocess.run(["nm", "-D", "--defined-only", ekm.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)
    # nothing else leaks out of the C ABI
    assert exported == set(_declared())


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "ekm.h"\nint main(void){ km_config c = {0}; (void)c; return 0; }\n')
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), "-c",
                           str(src), "-o", str(tmp_path / "t.o")])


def _cfg(ekm, **kw):
    base = dict(d=2, point_dtype=ekm.KM_F32, algo=ekm.KM_INDEXED, leaf_size=0, cand_tile=0, flags=0,
                workspace_limit_bytes=0)
    base.update(kw)
    return ekm.KmConfig(**base)


@pytest.mark.parametrize("kw,n,k,status", [
    (dict(d=4), 100, 10, 1),
    (dict(d=1), 100, 10, 1),
    (dict(point_dtype=7), 100, 10, 1),
    (dict(algo=9), 100, 10, 1),
    (dict(), 100, 0, 1),
    (dict(), 100, 101, 1),
    (dict(), 0, 1, 1),
    (dict(leaf_size=48), 100, 10, 1),
    (dict(leaf_size=128), 100, 10, 1),
    (dict(cand_tile=5000), 100, 10, 1),
    (dict(point_dtype=0), 100, 10, 4),  # FP64 points on the indexed path
    (dict(), 1 << 31, 10, 1),
])
def test_init_rejects_bad_arguments(lib, kw, n, k, status):
    import paper_2412_02244_amd as ekm
    cfg = _cfg(ekm, **kw)
    h = ctypes.c_void_p()
    st = lib.kmeans_init(ctypes.byref(h), ctypes.byref(cfg), ctypes.c_void_p(16), n, k, None)
    assert st == status
    assert h.value is None
    assert ekm.kmeans_last_error()


def test_null_pointers_rejected(lib):
    import paper_2412_02244_amd as ekm
    cfg = _cfg(ekm)
    h = ctypes.c_void_p()
    assert lib.kmeans_init(ctypes.byref(h), ctypes.byref(cfg), None, 100, 10, None) == ekm.KM_ERR_INVALID
    assert "null" in ekm.kmeans_last_error()
    assert lib.kmeans_init(None, ctypes.byref(cfg), ctypes.c_void_p(16), 100, 10, None) == ekm.KM_ERR_INVALID
    assert lib.kmeans_step(None, None, None, None, None) == ekm.KM_ERR_INVALID
    assert lib.kmeans_run(None, None, None, 1, 0, None, None) == ekm.KM_ERR_INVALID
    assert lib.kmeans_destroy(None) == ekm.KM_OK
    assert lib.kmeans_phase_times(None, None, None) == ekm.KM_ERR_INVALID
    assert lib.distortion_fwd(None, None, 1, 1, 1, 1, 3, None, None, None) == ekm.KM_ERR_INVALID
    assert lib.distortion_fwd(ctypes.c_void_p(16), ctypes.c_void_p(16), 1, 1, 1, 1, 4, ctypes.c_void_p(16),
                              ctypes.c_void_p(16), None) == ekm.KM_ERR_INVALID
    assert lib.distortion_bwd(ctypes.c_void_p(16), ctypes.c_void_p(16), None, None, 1, 1, 1, 1, 3, None, None,
                              None) == ekm.KM_ERR_INVALID


def test_workspace_limit_rejected_before_gpu_work(lib):
    import paper_2412_02244_amd as ekm
    cfg = _cfg(ekm, workspace_limit_bytes=1000)
    h = ctypes.c_void_p()
    assert lib.kmeans_init(ctypes.byref(h), ctypes.byref(cfg), ctypes.c_void_p(16), 100000, 10, None) == \
        ekm.KM_ERR_OOM
    assert "workspace" in ekm.kmeans_last_error()


def test_workspace_bytes_model(lib):
    import paper_2412_02244_amd as ekm
    small = ekm.kmeans_workspace_bytes(10_000, 100, 2)
    big = ekm.kmeans_workspace_bytes(1_000_000, 100, 2)
    assert 0 < small < big
    assert ekm.kmeans_workspace_bytes(100, 1000, 2) == 0  # k > n is invalid
    brute = ekm.kmeans_workspace_bytes(1_000_000, 1000, 2, algo=ekm.KM_BRUTE)
    assert 0 < brute < big
    # at least the points, the permutation and the assignment
    assert big >= 1_000_000 * (2 * 4 + 4 + 4)


def test_memory_model_and_leaf_size_from_budget(lib):
    """Eq. (10)-(12) on this library's buffers: the modelled workspace grows
    as the leaves shrink, and with a budget (and leaf_size 0) the leaf size is
    the smallest whose modelled workspace fits."""
    import paper_2412_02244_amd as ekm
    n, k = 1_000_000, 1000
    m = {f: ekm.kmeans_workspace_bytes(n, k, 2, leaf_size=f) for f in (8, 16, 32, 64)}
    assert m[8] > m[16] > m[32] > m[64] > 0
    # the difference between two leaf sizes is the per-leaf state of the extra leaves
    assert m[8] - m[64] > (n // 8 - n // 64) * 32
    assert ekm.kmeans_workspace_bytes(n, k, 2) == m[64]  # no budget: the default leaf size
    for f in (8, 16, 32, 64):
        assert ekm.kmeans_workspace_bytes(n, k, 2, workspace_limit_bytes=m[f]) == m[f]
        if f > 8:
            assert ekm.kmeans_workspace_bytes(n, k, 2, workspace_limit_bytes=m[f // 2] - 1) == m[f]
    # twice the points: about twice the workspace (points dominate)
    m2 = ekm.kmeans_workspace_bytes(2 * n, k, 2, leaf_size=64)
    assert 1.9 < m2 / m[64] < 2.1
    # a budget below the coarsest index is rejected before any GPU work
    cfg = _cfg(ekm, workspace_limit_bytes=m[64] - 1)
    h = ctypes.c_void_p()
    assert lib.kmeans_init(ctypes.byref(h), ctypes.byref(cfg), ctypes.c_void_p(16), n, k, None) == ekm.KM_ERR_OOM
    assert "workspace" in ekm.kmeans_last_error()
