"""The C-ABI library: loads, exports every declared symbol, host-side tables and validation (no GPU)."""
import os
import re

import numpy as np
import pytest

from oracle import basis, fastdiag, transfer

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2405_19004_amd", "libvps.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libvps.so not built (run python -m paper_2405_19004_amd.build)")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vps.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(vps_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    import ctypes
    L = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    import paper_2405_19004_amd as v
    assert set(names) == set(v.exported_symbols())


@pytest.mark.parametrize("k", range(1, 8))
def test_host_tables_match_oracle(k):
    import paper_2405_19004_amd as v
    assert np.allclose(v.vps_host_table(k, 0), basis.gll_nodes(k), atol=1e-15)
    A, M = basis.reference_matrices(k)
    assert np.allclose(np.reshape(v.vps_host_table(k, 1), A.shape), A, atol=1e-12 * np.abs(A).max())
    assert np.allclose(np.reshape(v.vps_host_table(k, 2), M.shape), M, atol=1e-15)
    m = 2 * k - 1
    S = np.reshape(v.vps_host_table(k, 3), (m, m))
    lam = np.array(v.vps_host_table(k, 4))
    A1, M1 = fastdiag.patch_1d_matrices(k, 1.0)
    assert np.allclose(S.T @ M1 @ S, np.eye(m), atol=1e-13)
    assert np.allclose(A1 @ S, M1 @ S @ np.diag(lam), atol=1e-12 * lam.max())
    # eigenvalues agree with the oracle's LAPACK route (the eigenvectors may differ in sign/order)
    assert np.allclose(np.sort(lam), np.sort(fastdiag.eigen_1d(k, 1.0)[1]), rtol=1e-12)
    # prolongation coefficients: first coarse cell of a level-2 prolongation
    P1 = transfer.prolongation_1d(k, 2)
    P = np.reshape(v.vps_host_table(k, 5), (2 * k + 1, k + 1))
    assert np.allclose(P, P1[:2 * k + 1, :k + 1], atol=1e-14)


def test_footprint_and_validation_need_no_device():
    import paper_2405_19004_amd as v
    a = v.vps_footprint_bytes(3, 4, 6, v.VPS_FLAG_FP64_HIERARCHY)
    b = v.vps_footprint_bytes(3, 4, 6, v.VPS_FLAG_FP64_HIERARCHY | v.VPS_FLAG_FP32_HIERARCHY)
    c = v.vps_footprint_bytes(3, 4, 5, v.VPS_FLAG_FP64_HIERARCHY)
    n = 257 ** 3
    assert b > a > c
    assert 40 * n < a < 60 * n  # four CG vectors + hierarchy scratch, FP64
    with pytest.raises(v.VpsError) as e:
        v.vps_create(4, 2, 3)
    assert e.value.status == v.VPS_EINVAL
    with pytest.raises(v.VpsError):
        v.vps_create(2, 8, 3)
    with pytest.raises(v.VpsError):
        v.vps_create(3, 2, 0)
    with pytest.raises(v.VpsError):
        v.vps_footprint_bytes(3, 7, 20)  # N >= 2^40
    assert "dim" in v.last_error() or "large" in v.last_error() or v.last_error()
    # a mixed-only hierarchy has no FP64 z (the mixed CG reads the FP32 V-cycle output): adding the
    # FP64 hierarchy adds its level buffers and z, i.e. the FP64-only footprint less r, p, q and the
    # scalar block, partial sums and flag (allocations rounded to 256 bytes)
    m = v.vps_footprint_bytes(3, 4, 6, v.VPS_FLAG_FP32_HIERARCHY)
    ru = lambda x: (x + 255) // 256 * 256
    assert b - m == a - 3 * ru(8 * n) - ru(16 * 8) - ru(2 * 1024 * 8) - 256


def test_server_completed_validates_on_host():
    import ctypes
    import paper_2405_19004_amd as v
    n = ctypes.c_int(-1)
    assert v.lib().vps_server_completed(None, None, 0, ctypes.byref(n)) == v.VPS_EINVAL
    s = v.vps_server_create(1 << 20, 4)
    try:
        assert v.vps_server_completed(s) == []  # nothing finished yet
        assert v.lib().vps_server_completed(s, None, 4, ctypes.byref(n)) == v.VPS_EINVAL  # cap > 0, no array
        assert v.lib().vps_server_completed(s, None, 0, None) == v.VPS_EINVAL
    finally:
        v.vps_server_destroy(s)


def test_server_rejects_oversize_request_on_host():
    import paper_2405_19004_amd as v
    s = v.vps_server_create(1 << 20, 4)
    try:
        with pytest.raises(v.VpsError) as e:
            v.vps_server_submit(s, 3, 4, 6, 1, 1, 1e-8, v.VPS_SOLVE_MIXED, 50)
        assert e.value.status == v.VPS_EBUSY
        with pytest.raises(v.VpsError):
            v.vps_server_submit(s, 3, 4, 2, 1, 1, -1.0, v.VPS_SOLVE_MIXED, 50)
    finally:
        v.vps_server_destroy(s)


def test_noalloc_restrict_refuses_on_the_host():
    """Sizes beyond the static scratch, bad shapes and precisions are refused before any device
    work (the pointers are never touched)."""
    import paper_2405_19004_amd as v
    L = v.lib()
    assert L.vps_restrict_noalloc(3, 4, 7, v.VPS_FP64, 1, 1, None) == v.VPS_EINVAL
    assert "exceeds" in v.last_error()
    assert L.vps_restrict_noalloc(3, 4, 1, v.VPS_FP64, 1, 1, None) == v.VPS_EINVAL
    assert L.vps_restrict_noalloc(4, 4, 3, v.VPS_FP64, 1, 1, None) == v.VPS_EINVAL
    assert L.vps_restrict_noalloc(3, 4, 3, 2, 1, 1, None) == v.VPS_EINVAL
    assert L.vps_restrict_noalloc(3, 4, 3, v.VPS_FP32, None, 1, None) == v.VPS_EINVAL
