"""bench.py on the CPU: the single-GPU guard and the structural facts its flop model relies on."""
import os
import subprocess
import sys

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import smoother

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


@pytest.mark.parametrize("k", range(1, 8))
def test_patch_rows_have_the_counted_nonzeros(k):
    """The model counts nnz = (2k-2)(k+1) + 2k+1 nonzeros in the interior rows of the 1D patch
    matrices (a cell-interior node couples to its own cell only)."""
    A, M = smoother.patch_1d_matrices(k, 1.0)
    nnz = (2 * k - 2) * (k + 1) + (2 * k + 1)
    for B in (A, M):
        rows = B[1:-1, :]
        assert np.count_nonzero(np.abs(rows) > 1e-14 * np.abs(rows).max()) == nnz


@pytest.mark.parametrize("k", range(1, 8))
def test_patch_eigenvectors_are_even_or_odd(k):
    """S and S^T cost (m^2+1)/2 multiply-adds per line: the k even and k-1 odd eigenvectors of the
    mirror-symmetric interior pair."""
    A, M = smoother.patch_1d_matrices(k, 1.0)
    Ai, Mi = A[1:-1, 1:-1], M[1:-1, 1:-1]
    lam, S = sla.eigh(Ai, Mi)
    m = 2 * k - 1
    even = odd = 0
    for a in range(m):
        v = S[:, a]
        if np.allclose(v, v[::-1], atol=1e-10):
            even += 1
        elif np.allclose(v, -v[::-1], atol=1e-10):
            odd += 1
    assert (even, odd) == (k, k - 1)
    h = k - 1
    assert even * (h + 1) + odd * h == (m * m + 1) // 2


def test_flop_model_at_degree_4():
    assert bench.colour_pass_issued_flops(3, 4) == 53201
    assert bench.colour_pass_bytes(3, 4, 4) == 4 * (9 ** 3 + 2 * 7 ** 3)


@pytest.mark.parametrize("d,k,patches,per_step", [(3, 4, 250047, 2.15e10), (2, 7, 261121, 1.04e10),
                                                   (3, 3, 29791, 7.59e8)])
def test_algorithmic_model_matches_the_workload_table(d, k, patches, per_step):
    """The algorithmic flops per smoothing step (one update of every patch) of the 3D Q4 64^3,
    2D Q7 512^2 and 3D Q3 32^3 workloads, as tabulated for the measurement model (3 digits)."""
    assert abs(bench.smoother_patch_flops(d, k) * patches / per_step - 1) < 5e-3


def test_algorithmic_words_3d_q4():
    # x on the 9^3 closure skeleton + b on the 7^3 interior read, x on the interior written
    assert bench.smoother_patch_min_words(3, 4) == (9 ** 3 - 7 ** 3) + 7 ** 3 + 7 ** 3 == 1072
    assert bench.smoother_patch_flops(3, 4) == 86072


def test_lds_traffic_model_3d_q4():
    """LDS words per patch of the closure-through-LDS colour pass (3D Q4, two patches per
    workgroup): closure 81 * 17 / 2, then per stage lines in and out, summed by hand."""
    import bench
    by_hand = 81 * 17 / 2 + (729 + 1134) + (1134 + 882) + (882 + 343) + 6 * 343 + 2 * 343
    assert by_hand == 8536.5
    assert bench.colour_pass_lds_bytes_3d(4, 4, 2) == 4 * by_hand
    assert bench.colour_pass_lds_bytes_3d(4, 8, 2) == 8 * by_hand
