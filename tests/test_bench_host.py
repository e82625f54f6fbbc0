"""Host-side checks of the benchmark's bookkeeping (CPU).

The roofline's algorithmic bytes must count every datum of one block
product once, from the pattern the oracle builds; the HBM-traffic figure
is the counters scaled by the copy probe's known bytes; a multi-GPU request
is refused before any device work.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_spmv_bytes_counts_each_datum_once():
    """Headline workload: 3x3 complex128 blocks + int32 column index per
    block, int32 row pointers, one complex128 x read and y written per
    unknown, counted from the oracle's block pattern."""
    p, _ = W.pec_cube(30)
    rp, ci = fem.block_pattern(p)
    nn, nnzb = len(rp) - 1, len(ci)
    by_parts = (nnzb * 9 * 16          # block values
                + ci.size * 4           # column indices
                + rp.size * 4           # row pointers
                + 3 * nn * 16           # x
                + 3 * nn * 16)          # y
    assert bench.spmv_bytes(nn, nnzb, 16, 16) == by_parts == 110825140


def test_spmm_bytes_reduces_to_spmv_for_one_column():
    p, _ = W.free_cube(6)
    rp, ci = fem.block_pattern(p)
    nn, nnzb = len(rp) - 1, len(ci)
    assert bench.spmm_bytes(nn, nnzb, 1) == bench.spmv_bytes(nn, nnzb, 16, 16)


def test_traffic_is_counters_scaled_by_the_copy_probe():
    if not bench.MEASURED_TRAFFIC:
        pytest.skip("no counter run recorded for the current kernels")
    for key, m in bench.MEASURED_TRAFFIC.items():
        t = bench.measured_traffic(key)
        if t is None:
            continue  # kernel source changed since the counters were taken
        fetch = m["fetch_kib"] * 1024 * m["copy_bytes"] / (m["copy_fetch_kib"] * 1024)
        write = m["write_kib"] * 1024 * m["copy_bytes"] / (m["copy_write_kib"] * 1024)
        assert t == pytest.approx(fetch + write, rel=1e-12)
        # the copy probe reads and writes 1 GiB: FETCH_SIZE counts half the
        # bytes read on this part, WRITE_SIZE all bytes written
        assert m["copy_bytes"] / (m["copy_fetch_kib"] * 1024) == pytest.approx(2.0, rel=1e-3)
        assert m["copy_bytes"] / (m["copy_write_kib"] * 1024) == pytest.approx(1.0, rel=1e-3)
    assert bench.measured_traffic("no such kernel") is None


def test_headline_bytes_are_the_complex64_matrix_product():
    """The headline roofline prices the matrix-mixed product: complex64 block
    values (8 bytes per complex) with complex128 vectors, on the 60^3 coated
    sphere's pattern (444.18 MB per launch)."""
    p, _ = W.pec_sphere_shell(60)
    rp, ci = fem.block_pattern(p)
    nn, nnzb = len(rp) - 1, len(ci)
    assert (nn, nnzb) == (214712, 5561948)
    assert bench.spmv_bytes(nn, nnzb, 8, 16) == nnzb * 76 + 4 * (nn + 1) + 2 * 3 * nn * 16 == 444179252


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_fifo_finish_times_of_a_one_at_a_time_solver():
    """The plain solver's latencies under load come from its service times by
    the first-in-first-out recursion; checked by hand on a queue that drains
    and refills: idle gap, back-to-back arrivals, a long job holding later ones."""
    arr = [0.0, 0.5, 0.6, 5.0, 5.1]
    svc = [1.0, 1.0, 2.0, 0.5, 0.1]
    fin = bench.fifo_finish_times(arr, svc)
    assert list(fin) == [1.0, 2.0, 4.0, 5.5, 5.6]
    assert list(fin - arr) == [1.0, 1.5, 3.4, 0.5, 0.5]


def test_unknown_serving_mode_is_refused():
    import pytest
    with pytest.raises(SystemExit):
        bench.serving_leg(None, None, None, 1, 10, 12, 1, [0.5], ["no_such_mode"])


def test_bic_apply_bytes_counts_each_array():
    """One block of two nodes whose L is the full 6 x 6 lower triangle (21
    entries, so U holds the 15 below-diagonal ones transposed): every array
    the application touches, counted by hand."""
    n = 6
    factor = (21 + 15) * (16 + 4)          # values and columns of L and U
    row_starts = 2 * (n + 1) * 4           # lrp and urp
    dinv = 2 * n * 16                      # 1 / l_uu, staged in both sweeps
    vectors = 2 * n * 16 + n * 16          # r twice, z once
    sums = 4 * 8 * 2                       # the block's four sums, written and read back
    assert bench.bic_apply_bytes(n, 21, 6) == factor + row_starts + dinv + vectors + sums
