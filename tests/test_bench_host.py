"""Host-side pieces of bench.py that need no GPU: the oracle split over worker
processes gives the oracle's own result bit for bit (it is the CPU baseline
the benchmark reports), and the work model of the edge kernels."""
import numpy as np

import bench
from oracle import sttsv_ref
from paper_2311_08595_amd import workloads as wl


def test_parallel_oracle_is_the_oracle():
    w = wl.zipf_powerlaw(seed=9, n=3000, m=9000, kmax=12)
    ref = sttsv_ref.sttsv(w["eptr"], w["eidx"], w["n"], 12, w["x"])
    for procs in (1, 3):
        y = bench.oracle_sttsv_parallel(w["eptr"], w["eidx"], w["n"], 12, w["x"], procs)
        assert y.tobytes() == ref.tobytes()


def test_edge_fma_counts():
    # k = 2: one dot of W-1 terms; k >= 4: 2(k-3) truncated products plus dots
    assert bench.edge_fma(2, 5) == 3
    assert bench.edge_fma(4, 5) == 2 * 1 * (2 * 1 // 2) + 5 * 2 - 1
    assert bench.edge_fma(1, 9) == 0
