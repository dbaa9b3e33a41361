"""Launch-cost microbenchmark (kernel overlap behind one released gate):
every released kernel's outputs are checked against the per-thread multiply-add chain computed here with numpy, and the timings are
checked for consistency."""
import numpy as np
import pytest

import paper_2605_12734_amd as od

pytestmark = pytest.mark.gpu


def _chain(n, work):
    x = (np.arange(n, dtype=np.uint64).astype(np.uint32)) ^ np.uint32(0x9E3779B9)
    with np.errstate(over="ignore"):
        for _ in range(work):
            x = x * np.uint32(1664525) + np.uint32(1013904223)
    return x


@pytest.mark.parametrize("total,nk", [(1 << 18, 1), (1 << 18, 8), (1 << 18, 64), (100003, 7), (1000, 1000)])
def test_overlap_outputs_and_timing(total, nk):
    work = 300
    r = od.launch_overlap(total, nk, work=work, return_outputs=True)
    assert r["nkernels"] == nk and r["total_threads"] == total and r["nstreams"] == min(nk, 64)
    assert np.array_equal(r["outputs"], _chain(total, work))
    assert 0 < r["makespan_us"] < 1e6
    assert r["enqueue_us"] > 0 and r["host_us"] > 0


def test_overlap_rejects_bad_arguments():
    with pytest.raises(od.ODError):
        od.launch_overlap(100, 101)          # more kernels than threads
    with pytest.raises(od.ODError):
        od.launch_overlap(100, 4, nstreams=0)
