"""dd_partition_ggg_noalloc, the partition entry point that allocates nothing
(its work arrays live in a file-scope device array per GPU), called through
the C-ABI: two calls in a row, the second on a smaller graph, each equal bit
for bit to dd_partition_ggg on the same input (integer work, the same rule)
and to the oracle's growing rule.  Sizes beyond the array are refused."""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import DeviceCSR, lib  # noqa: E402
from paper_2109_05908_amd.binding import _ptr, _stream  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _part(fn, dA, N, seed):
    part = torch.full((dA.n,), -7, dtype=torch.int32, device="cuda")
    cs = dA.cstruct()
    rc = getattr(lib(), fn)(C.byref(cs), N, seed, _ptr(part), _stream())
    torch.cuda.synchronize()
    return rc, part.cpu().numpy()


def test_noalloc_partition_equals_allocating_entry_point():
    cases = [(W.diffusion3d(40, seed=2), 200, 5), (W.poisson2d(30), 9, 1)]  # the second is smaller
    for A, N, seed in cases:
        dA = DeviceCSR.from_workload(A)
        log(f"[noalloc] n={A.n} N={N} seed={seed}")
        rc0, p0 = _part("dd_partition_ggg_noalloc", dA, N, seed)
        rc1, p1 = _part("dd_partition_ggg", dA, N, seed)
        assert rc0 == 0 and rc1 == 0
        assert np.array_equal(p0, p1)
        assert np.array_equal(p0, O.ggg_partition(A, N, seed))
        assert p0.min() >= 0 and p0.max() == N - 1


def test_noalloc_partition_refuses_sizes_beyond_its_array():
    A = W.poisson2d(8)
    dA = DeviceCSR.from_workload(A)
    part = torch.empty(A.n, dtype=torch.int32, device="cuda")
    cs = dA.cstruct()
    big = type(cs)(1 << 23, cs.nnz, cs.rowptr, cs.colind, cs.val)  # n beyond the array: refused before any kernel
    assert lib().dd_partition_ggg_noalloc(C.byref(big), 4, 0, _ptr(part), _stream()) == -1
    assert lib().dd_partition_ggg_noalloc(C.byref(cs), 0, 0, _ptr(part), _stream()) == -1
