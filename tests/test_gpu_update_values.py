"""dd_update_values (a family of matrices with one pattern and one partition):
after an update the handle behaves exactly as a fresh dd_setup on the new
values (the setup is deterministic, so applies agree bit for bit and PCG takes
the same iterations), and it matches the oracle built on the new values; an
update with non-finite values is rejected and leaves the handle as it was."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import DDError, DeviceCSR, Preconditioner  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _family(seed):
    return W.diffusion3d(16, seed)


def test_update_equals_fresh_setup_and_oracle():
    A0, A1 = _family(0), _family(1)
    assert np.array_equal(A0.rowptr, A1.rowptr) and np.array_equal(A0.colind, A1.colind)
    N = 16
    part = O.ggg_partition(A0, N, 0)
    pre = Preconditioner(DeviceCSR.from_workload(A0), part, N, 2, 0.02)
    pre.update_values(A1.val)
    fresh = Preconditioner(DeviceCSR.from_workload(A1), part, N, 2, 0.02)
    assert pre.info()["n_C"] == fresh.info()["n_C"]
    r = torch.as_tensor(W.rhs(A1.n, 4), device="cuda")
    assert torch.equal(pre.apply(r), fresh.apply(r))
    b = torch.as_tensor(W.rhs(A1.n, 0), device="cuda")
    x, its, rr, code = pre.pcg(b, rtol=1e-13, maxit=500)
    xf, itsf, rrf, codef = fresh.pcg(b, rtol=1e-13, maxit=500)
    assert code == 0 and its == itsf and torch.equal(x, xf)
    ora = O.build(A1, part, N, 2, 0.02)
    xo, itso, _ = O.pcg(A1, W.rhs(A1.n, 0), ora.apply, rtol=1e-13, maxit=500)
    log(f"[update] its after update {its[0]}, fresh {itsf[0]}, oracle {itso}")
    assert abs(its[0] - itso) <= 1
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


def test_update_with_nan_keeps_handle():
    A0 = _family(0)
    N = 16
    part = O.ggg_partition(A0, N, 0)
    pre = Preconditioner(DeviceCSR.from_workload(A0), part, N, 2, 0.02)
    r = torch.as_tensor(W.rhs(A0.n, 4), device="cuda")
    z0 = pre.apply(r)
    bad = A0.val.copy()
    bad[11] = np.nan
    with pytest.raises(DDError) as e:
        pre.update_values(bad)
    assert e.value.code == -4
    assert torch.equal(pre.apply(r), z0)
