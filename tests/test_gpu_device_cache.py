"""The library's device cache: setups that run on reused (and then trimmed)
device memory give bit-identical preconditioners and solves, so no phase
reads memory it did not write."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import DeviceCSR, Preconditioner, trim_device_cache  # noqa: E402


def test_repeated_setups_bit_identical():
    cfg = W.config_small3d(16, 16)
    part = O.ggg_partition(cfg.A, cfg.N, cfg.ggg_seed)
    dA = DeviceCSR.from_workload(cfg.A)
    r = torch.as_tensor(W.rhs(cfg.A.n, 3), device="cuda")
    b = torch.as_tensor(W.rhs(cfg.A.n, 4), device="cuda")
    out = []
    for k in range(4):
        pre = Preconditioner(dA, part, cfg.N, cfg.overlap, cfg.tau, levels=3, coarsen=4)
        z = pre.apply(r).cpu().numpy()
        x, its, rr, code = pre.pcg(b, rtol=1e-10)
        assert code == 0
        out.append((z, x.cpu().numpy(), its[0]))
        print(f"[cache] setup {k}: its {its[0]} relres {rr[0]:.2e}", flush=True)
        sys.stdout.flush()
        del pre
        if k == 1:
            trim_device_cache()
    for z, x, its in out[1:]:
        assert its == out[0][2]
        np.testing.assert_array_equal(z, out[0][0])
        np.testing.assert_array_equal(x, out[0][1])
