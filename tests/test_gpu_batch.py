"""dd_setup_batch: several independent systems of uneven size and type in one
handle (all their subdomains in the same batched launches) and one PCG per
system in lockstep.  With two levels every system must behave as with its own
dd_setup: the batched apply equals the separate applies, and each system's
PCG matches its separate solve (iterations within 1, x within 1e-10 at rtol
1e-13) and the oracle; the systems converge at their own iteration counts."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import DeviceCSR, Preconditioner  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _systems():
    A1 = W.poisson2d(32)
    p1 = W.grid2d_partition(32, 2, 2)
    A2 = W.diffusion3d(10, seed=3)
    p2 = O.ggg_partition(A2, 8, 0)
    A3 = W.random_spd(500, 5, seed=9, positive_offdiag=True)
    p3 = O.ggg_partition(A3, 4, 0)
    return [(A1, p1, 4), (A2, p2, 8), (A3, p3, 4)]


def test_batch_matches_separate_setups_and_oracle():
    sysl = _systems()
    As = [DeviceCSR.from_workload(A) for A, _, _ in sysl]
    pre = Preconditioner.batch(As, [p for _, p, _ in sysl], [N for _, _, N in sysl], 1, 0.1)
    sep = [Preconditioner(dA, p, N, 1, 0.1) for dA, (_, p, N) in zip(As, sysl)]
    ns = [A.n for A, _, _ in sysl]
    off = np.concatenate([[0], np.cumsum(ns)])
    r = np.concatenate([W.rhs(n, 20 + j) for j, n in enumerate(ns)])
    z = pre.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
    for j, P in enumerate(sep):
        zj = P.apply(torch.as_tensor(r[off[j]:off[j + 1]], device="cuda")).cpu().numpy()
        assert np.linalg.norm(z[off[j]:off[j + 1]] - zj) <= 1e-12 * np.linalg.norm(zj)
    b = np.concatenate([W.rhs(n, j) for j, n in enumerate(ns)])
    x, its, rr, code = pre.pcg(torch.as_tensor(b, device="cuda"), rtol=1e-13, maxit=1000)
    assert code == 0 and len(its) == 3
    xg = x.cpu().numpy()
    for j, ((A, p, N), P) in enumerate(zip(sysl, sep)):
        bj = b[off[j]:off[j + 1]]
        xs, itss, rrs, _ = P.pcg(torch.as_tensor(bj, device="cuda"), rtol=1e-13, maxit=1000)
        ora = O.build(A, p, N, 1, 0.1)
        xo, itso, _ = O.pcg(A, bj, ora.apply, rtol=1e-13, maxit=1000)
        log(f"[batch] system {j}: n={A.n} its batch {its[j]} separate {itss[0]} oracle {itso}, relres {rr[j]:.2e}")
        assert rr[j] <= 2e-13
        assert abs(its[j] - itss[0]) <= 1 and abs(its[j] - itso) <= 1
        xj = xg[off[j]:off[j + 1]]
        assert np.linalg.norm(xj - xs.cpu().numpy()) <= 1e-10 * np.linalg.norm(xo)
        assert np.linalg.norm(xj - xo) <= 1e-10 * np.linalg.norm(xo)
    assert len(set(its)) > 1  # the systems stop at their own counts


def test_batch_three_levels_per_system():
    """Three levels: every system's second level is partitioned on its own and
    its inner coarse solves run per system, so each system gets the hierarchy
    and the solve of its own setup and of the oracle."""
    sysl = _systems()
    As = [DeviceCSR.from_workload(A) for A, _, _ in sysl]
    pre = Preconditioner.batch(As, [p for _, p, _ in sysl], [N for _, _, N in sysl], 1, 0.1, levels=3, coarsen=4)
    assert pre.info()["levels"] == 3
    ns = [A.n for A, _, _ in sysl]
    off = np.concatenate([[0], np.cumsum(ns)])
    b = np.concatenate([W.rhs(n, j) for j, n in enumerate(ns)])
    x, its, rr, code = pre.pcg(torch.as_tensor(b, device="cuda"), rtol=1e-13, maxit=1000)
    xg = x.cpu().numpy()
    assert code == 0
    for j, ((A, p, N), dA) in enumerate(zip(sysl, As)):
        bj = b[off[j]:off[j + 1]]
        P = Preconditioner(dA, p, N, 1, 0.1, levels=3, coarsen=4)
        xs, itss, _, _ = P.pcg(torch.as_tensor(bj, device="cuda"), rtol=1e-13, maxit=1000)
        ora = O.build(A, p, N, 1, 0.1, levels=3, coarsen=4)
        xo, itso, _ = O.flexible_pcg(A, bj, ora.apply, rtol=1e-13, maxit=1000)
        log(f"[batch] 3 levels, system {j}: its batch {its[j]} separate {itss[0]} oracle {itso}, relres {rr[j]:.2e}")
        assert rr[j] <= 2e-13
        assert abs(its[j] - itss[0]) <= 1 and abs(its[j] - itso) <= 1
        xj = xg[off[j]:off[j + 1]]
        assert np.linalg.norm(xj - xs.cpu().numpy()) <= 1e-10 * np.linalg.norm(xo)
        assert np.linalg.norm(xj - xo) <= 1e-10 * np.linalg.norm(xo)
