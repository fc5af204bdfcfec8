"""PCG iterations as a replayed HIP graph (dd_options.graph_pcg), through the C-ABI.

The captured iteration computes alpha, beta and the stopping test on the
device with the host loop's arithmetic (same dot kernels, IEEE divisions), so
iteration counts, iterates and reported residuals equal the host-driven PCG
bit for bit.  Each test replays the graph several times with other eager work
and synchronisations in between, and checks every replay; a solve stopped by
maxit leaves the iterate of that step.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import DD_FP32, DeviceCSR, Preconditioner  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(name):
    if name == "c1":
        c = W.config_c1()
        return c.A, c.part, 16, 1, 0.1
    if name == "small3d":
        c = W.config_small3d()
        return c.A, O.ggg_partition(c.A, c.N, 0), c.N, 2, 0.02
    if name == "rand":
        A = W.random_spd(600, 5, seed=1)
        return A, W.contiguous_partition(600, 6), 6, 2, 0.1
    c = W.config_small_elasticity()
    return c.A, c.part, c.N, c.overlap, c.tau


@pytest.mark.parametrize("name", ["c1", "small3d", "rand", "elast"])
def test_graph_pcg_equals_host_loop(name):
    A, part, N, delta, tau = _case(name)
    dA = DeviceCSR.from_workload(A)
    eager = Preconditioner(dA, part, N, delta, tau)
    graph = Preconditioner(dA, part, N, delta, tau, graph_pcg=8)
    for rep in range(3):
        b = torch.as_tensor(W.rhs(A.n, 10 + rep), device="cuda")
        x0, i0, r0, c0 = eager.pcg(b, rtol=1e-12, maxit=1000)
        torch.cuda.synchronize()
        _ = eager.apply(b)  # unrelated eager work between replays
        x1, i1, r1, c1 = graph.pcg(b, rtol=1e-12, maxit=1000)
        log(f"[graph] {name} replay {rep}: its host {i0[0]} graph {i1[0]}, relres {r0[0]:.3e} {r1[0]:.3e}")
        assert c0 == c1 == 0 and i0 == i1 and r0 == r1
        assert torch.equal(x0, x1)


def test_graph_pcg_multi_rhs_maxit_and_fp32():
    c = W.config_c1()
    dA = DeviceCSR.from_workload(c.A)
    for prec in (0, DD_FP32):
        eager = Preconditioner(dA, c.part, 16, 1, 0.1, local_prec=prec)
        graph = Preconditioner(dA, c.part, 16, 1, 0.1, local_prec=prec, graph_pcg=5)
        B = torch.as_tensor(W.rhs(c.A.n, 3, nrhs=2), device="cuda")
        x0, i0, r0, c0 = eager.pcg(B, rtol=1e-10)
        x1, i1, r1, c1 = graph.pcg(B, rtol=1e-10)
        assert i0 == i1 and r0 == r1 and torch.equal(x0, x1)
        b = torch.as_tensor(W.rhs(c.A.n, 4), device="cuda")
        x0, i0, r0, c0 = eager.pcg(b, rtol=1e-12, maxit=4)
        x1, i1, r1, c1 = graph.pcg(b, rtol=1e-12, maxit=4)
        log(f"[graph] maxit 4 (prec {prec}): codes {c0} {c1}, its {i0} {i1}")
        assert c0 == c1 == 1 and i0 == i1 == [4] and r0 == r1 and torch.equal(x0, x1)


def test_graph_option_ignored_with_three_levels():
    c = W.config_c1()
    dA = DeviceCSR.from_workload(c.A)
    b = torch.as_tensor(W.rhs(c.A.n, 0), device="cuda")
    p0 = Preconditioner(dA, c.part, 16, 1, 0.1, levels=3, coarsen=4)
    p1 = Preconditioner(dA, c.part, 16, 1, 0.1, levels=3, coarsen=4, graph_pcg=8)
    x0, i0, r0, _ = p0.pcg(b, rtol=1e-10)
    x1, i1, r1, _ = p1.pcg(b, rtol=1e-10)
    assert i0 == i1 and torch.equal(x0, x1)


def test_graph_and_block_after_update_values():
    """dd_update_values replaces the levels of a handle; the PCG graph captured
    before (and the block state of several right-hand sides) pointed into the
    old levels' buffers and must be rebuilt: after the update, one and two
    right-hand sides give bit for bit what a fresh setup on the new values
    gives."""
    c0, c1 = W.config_small3d(16, 16, 0), W.config_small3d(16, 16, 1)
    part = O.ggg_partition(c0.A, c0.N, 0)
    assert np.array_equal(c0.A.colind, c1.A.colind)
    b = torch.as_tensor(W.rhs(c0.A.n, 2), device="cuda")
    B = torch.as_tensor(W.rhs(c0.A.n, 3, nrhs=2).reshape(c0.A.n, 2), device="cuda")
    pre = Preconditioner(DeviceCSR.from_workload(c0.A), part, c0.N, 2, 0.02, graph_pcg=8)
    pre.pcg(b, rtol=1e-10)
    pre.pcg(B, rtol=1e-10)
    pre.update_values(torch.as_tensor(c1.A.val))
    fresh = Preconditioner(DeviceCSR.from_workload(c1.A), part, c0.N, 2, 0.02, graph_pcg=8)
    for rhs in (b, B):
        x0, i0, r0, _ = fresh.pcg(rhs, rtol=1e-10)
        x1, i1, r1, _ = pre.pcg(rhs, rtol=1e-10)
        log(f"[graph] after update_values: its {i1} (fresh setup {i0})")
        assert i0 == i1 and r0 == r1 and torch.equal(x0, x1)
