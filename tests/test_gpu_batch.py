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


def test_batch_graph_pcg_equals_host_loop():
    """graph_pcg on a batch handle: the captured iteration with one set of
    scalars and one stopping test per system gives every system the host
    loop's iterations, residuals and iterates bit for bit, also with FP32
    local solves, several right-hand sides and a maxit stop."""
    from paper_2109_05908_amd import DD_FP32
    sysl = _systems()
    As = [DeviceCSR.from_workload(A) for A, _, _ in sysl]
    parts, Ns = [p for _, p, _ in sysl], [N for _, _, N in sysl]
    ns = [A.n for A, _, _ in sysl]
    b = np.stack([np.concatenate([W.rhs(n, 40 + 3 * j + k) for j, n in enumerate(ns)]) for k in range(3)], axis=1)
    bt = torch.as_tensor(b, device="cuda")
    for prec in (0, DD_FP32):
        host = Preconditioner.batch(As, parts, Ns, 1, 0.1, local_prec=prec)
        graph = Preconditioner.batch(As, parts, Ns, 1, 0.1, local_prec=prec, graph_pcg=8)
        for maxit, want in ((1000, 0), (3, 1)):
            log(f"[batch-graph] local_prec={prec} maxit={maxit}")
            x0, i0, r0, c0 = host.pcg(bt, rtol=1e-10, maxit=maxit)
            x1, i1, r1, c1 = graph.pcg(bt, rtol=1e-10, maxit=maxit)
            assert c0 == c1 == want
            assert i0 == i1 and r0 == r1
            assert torch.equal(x0, x1)
            if want == 0:
                assert len(set(i0[:3])) > 1  # the systems stop at their own counts


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


def test_batch_update_values_three_levels_equals_fresh_batch():
    """dd_update_values on a three-level batch handle: every level is partitioned
    system by system again, so the result equals a fresh dd_setup_batch on the new
    values (same applies bit for bit, same per-system iterations and solutions)."""
    sysl = _systems()
    As = [DeviceCSR.from_workload(A) for A, _, _ in sysl]
    parts, Ns = [p for _, p, _ in sysl], [N for _, _, N in sysl]
    pre = Preconditioner.batch(As, parts, Ns, 1, 0.1, levels=3, coarsen=4)
    A2b = W.diffusion3d(10, seed=4)  # same pattern as system 1, new coefficients
    assert np.array_equal(A2b.colind, sysl[1][0].colind)
    newvals = [sysl[0][0].val * 2.0, A2b.val, sysl[2][0].val]
    log("[batch] update_values on a 3-level batch handle")
    pre.update_values(np.concatenate(newvals))
    As2 = [DeviceCSR(A.n, A.rowptr, A.colind, v) for (A, _, _), v in zip(sysl, newvals)]
    fresh = Preconditioner.batch(As2, parts, Ns, 1, 0.1, levels=3, coarsen=4)
    assert pre.info()["n"] == fresh.info()["n"]
    ns = [A.n for A, _, _ in sysl]
    r = torch.as_tensor(np.concatenate([W.rhs(n, 30 + j) for j, n in enumerate(ns)]), device="cuda")
    assert torch.equal(pre.apply(r), fresh.apply(r))
    b = torch.as_tensor(np.concatenate([W.rhs(n, j) for j, n in enumerate(ns)]), device="cuda")
    x, its, rr, code = pre.pcg(b, rtol=1e-12, maxit=1000)
    xf, itsf, rrf, codef = fresh.pcg(b, rtol=1e-12, maxit=1000)
    log(f"[batch] after update its {its}, fresh {itsf}")
    assert code == 0 and its == itsf and torch.equal(x, xf)


def test_batch_system_without_coarse_modes_at_four_levels():
    """A system that keeps no coarse mode (one subdomain: every lambda is ~1) next
    to one that does, with four levels: the level-1 partition skips the empty
    system and each system still gets the solve of its own setup."""
    A1 = W.poisson2d(32)
    p1 = W.grid2d_partition(32, 4, 4)
    A2 = W.poisson2d(12)
    p2 = np.zeros(A2.n, dtype=np.int32)
    As = [DeviceCSR.from_workload(A1), DeviceCSR.from_workload(A2)]
    log("[batch] 4 levels, second system with a single subdomain")
    pre = Preconditioner.batch(As, [p1, p2], [16, 1], 1, 0.1, levels=4, coarsen=4)
    b1, b2 = W.rhs(A1.n, 1), W.rhs(A2.n, 2)
    x, its, rr, code = pre.pcg(torch.as_tensor(np.concatenate([b1, b2]), device="cuda"), rtol=1e-12, maxit=500)
    assert code == 0
    xg = x.cpu().numpy()
    s1 = Preconditioner(As[0], p1, 16, 1, 0.1, levels=4, coarsen=4)
    s2 = Preconditioner(As[1], p2, 1, 1, 0.1, levels=4, coarsen=4)
    assert s2.info()["n_C"] == 0
    x1, i1, _, _ = s1.pcg(torch.as_tensor(b1, device="cuda"), rtol=1e-12, maxit=500)
    x2, i2, _, _ = s2.pcg(torch.as_tensor(b2, device="cuda"), rtol=1e-12, maxit=500)
    log(f"[batch] its batch {its}, separate {i1[0]} {i2[0]}")
    assert abs(its[0] - i1[0]) <= 1 and its[1] == i2[0] == 1
    x1 = x1.cpu().numpy()
    assert np.linalg.norm(xg[:A1.n] - x1) <= 1e-10 * np.linalg.norm(x1)
    assert np.linalg.norm(xg[A1.n:] - x2.cpu().numpy()) <= 1e-10 * np.linalg.norm(x2.cpu().numpy())


def test_batch_validates_each_system_and_refuses_deflated():
    """validate checks every system's own CSR before the union is formed (a column
    index of system 0 that is out of its range but inside the union is caught, and
    so is a wrong rowptr[n_0]); the deflated variant is refused for a batch."""
    from paper_2109_05908_amd import DD_SCHWARZ_DEFLATED, DDError
    A1 = W.poisson2d(12)
    A2 = W.poisson2d(10)
    p1 = W.grid2d_partition(12, 2, 2)
    p2 = W.grid2d_partition(10, 2, 2)
    good = [DeviceCSR.from_workload(A1), DeviceCSR.from_workload(A2)]
    ok = Preconditioner.batch(good, [p1, p2], [4, 4], 1, 0.1, validate=True)
    assert ok.info()["n_C"] > 0
    ix = A1.colind.copy()
    ix[A1.rowptr[A1.n] - 1] = A1.n + 3  # last entry of the last row: beyond n_0, inside the union
    bad_col = DeviceCSR(A1.n, A1.rowptr, ix, A1.val)
    rp = A1.rowptr.copy()
    rp[A1.n] -= 1
    bad_end = DeviceCSR(A1.n, rp, A1.colind, A1.val)
    for bad in (bad_col, bad_end):
        with pytest.raises(DDError) as e:
            Preconditioner.batch([bad, good[1]], [p1, p2], [4, 4], 1, 0.1, validate=True)
        assert e.value.code == -1
    with pytest.raises(DDError) as e:
        Preconditioner.batch(good, [p1, p2], [4, 4], 1, 0.1, schwarz=DD_SCHWARZ_DEFLATED)
    assert e.value.code == -1
