"""Further parity cases through the C-ABI:

* several right-hand sides in one call: dd_apply, dd_pcg and dd_gmres on an
  n x 3 block (column-major) give, column by column, bit for bit what single
  calls give;
* four levels (the 64 x 64 Poisson problem in 64 geometric parts, coarsened
  by 4: 64 -> 16 -> 4): the sets of levels 1 and 2 bit-exact against the
  oracle, flexible CG to 1e-13 with x within 1e-10 of the oracle's;
* a batch of the three workload types (2-D Poisson, 3-D high-contrast
  diffusion, layered elasticity) and a random graph, three right-hand sides:
  every system and column solved as by its own setup (iterations within 1, x
  within 1e-10);
* FP32 local solves under the deflated variant: flexible GMRES reaches 1e-13
  and x agrees with the oracle's FP64 deflated solve to 1e-10.
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

from paper_2109_05908_amd import DD_FP32, DD_SCHWARZ_DEFLATED, DeviceCSR, Preconditioner  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_multiple_right_hand_sides():
    cfg = W.config_small3d(16, 16)
    part = O.ggg_partition(cfg.A, cfg.N, cfg.ggg_seed)
    dA = DeviceCSR.from_workload(cfg.A)
    B = torch.as_tensor(W.rhs(cfg.A.n, 7, nrhs=3).reshape(cfg.A.n, 3), device="cuda")
    for schwarz in (0, DD_SCHWARZ_DEFLATED):
        pre = Preconditioner(dA, part, cfg.N, cfg.overlap, cfg.tau, schwarz=schwarz)
        Z = pre.apply(B).cpu().numpy()
        solve = pre.gmres if schwarz else pre.pcg
        X, its, rr, code = solve(B, rtol=1e-12)
        X = X.cpu().numpy()
        assert code == 0 and len(its) == 3
        for k in range(3):
            bk = B[:, k].contiguous()
            np.testing.assert_array_equal(Z[:, k], pre.apply(bk).cpu().numpy())
            xk, itk, rrk, _ = solve(bk, rtol=1e-12)
            assert itk[0] == its[k] and rrk[0] == rr[k]
            np.testing.assert_array_equal(X[:, k], xk.cpu().numpy())
        log(f"[more] 3 right-hand sides, schwarz={schwarz}: its {its}")


def test_four_levels():
    cfg = W.config_c1()
    part = W.grid2d_partition(64, 8, 8)
    N = 64
    pre = Preconditioner(DeviceCSR.from_workload(cfg.A), part, N, 1, cfg.tau, levels=4, coarsen=4)
    info = pre.info()
    assert info["levels"] == 4
    ora = O.build(cfg.A, part, N, 1, cfg.tau, levels=4, coarsen=4)
    for lvl, o in ((1, ora.inner), (2, ora.inner.inner)):
        assert pre.count(lvl) == len(o.locals)
        for i, L in enumerate(o.locals):
            I, G, D = pre.sets(i, level=lvl)
            np.testing.assert_array_equal(I, L.sets.I)
            np.testing.assert_array_equal(G, L.sets.Gamma)
            np.testing.assert_array_equal(D, L.sets.Delta)
    b = W.rhs(cfg.A.n, 5)
    x, its, rr, code = pre.pcg(torch.as_tensor(b, device="cuda"), rtol=1e-13, maxit=500)
    xo, itso, _ = O.flexible_pcg(cfg.A, b, ora.apply, rtol=1e-13, maxit=500)
    log(f"[more] 4 levels: N per level {info['N']}, its gpu {its[0]} oracle {itso}, relres {rr[0]:.2e}")
    assert code == 0 and rr[0] <= 2e-13 and abs(its[0] - itso) <= 2
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


def test_batch_mixed_types_multi_rhs():
    e = W.config_small_elasticity()
    A2 = W.diffusion3d(10, seed=3)
    A4 = W.random_spd(500, 5, seed=9, positive_offdiag=True)
    sysl = [(W.poisson2d(32), W.grid2d_partition(32, 2, 2), 4), (A2, O.ggg_partition(A2, 8, 0), 8),
            (e.A, e.part, e.N), (A4, O.ggg_partition(A4, 4, 0), 4)]
    As = [DeviceCSR.from_workload(A) for A, _, _ in sysl]
    pre = Preconditioner.batch(As, [p for _, p, _ in sysl], [N for _, _, N in sysl], 1, 0.1)
    ns = [A.n for A, _, _ in sysl]
    off = np.concatenate([[0], np.cumsum(ns)])
    nrhs, nsys = 3, len(sysl)
    Bh = np.concatenate([W.rhs(n, 30 + j, nrhs=nrhs).reshape(n, nrhs) for j, n in enumerate(ns)])
    X, its, rr, code = pre.pcg(torch.as_tensor(Bh, device="cuda"), rtol=1e-13, maxit=1000)
    assert code == 0 and len(its) == nrhs * nsys
    X = X.cpu().numpy()
    for j, ((A, p, N), dA) in enumerate(zip(sysl, As)):
        P = Preconditioner(dA, p, N, 1, 0.1)
        Bj = torch.as_tensor(np.ascontiguousarray(Bh[off[j]:off[j + 1]]), device="cuda")
        Xs, itss, _, _ = P.pcg(Bj, rtol=1e-13, maxit=1000)
        Xs = Xs.cpu().numpy()
        for k in range(nrhs):
            its_b = its[k * nsys + j]
            assert rr[k * nsys + j] <= 2e-13 and abs(its_b - itss[k]) <= 1
            xs = Xs[:, k]
            assert np.linalg.norm(X[off[j]:off[j + 1], k] - xs) <= 1e-10 * np.linalg.norm(xs)
        log(f"[more] batch system {j} (n={A.n}): its per RHS {[its[k * nsys + j] for k in range(nrhs)]}, "
            f"separate {itss}")


def test_fp32_local_solves_deflated_gmres():
    cfg = W.config_small3d(16, 16)
    part = O.ggg_partition(cfg.A, cfg.N, cfg.ggg_seed)
    pre = Preconditioner(DeviceCSR.from_workload(cfg.A), part, cfg.N, cfg.overlap, cfg.tau, local_prec=DD_FP32,
                         schwarz=DD_SCHWARZ_DEFLATED)
    ora = O.build(cfg.A, part, cfg.N, cfg.overlap, cfg.tau, variant="deflated")
    b = W.rhs(cfg.A.n, 6)
    x, its, rr, code = pre.gmres(torch.as_tensor(b, device="cuda"), rtol=1e-13, maxit=600)
    xo, itso, _ = O.gmres(cfg.A, b, ora.apply, rtol=1e-13, maxit=600)
    log(f"[more] FP32 local solves, deflated: GMRES its {its[0]} (oracle FP64 {itso}), relres {rr[0]:.2e}")
    assert code == 0 and rr[0] <= 1e-13
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


def test_gmres_edge_cases():
    # a system smaller than the restart length: Arnoldi ends on a happy breakdown
    A = W.poisson2d(4)
    part = W.grid2d_partition(4, 2, 1)
    pre = Preconditioner(DeviceCSR.from_workload(A), part, 2, 1, 1e-30, schwarz=DD_SCHWARZ_DEFLATED)
    b = W.rhs(A.n, 1)
    x, its, rr, code = pre.gmres(torch.as_tensor(b, device="cuda"), rtol=1e-13, restart=30)
    xd = np.linalg.solve(A.to_scipy().toarray(), b)
    log(f"[more] n={A.n} with restart 30: its {its[0]}, relres {rr[0]:.2e}")
    assert code == 0 and its[0] <= A.n and rr[0] <= 1e-13
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-10 * np.linalg.norm(xd)
    # maxit reached: the warning code, the iterations done and the true residual of the iterate
    cfg = W.config_c1()
    pre = Preconditioner(DeviceCSR.from_workload(cfg.A), cfg.part, cfg.N, cfg.overlap, cfg.tau)
    b = W.rhs(cfg.A.n, 2)
    x, its, rr, code = pre.gmres(torch.as_tensor(b, device="cuda"), rtol=1e-13, maxit=3, restart=2)
    true = np.linalg.norm(b - cfg.A.to_scipy() @ x.cpu().numpy()) / np.linalg.norm(b)
    assert code == 1 and its[0] == 3
    assert abs(true - rr[0]) <= 1e-10 * true and 1e-13 < true < 1.0


def test_block_pcg_many_columns():
    """Eleven right-hand sides in one dd_pcg call run as two groups of at most
    eight columns in lockstep (A and every local inverse read once per group).
    With a zero column, a column started from an already converged x0, FP64
    and FP32 local solves, and a stop at maxit, every column equals its own
    single call bit for bit (iterations, residual, iterate), and dd_apply on
    the block equals the column-by-column apply."""
    cfg = W.config_c1()
    n = cfg.A.n
    dA = DeviceCSR.from_workload(cfg.A)
    B = torch.as_tensor(W.rhs(n, 11, nrhs=11).reshape(n, 11), device="cuda").clone()
    B[:, 3] = 0.0
    for prec in (0, DD_FP32):
        pre = Preconditioner(dA, cfg.part, 16, 1, 0.1, local_prec=prec)
        xs, _, _, _ = pre.pcg(B[:, 5].contiguous(), rtol=1e-13)
        X0 = torch.zeros_like(B)
        X0[:, 5] = xs
        Z = pre.apply(B)
        for k in range(11):
            assert torch.equal(Z[:, k], pre.apply(B[:, k].contiguous()))
        for rtol, maxit in ((1e-10, 1000), (1e-12, 4)):
            X, its, rr, code = pre.pcg(B, x0=X0, rtol=rtol, maxit=maxit)
            for k in range(11):
                xk, itk, rrk, _ = pre.pcg(B[:, k].contiguous(), x0=X0[:, k].contiguous(), rtol=rtol, maxit=maxit)
                assert itk[0] == its[k] and rrk[0] == rr[k], (prec, rtol, k, itk, its[k])
                assert torch.equal(X[:, k], xk)
            log(f"[more] 11 columns, prec {prec}, rtol {rtol}, maxit {maxit}: code {code}, its {its}")
            assert its[3] == 0 and rr[3] == 0.0 and its[5] == 0
