"""Parity at the full size of the 3-D elasticity workload: layered Young's
modulus 1 / 1e5 and Poisson ratio 0.3 / 0.45, 48^3 nodes with the face x = 0
clamped (n = 324864, 3 dofs per node), 8x8x8 geometric subdomains, overlap 1,
lambda > 10 with at most 20 kept modes per subdomain (the capped selection),
three levels.  As for the diffusion workload, the oracle cannot run the whole
setup, so:

* index sets of all 512 subdomains: bit-exact;
* sigma_1 and the kept eigenvalues on a size-stratified sample of subdomains:
  oracle per subdomain, with the same cap;
* the solve: the true relative residual of the returned x, recomputed on the
  CPU with an FP64 SpMV, is <= 1e-8; three levels were built; n_C equals the
  sum of the per-subdomain counts.
"""
import sys
import time

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import DD_SEL_THRESHOLD_CAP, DeviceCSR, Preconditioner  # noqa: E402

MU_FLOOR = 1e-6
MU_RTOL = 1e-4


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


_STATE = {}


def residual_floor(A, x, b):
    """Rounding bound of a relative residual evaluated in FP64: each entry of
    b - A x carries an error below k eps (|b| + |A| |x|), k the longest row, so
    two evaluations (GPU, CPU) may differ by up to twice that in norm."""
    k = int(np.diff(A.indptr).max()) + 1
    return 2 * k * 2.2e-16 * np.linalg.norm(np.abs(b) + abs(A) @ np.abs(x)) / np.linalg.norm(b)


def state():
    if not _STATE:
        cfg = W.config_c3()
        log(f"[elasticity] building 48^3 elasticity: n={cfg.A.n} nnz={cfg.A.nnz} N={cfg.N} delta={cfg.overlap} "
            f"tau={cfg.tau} levels={cfg.levels} nev_cap={cfg.nev_cap}")
        dA = DeviceCSR.from_workload(cfg.A)
        t0 = time.perf_counter()
        pre = Preconditioner(dA, cfg.part, cfg.N, cfg.overlap, cfg.tau, levels=cfg.levels,
                             select=DD_SEL_THRESHOLD_CAP, nev_cap=cfg.nev_cap)
        torch.cuda.synchronize()
        log(f"[elasticity] setup {time.perf_counter() - t0:.2f}s")
        A = O.as_scipy(cfg.A)
        sets = O.subdomain_sets(A, cfg.part, cfg.N, cfg.overlap)
        _STATE.update(cfg=cfg, dA=dA, pre=pre, A=A, sets=sets)
    return _STATE


def test_elasticity_sets_bit_exact():
    st = state()
    pre = st["pre"]
    for i, s in enumerate(st["sets"]):
        I, G, D = pre.sets(i)
        np.testing.assert_array_equal(I, s.I)
        np.testing.assert_array_equal(G, s.Gamma)
        np.testing.assert_array_equal(D, s.Delta)


def test_elasticity_sampled_eigenvalues():
    st = state()
    pre, sets, A, cfg = st["pre"], st["sets"], st["A"], st["cfg"]
    ni = np.array([s.Omega.size for s in sets])
    order = np.argsort(ni, kind="stable")
    sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    sizes = pre.sizes()
    s1 = pre.sigma1()
    for i in sample:
        s = sets[i]
        log(f"[elasticity] oracle subdomain {i}: n_I={s.I.size} n_i={s.Omega.size} n~_i={s.Omega_ext.size}")
        Aii, Xi = O.extract(A, s)
        spl = O.local_splitting(Xi, s.I.size, s.Gamma.size)
        mu_all, mu_keep, _ = O.local_eigen(Aii, spl.S_I, s.I.size, cfg.tau, cfg.nev_cap)
        assert abs(s1[i] - spl.sigma1) <= 1e-9 * spl.sigma1
        below = np.sort(mu_all[mu_all < cfg.tau])
        near = np.abs(mu_all - cfg.tau) <= 1e-6 * cfg.tau
        if below.size > cfg.nev_cap:  # the cap decides: no tie at the cut
            near = near | (np.abs(mu_all - below[cfg.nev_cap - 1]) <= 1e-9 * below[cfg.nev_cap - 1]).any()
        if not np.any(near):
            assert sizes[i, 3] == mu_keep.size, (i, sizes[i, 3], mu_keep.size)
        mu_g = pre.eigs(i)
        k = min(mu_g.size, mu_keep.size)
        big = mu_keep[:k] >= MU_FLOOR
        if big.any():
            rel = np.abs(mu_g[:k][big] - mu_keep[:k][big]) / mu_keep[:k][big]
            log(f"[elasticity] subdomain {i}: p={mu_keep.size}, worst kept-mu rel error {rel.max():.2e}")
            assert rel.max() <= MU_RTOL


def test_elasticity_solve_residual():
    st = state()
    pre, A = st["pre"], st["A"]
    info = pre.info()
    assert info["levels"] == 3
    sizes = pre.sizes()
    assert info["n_C"] == int(sizes[:, 3].sum())
    assert int(sizes[:, 3].max()) <= st["cfg"].nev_cap
    b_h = W.rhs(A.shape[0], 0)
    b = torch.as_tensor(b_h, device="cuda:0")
    t0 = time.perf_counter()
    x, its, rr, code = pre.pcg(b, rtol=1e-8, maxit=1000)
    torch.cuda.synchronize()
    assert code == 0
    x_h = x.cpu().numpy().reshape(-1)
    true_rr = np.linalg.norm(b_h - A @ x_h) / np.linalg.norm(b_h)
    log(f"[elasticity] n_C={info['n_C']} PCG its={its[0]} ({time.perf_counter() - t0:.2f}s) "
        f"relres(gpu)={rr[0]:.3e} relres(cpu spmv)={true_rr:.3e}")
    assert true_rr <= 1e-8
    assert abs(true_rr - rr[0]) <= 1e-3 * true_rr + residual_floor(A, x_h, b_h)


def test_elasticity_threshold_two_levels():
    """The same matrix and partition with the plain threshold selection (every
    mode with lambda > 10 kept) and two levels: the coarse space the bound of
    Sec. 3.2 asks for (n_C about 2.1e5, factored by the supernodal Cholesky),
    which brings PCG from hundreds of iterations with the cap to a few tens."""
    st = state()
    cfg, A = st["cfg"], st["A"]
    t0 = time.perf_counter()
    pre = Preconditioner(st["dA"], cfg.part, cfg.N, cfg.overlap, cfg.tau, levels=2)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    info = pre.info()
    sizes = pre.sizes()
    assert info["levels"] == 2 and info["n_C"] == int(sizes[:, 3].sum())
    b_h = W.rhs(A.shape[0], 0)
    t0 = time.perf_counter()
    x, its, rr, code = pre.pcg(torch.as_tensor(b_h, device="cuda:0"), rtol=1e-8, maxit=1000)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    x_h = x.cpu().numpy().reshape(-1)
    true_rr = np.linalg.norm(b_h - A @ x_h) / np.linalg.norm(b_h)
    log(f"[elasticity] threshold, 2 levels: n_C={info['n_C']} setup {ts:.2f}s, PCG its={its[0]} ({tp:.2f}s) "
        f"relres {true_rr:.3e}")
    assert code == 0 and true_rr <= 1e-8
    assert its[0] <= 60
    del pre
    torch.cuda.empty_cache()


def test_elasticity_cap_256_two_levels():
    """Cap 256 per subdomain (threshold and cap) on two levels: the smallest
    cap of the sweep 32..256 within twice the threshold's iterations (the
    near-kernel cluster of an interior subdomain holds 456 modes, so smaller
    caps leave most of it out: 179 iterations at 128, 392 at 64)."""
    st = state()
    cfg, A = st["cfg"], st["A"]
    pre = Preconditioner(st["dA"], cfg.part, cfg.N, cfg.overlap, cfg.tau, levels=2, select=DD_SEL_THRESHOLD_CAP,
                         nev_cap=256)
    info = pre.info()
    assert int(pre.sizes()[:, 3].max()) <= 256
    b_h = W.rhs(A.shape[0], 0)
    x, its, rr, code = pre.pcg(torch.as_tensor(b_h, device="cuda:0"), rtol=1e-8, maxit=1000)
    x_h = x.cpu().numpy().reshape(-1)
    true_rr = np.linalg.norm(b_h - A @ x_h) / np.linalg.norm(b_h)
    log(f"[elasticity] cap 256, 2 levels: n_C={info['n_C']} PCG its={its[0]} relres {true_rr:.3e}")
    assert code == 0 and true_rr <= 1e-8
    assert its[0] <= 60
    del pre
    torch.cuda.empty_cache()


@pytest.mark.parametrize("levels,cap", [(3, True), (2, False)], ids=["capped_3_levels", "threshold_2_levels"])
def test_elasticity_deflated_gmres(levels, cap):
    """The deflated variant of the paper's experiments on the same matrix and
    partition: flexible GMRES(30) with GMRES(30) coarse solves to 1e-4 for the
    capped selection on three levels, GMRES(30) for the plain threshold on two;
    the true residual recomputed on the CPU reaches 1e-8."""
    from paper_2109_05908_amd import DD_SCHWARZ_DEFLATED
    st = state()
    cfg, A = st["cfg"], st["A"]
    kw = dict(select=DD_SEL_THRESHOLD_CAP, nev_cap=cfg.nev_cap) if cap else {}
    t0 = time.perf_counter()
    pre = Preconditioner(st["dA"], cfg.part, cfg.N, cfg.overlap, cfg.tau, levels=levels,
                         schwarz=DD_SCHWARZ_DEFLATED, **kw)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    info = pre.info()
    assert info["levels"] == levels
    b_h = W.rhs(A.shape[0], 0)
    t0 = time.perf_counter()
    x, its, rr, code = pre.gmres(torch.as_tensor(b_h, device="cuda:0"), rtol=1e-8, maxit=2000)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    x_h = x.cpu().numpy().reshape(-1)
    true_rr = np.linalg.norm(b_h - A @ x_h) / np.linalg.norm(b_h)
    log(f"[elasticity] deflated, {'capped' if cap else 'threshold'}, {levels} levels: n_C={info['n_C']} "
        f"setup {ts:.2f}s, GMRES its={its[0]} ({tg:.2f}s) relres(gpu)={rr[0]:.3e} relres(cpu spmv)={true_rr:.3e}")
    assert code == 0 and true_rr <= 1e-8
    floor = residual_floor(A, x_h, b_h)
    log(f"[elasticity] residual rounding floor {floor:.1e}")
    assert abs(true_rr - rr[0]) <= 1e-3 * true_rr + floor
    del pre
    torch.cuda.empty_cache()
