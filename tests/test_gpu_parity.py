"""GPU path vs the FP64 CPU oracle, through the C-ABI (needs an MI355X).

Tolerances: bit-exact for partitions, sets and index maps; kept eigenvalues
mu = 1/lambda within 1e-4 relative for mu >= 1e-6 (the near-kernel cluster is
compared by count and span); the FP64 solution within 1e-10 relative when
both solvers run to rtol 1e-13.
"""
import sys

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import DeviceCSR, Preconditioner, partition_ggg  # noqa: E402

MU_FLOOR = 1e-6
MU_RTOL = 1e-4


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(name):
    if name == "c1":
        cfg = W.config_c1()
        part = cfg.part
    elif name == "small3d":
        cfg = W.config_small3d(16, 16)
        part = None
    elif name == "rand":
        A = W.random_spd(600, 5, seed=4, positive_offdiag=True)
        cfg = W.Config("random_spd_600", A, None, 6, 1, 0.1, 2)
        part = None
    elif name == "elast":  # layered 3-D elasticity, 3 dofs per node, 2x2x2 geometric parts
        cfg = W.config_small_elasticity()
        part = cfg.part
    else:
        raise KeyError(name)
    if part is None:
        part = O.ggg_partition(cfg.A, cfg.N, cfg.ggg_seed)
    return cfg, part


CASES = ["c1", "small3d", "rand", "elast"]

_CACHE = {}


def built(name):
    if name not in _CACHE:
        cfg, part = _case(name)
        log(f"[parity] building {name}: n={cfg.A.n} N={cfg.N} delta={cfg.overlap} tau={cfg.tau}")
        dA = DeviceCSR.from_workload(cfg.A)
        pre = Preconditioner(dA, part, cfg.N, cfg.overlap, cfg.tau)
        torch.cuda.synchronize()
        ora = O.build(cfg.A, part, cfg.N, cfg.overlap, cfg.tau)
        _CACHE[name] = (cfg, part, dA, pre, ora)
    return _CACHE[name]


@pytest.mark.parametrize("m,N,seed", [(16, 16, 0), (12, 7, 3), (64, 256, 0)])
def test_partition_ggg_bit_exact(m, N, seed):
    A = W.diffusion3d(m, seed=1)
    log(f"[parity] ggg m={m} N={N} seed={seed}")
    got = partition_ggg(DeviceCSR.from_workload(A), N, seed).cpu().numpy()
    np.testing.assert_array_equal(got, O.ggg_partition(A, N, seed))


@pytest.mark.parametrize("name", CASES)
def test_sets_bit_exact(name):
    cfg, part, dA, pre, ora = built(name)
    for i, L in enumerate(ora.locals):
        I, G, D = pre.sets(i)
        np.testing.assert_array_equal(I, L.sets.I)
        np.testing.assert_array_equal(G, L.sets.Gamma)
        np.testing.assert_array_equal(D, L.sets.Delta)


@pytest.mark.parametrize("name", CASES)
def test_sigma1(name):
    cfg, part, dA, pre, ora = built(name)
    s1 = pre.sigma1()
    for i, L in enumerate(ora.locals):
        assert abs(s1[i] - L.split.sigma1) <= 1e-9 * L.split.sigma1


@pytest.mark.parametrize("name", CASES)
def test_kept_eigenvalues(name):
    cfg, part, dA, pre, ora = built(name)
    sizes = pre.sizes()
    worst = 0.0
    for i, L in enumerate(ora.locals):
        mu_o = L.mu_keep
        mu_g = pre.eigs(i)
        # counts: equal unless an oracle eigenvalue sits within 1e-6 (relative) of tau
        near = np.abs(L.mu_all - cfg.tau) <= 1e-6 * cfg.tau
        if not near.any():
            assert sizes[i, 3] == mu_o.size, (i, sizes[i, 3], mu_o.size)
        k = min(mu_o.size, mu_g.size)
        big = mu_o[:k] >= MU_FLOOR
        if big.any():
            rel = np.abs(mu_g[:k][big] - mu_o[:k][big]) / mu_o[:k][big]
            worst = max(worst, rel.max())
    log(f"[parity] {name}: worst kept-mu relative error {worst:.2e}")
    assert worst <= MU_RTOL


EPS = 2.0 ** -52


@pytest.mark.parametrize("name", CASES)
def test_coarse_spans(name):
    """Kept subspaces agree in the A_I (energy) metric within the Davis-Kahan
    estimate of their sensitivity to a backward error of size eps*sigma_1 in
    the shifted square root: angle <= 64 eps sigma_1 / (lambda_min(A_I) gap),
    gap = distance from the kept mu to the first discarded mu."""
    cfg, part, dA, pre, ora = built(name)
    worst_ratio = 0.0
    for i, L in enumerate(ora.locals):
        Zg = pre.basis(i)
        Zo = L.Z_I
        if Zo.shape[1] == 0:
            assert Zg.shape[1] == 0
            continue
        assert Zg.shape[1] == Zo.shape[1]
        np.testing.assert_allclose(Zg.T @ Zg, np.eye(Zg.shape[1]), atol=1e-10)
        nI = L.sets.I.size
        AI = L.Aii[:nI, :nI]
        C = np.linalg.cholesky(AI)
        ang = sla.subspace_angles(C.T @ Zg, C.T @ Zo).max()
        rest = L.mu_all[L.mu_all >= cfg.tau]
        gap = (rest.min() - L.mu_keep.max()) if rest.size else 1.0
        tol = max(1e-9, 64 * EPS * L.split.sigma1 / (np.linalg.eigvalsh(AI).min() * gap))
        worst_ratio = max(worst_ratio, ang / tol)
        assert ang <= tol, (i, ang, tol)
    log(f"[parity] {name}: worst angle/tolerance {worst_ratio:.2e}")


def _gpu_dense_pieces(cfg, pre, ora):
    import scipy.sparse as sp
    n = cfg.A.n
    rows, cols, vals = [], [], []
    off = 0
    for i, L in enumerate(ora.locals):
        Zg = pre.basis(i)
        p = Zg.shape[1]
        rr, cc = np.meshgrid(L.sets.I, np.arange(off, off + p), indexing="ij")
        rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(Zg.ravel())
        off += p
    Z = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, off))
    return Z


@pytest.mark.parametrize("name", CASES)
def test_coarse_operator_definition(name):
    """E assembled on the GPU equals Z^T A Z for the GPU's own Z (E = R_0 A R_0^T, (2.1))."""
    cfg, part, dA, pre, ora = built(name)
    Z = _gpu_dense_pieces(cfg, pre, ora)
    Eref = (Z.T @ (cfg.A.to_scipy() @ Z)).toarray()
    E = pre.coarse_matrix()
    assert np.abs(E - Eref).max() <= 1e-12 * np.abs(Eref).max()
    assert np.linalg.eigvalsh(0.5 * (E + E.T)).min() > 0


@pytest.mark.parametrize("name", CASES)
def test_apply_matches_definition(name):
    """dd_apply = sum_i R_i^T A_ii^{-1} R_i r + Z E^{-1} Z^T r (2.1), evaluated densely
    on the CPU with the GPU's own Z."""
    cfg, part, dA, pre, ora = built(name)
    Z = _gpu_dense_pieces(cfg, pre, ora)
    E = pre.coarse_matrix()
    E = np.tril(E) + np.tril(E, -1).T
    r = W.rhs(cfg.A.n, 11)
    zref = ora.apply_local(r)
    if Z.shape[1]:
        zref = zref + Z @ np.linalg.solve(E, Z.T @ r)
    zg = pre.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
    assert np.linalg.norm(zg - zref) <= 1e-10 * np.linalg.norm(zref)


@pytest.mark.parametrize("name", CASES)
def test_apply_matches_oracle_energy(name):
    """Method-level: for r = A e the coarse part is the A-orthogonal projection
    of e, so GPU and oracle applies agree in the A-norm to the subspace
    sensitivity (loose bound 1e-4; C1 and the random matrix are far tighter)."""
    cfg, part, dA, pre, ora = built(name)
    e = W.rhs(cfg.A.n, 12)
    A = cfg.A.to_scipy()
    r = A @ e
    zg = pre.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
    zo = ora.apply(r)
    d = zg - zo
    rel = np.sqrt(d @ (A @ d)) / np.sqrt(zo @ (A @ zo))
    log(f"[parity] {name}: apply A-norm relative difference {rel:.2e}")
    assert rel <= (1e-10 if name in ("c1", "rand", "elast") else 1e-4)


@pytest.mark.parametrize("name", CASES)
def test_pcg_solution(name):
    cfg, part, dA, pre, ora = built(name)
    b = W.rhs(cfg.A.n, 0)
    x, its, rr, code = pre.pcg(torch.as_tensor(b, device="cuda"), rtol=1e-13, maxit=500)
    xo, itso, rro = O.pcg(cfg.A, b, ora.apply, rtol=1e-13, maxit=500)
    xg = x.cpu().numpy()
    log(f"[parity] {name}: its gpu {its[0]} oracle {itso}, relres {rr[0]:.2e}")
    # the stop is on the recurrence residual; the true residual reported at
    # exit may exceed rtol by the residual gap, which at rtol 1e-13 on the
    # layered elasticity (contrast 1e5) reaches about 10 %
    assert code == 0 and rr[0] <= 2e-13
    assert abs(its[0] - itso) <= 1
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)
    # rtol 1e-8 iteration count
    x8, its8, rr8, _ = pre.pcg(torch.as_tensor(b, device="cuda"), rtol=1e-8)
    _, itso8, _ = O.pcg(cfg.A, b, ora.apply, rtol=1e-8)
    assert abs(its8[0] - itso8) <= 1 and rr8[0] <= 1e-8


def test_c1_expected_coarse_size():
    cfg, part, dA, pre, ora = built("c1")
    info = pre.info()
    assert info["n_C"] == ora.nC == 732
    assert abs(info["grid_complexity"] - (4096 + 732) / 4096) < 1e-12


def test_invalid_partition_rejected():
    cfg = W.config_c1()
    dA = DeviceCSR.from_workload(cfg.A)
    bad = cfg.part.copy()
    bad[5] = 99
    with pytest.raises(Exception) as e:
        Preconditioner(dA, bad, 16, 1, 0.1)
    assert getattr(e.value, "code", None) == -1
