"""Pins of the oracle's deflated variant (Sec. 4: M_deflated with the one-level
restricted additive Schwarz method) and of its right-preconditioned GMRES,
against facts that follow from the definitions and from GMRES's minimal
residual property, not from the oracle's own code paths (CPU only).

* RAS locality: a row of Omega_i couples only to Omega_i and Delta_i, so
  R_i A u = A_ii R_i u whenever u vanishes on Delta_i; with the Boolean D_i the
  restricted method then returns u on Omega_Ii, and M_RAS A u = u for every u
  that vanishes on all the Delta_i.  The additive method returns the
  multiplicity times u there, so the pin tells the two apart on overlap dofs.
* Deflation: Z^T A Z = E gives M_deflated A Z = Z whatever the one-level part.
* Full coarse space (every mode kept): Z E^{-1} Z^T = A^{-1} and the one-level
  correction vanishes, so M_deflated = A^{-1}; one subdomain: M_RAS = A^{-1}.
* GMRES: the k-th iterate minimises ||b - A x|| over M K_k(A M, b), checked by
  least squares on an explicit Krylov basis (also across a restart); with
  M = A^{-1} it stops after one step; with M = I on a matrix of d distinct
  eigenvalues after d steps; the flexible form with a fixed M gives the same
  iterates.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
import workloads as W


def _dense(A):
    return O.as_scipy(A).toarray()


def _cases():
    A1 = W.poisson2d(24)
    A2 = W.random_spd(120, 5, seed=4, positive_offdiag=True)
    A3 = W.diffusion3d(8, seed=1)
    return [
        ("poisson2d", A1, W.grid2d_partition(24, 3, 2), 6, 1, 0.1),
        ("poisson2d_d2", A1, W.grid2d_partition(24, 2, 2), 4, 2, 0.1),
        ("random_spd", A2, O.ggg_partition(A2, 4, 0), 4, 1, 0.1),
        ("diffusion3d", A3, O.ggg_partition(A3, 8, 0), 8, 1, 0.05),
    ]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_ras_locality(case):
    _, A, part, N, delta, tau = case
    pre = O.build(A, part, N, delta, tau)
    n = pre.n
    in_delta = np.zeros(n, dtype=bool)
    in_gamma = np.zeros(n, dtype=bool)
    for L in pre.locals:
        in_delta[L.sets.Delta] = True
        in_gamma[L.sets.Gamma] = True
    free = ~in_delta
    # the pin must reach overlap dofs, where the additive method differs
    assert (free & in_gamma).any()
    rng = np.random.default_rng(3)
    u = np.where(free, rng.standard_normal(n), 0.0)
    Au = pre.A @ u
    z = pre.apply_ras(Au)
    assert np.linalg.norm(z - u) <= 1e-11 * np.linalg.norm(u)
    za = pre.apply_local(Au)
    assert np.linalg.norm((za - u)[free & in_gamma]) > 0.1 * np.linalg.norm(u[free & in_gamma])


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_deflation_identity(case):
    _, A, part, N, delta, tau = case
    pre = O.build(A, part, N, delta, tau, variant="deflated")
    assert pre.nC > 0
    Z = pre.Z.toarray()
    worst = 0.0
    for k in range(0, pre.nC, max(1, pre.nC // 40)):
        z = Z[:, k]
        got = pre.apply(pre.A @ z)
        worst = max(worst, np.linalg.norm(got - z) / np.linalg.norm(z))
    assert worst <= 1e-9


def test_full_coarse_space_deflated_is_inverse():
    A = W.random_spd(150, 5, seed=7, positive_offdiag=True)
    part = O.ggg_partition(A, 4, 0)
    pre = O.build(A, part, 4, 1, 1.5, variant="deflated")
    assert pre.nC == A.n
    Ad = _dense(A)
    r = W.rhs(A.n, 2)
    x = np.linalg.solve(Ad, r)
    assert np.linalg.norm(pre.apply(r) - x) <= 1e-10 * np.linalg.norm(x)


def test_single_subdomain_ras_is_inverse():
    A = W.poisson2d(16)
    part = np.zeros(A.n, dtype=np.int32)
    pre = O.build(A, part, 1, 1, 0.1, variant="deflated")
    assert pre.nC == 0
    r = W.rhs(A.n, 3)
    x = np.linalg.solve(_dense(A), r)
    assert np.linalg.norm(pre.apply_ras(r) - x) <= 1e-12 * np.linalg.norm(x)
    assert np.linalg.norm(pre.apply(r) - x) <= 1e-12 * np.linalg.norm(x)


def _krylov_min(A, M, x0, r0, k):
    """argmin of ||b - A x|| over x0 + M K_k(A M, r0), by least squares on an
    orthonormalised explicit Krylov basis (tiny k only)."""
    K = np.empty((r0.size, k))
    v = r0 / np.linalg.norm(r0)
    for j in range(k):
        K[:, j] = v
        v = A @ (M @ v)
        v = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(K)
    B = A @ (M @ Q)
    c, *_ = np.linalg.lstsq(B, r0, rcond=None)
    return x0 + M @ (Q @ c)


def _nonsymmetric_case():
    A = W.random_spd(60, 5, seed=11, positive_offdiag=True)
    part = O.ggg_partition(A, 3, 0)
    pre = O.build(A, part, 3, 1, 0.05, variant="deflated")
    Ad = _dense(A)
    M = np.column_stack([pre.apply(e) for e in np.eye(A.n)])
    assert np.linalg.norm(M - M.T) > 1e-3 * np.linalg.norm(M)  # M_deflated is not symmetric
    return Ad, M


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_gmres_minimal_residual(k):
    Ad, M = _nonsymmetric_case()
    b = W.rhs(Ad.shape[0], 5)
    x, its, _ = O.gmres(sp.csr_matrix(Ad), b, lambda v: M @ v, rtol=1e-300, restart=30, maxit=k)
    assert its == k
    xb = _krylov_min(Ad, M, np.zeros_like(b), b, k)
    assert np.linalg.norm(x - xb) <= 1e-8 * np.linalg.norm(xb)


def test_gmres_restart_minimal_residual():
    Ad, M = _nonsymmetric_case()
    b = W.rhs(Ad.shape[0], 6)
    m, k = 3, 5
    x, its, _ = O.gmres(sp.csr_matrix(Ad), b, lambda v: M @ v, rtol=1e-300, restart=m, maxit=k)
    assert its == k
    x1 = _krylov_min(Ad, M, np.zeros_like(b), b, m)
    x2 = _krylov_min(Ad, M, x1, b - Ad @ x1, k - m)
    assert np.linalg.norm(x - x2) <= 1e-8 * np.linalg.norm(x2)


def test_gmres_exact_preconditioner_one_step():
    A = W.poisson2d(12)
    Ad = _dense(A)
    cf = sla.cho_factor(Ad)
    b = W.rhs(A.n, 1)
    x, its, rr = O.gmres(A, b, lambda v: sla.cho_solve(cf, v), rtol=1e-12)
    assert its == 1 and rr <= 1e-12


def test_gmres_distinct_eigenvalues():
    rng = np.random.default_rng(2)
    d = np.repeat([1.0, 2.5, 4.0, 7.0], 10)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    Ad = (Q * d) @ Q.T
    b = rng.standard_normal(40)
    x, its, rr = O.gmres(sp.csr_matrix(Ad), b, lambda v: v, rtol=1e-12)
    assert its == 4 and rr <= 1e-12


def test_flexible_equals_plain_for_fixed_preconditioner():
    Ad, M = _nonsymmetric_case()
    b = W.rhs(Ad.shape[0], 7)
    A = sp.csr_matrix(Ad)
    x1, i1, r1 = O.gmres(A, b, lambda v: M @ v, rtol=1e-10, restart=4)
    x2, i2, r2 = O.gmres(A, b, lambda v: M @ v, rtol=1e-10, restart=4, flexible=True)
    assert i1 == i2
    assert np.linalg.norm(x1 - x2) <= 1e-10 * np.linalg.norm(x1)


def test_deflated_gmres_solution_against_dense_solve():
    cfg = W.config_c1()
    pre = O.build(cfg.A, cfg.part, cfg.N, cfg.overlap, cfg.tau, variant="deflated")
    b = W.rhs(cfg.A.n, 0)
    x, its, rr = O.gmres(cfg.A, b, pre.apply, rtol=1e-13, maxit=500)
    xd = np.linalg.solve(_dense(cfg.A), b)
    assert rr <= 1e-13
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # the deflated preconditioner needs no more iterations than the additive one
    pa = O.build(cfg.A, cfg.part, cfg.N, cfg.overlap, cfg.tau)
    _, its_a, _ = O.gmres(cfg.A, b, pa.apply, rtol=1e-13, maxit=500)
    assert its <= its_a


def test_three_level_deflated_flexible_gmres_converges():
    cfg = W.config_small3d(12, 16)
    part = O.ggg_partition(cfg.A, cfg.N, cfg.ggg_seed)
    pre = O.build(cfg.A, part, cfg.N, cfg.overlap, cfg.tau, levels=3, coarsen=4, variant="deflated")
    assert pre.inner is not None and pre.inner.variant == "deflated"
    b = W.rhs(cfg.A.n, 1)
    x, its, rr = O.gmres(cfg.A, b, pre.apply, rtol=1e-8, flexible=True)
    assert rr <= 1e-8
    two = O.build(cfg.A, part, cfg.N, cfg.overlap, cfg.tau, variant="deflated")
    _, its2, _ = O.gmres(cfg.A, b, two.apply, rtol=1e-8)
    assert its <= its2 + 3  # inner solves to 1e-4 keep the outer count close to the exact coarse solve
