"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
independent of the oracle's own code paths (CPU only).

Each test names the passage it checks.  A plausible mistake in the oracle
(a dropped term, a wrong sign or index, a transposed operand, a wrong set
order) fails at least one of them.
"""
import collections
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------------------
# partition generator (input of the method)
# ---------------------------------------------------------------------------
def test_splitmix64_reference_vectors():
    for seed, *outs in _read_golden("splitmix64.txt"):
        got = O.splitmix64(int(seed), 3)
        assert got == [int(x, 16) for x in outs]


def _ggg_bruteforce(A, N, seed):
    """Sequential vertex-by-vertex restatement of the growing rule."""
    A = O.as_scipy(A)
    n = A.shape[0]
    adj = [set(A.indices[A.indptr[i]:A.indptr[i + 1]]) - {i} for i in range(n)]
    part = [-1] * n
    chosen, k = 0, 0
    vals = O.splitmix64(seed, 4 * n + 64)
    while chosen < N:
        v = vals[k] % n
        k += 1
        if part[v] < 0:
            part[v] = chosen
            chosen += 1
    frontier = {v for v in range(n) if part[v] >= 0}
    while frontier:
        newp = {}
        for v in range(n):
            if part[v] < 0:
                ids = [part[u] for u in adj[v] if u in frontier]
                if ids:
                    newp[v] = min(ids)
        for v, p in newp.items():
            part[v] = p
        frontier = set(newp)
    sizes = collections.Counter(p for p in part if p >= 0)
    if any(p < 0 for p in part):
        smallest = min(range(N), key=lambda i: (sizes.get(i, 0), i))
        part = [smallest if p < 0 else p for p in part]
    return np.array(part, dtype=np.int32)


@pytest.mark.parametrize("maker", [
    lambda: W.poisson2d(9),
    lambda: W.laplace1d(31),
    lambda: W.random_spd(60, 3, seed=3),
    lambda: W.diffusion3d(5, seed=1),
])
def test_ggg_matches_bruteforce(maker):
    A = maker()
    for N in (1, 3, 7):
        for seed in (0, 11):
            np.testing.assert_array_equal(O.ggg_partition(A, N, seed), _ggg_bruteforce(A, N, seed))


def test_ggg_disconnected_remainder_goes_to_smallest_part():
    # two disconnected paths; N=2 seeds may both land in one component
    A1 = W.laplace1d(10).to_scipy()
    A = sp.block_diag([A1, A1]).tocsr()
    for seed in range(6):
        p = O.ggg_partition(A, 2, seed)
        assert set(np.unique(p)) <= {0, 1}
        np.testing.assert_array_equal(p, _ggg_bruteforce(A, 2, seed))


# ---------------------------------------------------------------------------
# Sec. 2: sets Omega_Ii, Gamma_i, Delta_i
# ---------------------------------------------------------------------------
def _bfs_dist(A, sources):
    A = O.as_scipy(A)
    n = A.shape[0]
    dist = np.full(n, -1)
    dq = collections.deque()
    for s in sources:
        dist[s] = 0
        dq.append(s)
    while dq:
        v = dq.popleft()
        for u in A.indices[A.indptr[v]:A.indptr[v + 1]]:
            if dist[u] < 0:
                dist[u] = dist[v] + 1
                dq.append(u)
    return dist


@pytest.mark.parametrize("delta", [1, 2, 3])
def test_sets_match_bfs_distances(delta):
    for A, part, N in [
        (W.poisson2d(12), W.grid2d_partition(12, 3, 2), 6),
        (W.random_spd(80, 4, seed=5), None, 5),
    ]:
        if part is None:
            part = O.ggg_partition(A, N, 2)
        sets = O.subdomain_sets(A, part, N, delta)
        for i, s in enumerate(sets):
            d = _bfs_dist(A, np.flatnonzero(part == i))
            np.testing.assert_array_equal(s.I, np.flatnonzero(d == 0))
            np.testing.assert_array_equal(s.Gamma, np.flatnonzero((d >= 1) & (d <= delta)))
            np.testing.assert_array_equal(s.Delta, np.flatnonzero(d == delta + 1))


def test_c1_sizes_closed_form():
    cfg = W.config_c1()
    sets = O.subdomain_sets(cfg.A, cfg.part, cfg.N, cfg.overlap)
    gold = {r[0]: tuple(int(x) for x in r[1:]) for r in _read_golden("c1_subdomain_sizes.txt")}
    for i, s in enumerate(sets):
        by, bx = divmod(i, 4)
        nb = (by in (0, 3)) + (bx in (0, 3))
        kind = {2: "corner", 1: "edge", 0: "interior"}[nb]
        nI, nG, nD, ni, nt = gold[kind]
        assert (s.I.size, s.Gamma.size, s.Delta.size) == (nI, nG, nD)
        assert (s.Omega.size, s.Omega_ext.size) == (ni, nt)


# ---------------------------------------------------------------------------
# Sec. 3.1, (3.1): X_i and the A^2 splitting  (PIN-1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("delta", [1, 2])
def test_a2_splitting_sum_bit_exact(delta):
    """sum_i R~_i^T X_i^T X_i R~_i = A diag(mult) A, mult_j = #{i : j in Omega_i};
    exact in FP64 for the integer-valued Poisson matrix."""
    m = 10
    A = W.poisson2d(m)
    part = W.grid2d_partition(m, 2, 2)
    sets = O.subdomain_sets(A, part, 4, delta)
    Ad = A.to_scipy().toarray()
    n = Ad.shape[0]
    S = np.zeros((n, n))
    mult = np.zeros(n)
    for s in sets:
        Aii, Xi = O.extract(A, s)
        S[np.ix_(s.Omega_ext, s.Omega_ext)] += Xi.T @ Xi
        mult[s.Omega] += 1
        # X_i^T X_i = R~_i A R_i^T R_i A R~_i^T  (3.1)
        Ri = np.eye(n)[s.Omega]
        Rt = np.eye(n)[s.Omega_ext]
        np.testing.assert_array_equal(Xi.T @ Xi, Rt @ Ad @ Ri.T @ Ri @ Ad @ Rt.T)
        np.testing.assert_array_equal(Aii, Ad[np.ix_(s.Omega, s.Omega)])
    np.testing.assert_array_equal(S, Ad @ np.diag(mult) @ Ad)


# ---------------------------------------------------------------------------
# square-root lemma, Schur lemma, shift remark  (PIN-2, PIN-3)
# ---------------------------------------------------------------------------
def _tiny_cases():
    yield W.laplace1d(20), W.contiguous_partition(20, 4), 4, 1
    yield W.poisson2d(8), W.grid2d_partition(8, 2, 2), 4, 1
    A = W.random_spd(50, 4, seed=7)
    yield A, O.ggg_partition(A, 4, 1), 4, 1
    A = W.diffusion3d(4, seed=2, sigma=1.0, channels=1, contrast=1e3)
    yield A, O.ggg_partition(A, 3, 0), 3, 2


def test_square_root_against_gram_eigendecomposition():
    """Fhat^T Fhat - sI is the PSD square root of X^T X (square-root lemma):
    compare with sqrt of the eigen-decomposition of the Gram matrix."""
    for A, part, N, d in _tiny_cases():
        for s in O.subdomain_sets(A, part, N, d):
            Aii, Xi = O.extract(A, s)
            spl = O.local_splitting(Xi, s.I.size, s.Gamma.size)
            M = spl.Fhat.T @ spl.Fhat - spl.s * np.eye(Xi.shape[1])
            w, V = np.linalg.eigh(Xi.T @ Xi)
            Msq = (V * np.sqrt(np.clip(w, 0, None))) @ V.T
            assert np.abs(M - Msq).max() <= 1e-7 * spl.sigma1
            np.testing.assert_allclose(M @ M, Xi.T @ Xi, atol=1e-12 * spl.sigma1 ** 2)
            # shift: s = sigma_1 * 2^-52, sigma_1 = ||X_i||_2
            assert spl.s == spl.sigma1 * 2.0 ** -52
            assert abs(spl.sigma1 - np.linalg.norm(Xi, 2)) <= 1e-12 * spl.sigma1


def test_lemma_splittings_bounded_by_A():
    """Square-root lemma: 0 <= R~^T A~_ext R~ <= A; Schur lemma: 0 <= R^T A~_ii R <= A,
    up to rounding of the size of the shift."""
    for A, part, N, d in _tiny_cases():
        Ad = O.as_scipy(A).toarray()
        n = Ad.shape[0]
        for s in O.subdomain_sets(A, part, N, d):
            Aii, Xi = O.extract(A, s)
            spl = O.local_splitting(Xi, s.I.size, s.Gamma.size)
            tol = 64 * Xi.shape[1] * spl.s + 1e-14 * spl.sigma1
            Mext = spl.Fhat.T @ spl.Fhat - spl.s * np.eye(Xi.shape[1])
            big = np.zeros((n, n))
            big[np.ix_(s.Omega_ext, s.Omega_ext)] = Mext
            assert np.linalg.eigvalsh(Ad - big).min() >= -tol
            big = np.zeros((n, n))
            big[np.ix_(s.Omega, s.Omega)] = spl.Atilde_ii
            assert np.linalg.eigvalsh(spl.Atilde_ii).min() >= -tol
            assert np.linalg.eigvalsh(Ad - big).min() >= -tol


def test_schur_complement_three_routes_agree():
    """With a test-only shift large enough to avoid cancellation, the QR route,
    the literal formula (3.2) and the inverse formula (3.4) coincide."""
    for A, part, N, d in _tiny_cases():
        for s in O.subdomain_sets(A, part, N, d):
            Aii, Xi = O.extract(A, s)
            sig1 = np.linalg.norm(Xi, 2)
            sh = 1e-3 * sig1
            spl = O.local_splitting(Xi, s.I.size, s.Gamma.size, shift=sh)
            ni, nt = Xi.shape
            # underline{A~}_ii = V (Sigma + s I) V^T + s (I - V V^T)  (economic SVD)
            U, sg, Vt = np.linalg.svd(Xi, full_matrices=False)
            V = Vt.T
            Mext = V @ np.diag(sg + sh) @ V.T + sh * (np.eye(nt) - V @ V.T)
            X11, X12 = Mext[:ni, :ni], Mext[:ni, ni:]
            X21, X22 = Mext[ni:, :ni], Mext[ni:, ni:]
            lit = X11 - X12 @ np.linalg.solve(X22, X21) if nt > ni else X11
            Minv = V @ np.diag(1.0 / (sg + sh)) @ V.T + (np.eye(nt) - V @ V.T) / sh   # (3.4)
            via34 = np.linalg.inv(Minv[:ni, :ni])
            scale = np.abs(lit).max()
            assert np.abs(spl.Atilde_ii - lit).max() <= 1e-10 * scale
            assert np.abs(via34 - lit).max() <= 1e-8 * scale
            # quotient property: S_I = Schur of A~_ii onto Omega_Ii
            nI = s.I.size
            T = spl.Atilde_ii
            SI = T[:nI, :nI] - T[:nI, nI:] @ np.linalg.solve(T[nI:, nI:], T[nI:, :nI]) if ni > nI else T
            assert np.abs(spl.S_I - SI).max() <= 1e-9 * scale


# ---------------------------------------------------------------------------
# (3.3) eigenproblem with Boolean D_i  (PIN-5, PIN-6, PIN-10)
# ---------------------------------------------------------------------------
def test_eigs_reciprocal_form_matches_full_pencil():
    """Nonzero lambda of D A_ii D u = lambda A~_ii u equal 1/mu of the reduced
    problem (brute force through the full pencil with a test shift)."""
    for A, part, N, d in _tiny_cases():
        for s in O.subdomain_sets(A, part, N, d):
            Aii, Xi = O.extract(A, s)
            spl = O.local_splitting(Xi, s.I.size, s.Gamma.size, shift=1e-3 * np.linalg.norm(Xi, 2))
            nI = s.I.size
            D = np.diag(np.r_[np.ones(nI), np.zeros(s.Gamma.size)])
            lam = sla.eigh(D @ Aii @ D, spl.Atilde_ii, eigvals_only=True)
            lam_nz = np.sort(lam[np.abs(lam) > 1e-9 * np.abs(lam).max()])
            mu, _, _ = O.local_eigen(Aii, spl.S_I, nI, 0.5)
            np.testing.assert_allclose(np.sort(1.0 / mu), lam_nz, rtol=1e-8)


def test_lambda_at_least_one_boolean_D():
    """Boolean D and the Schur lemma give A~_ii <= A_ii on Omega_Ii, so every
    nonzero lambda >= 1 (mu <= 1) up to rounding."""
    for A, part, N, d in _tiny_cases():
        for s in O.subdomain_sets(A, part, N, d):
            Aii, Xi = O.extract(A, s)
            spl = O.local_splitting(Xi, s.I.size, s.Gamma.size)
            mu, _, _ = O.local_eigen(Aii, spl.S_I, s.I.size, 0.5)
            assert mu.max() <= 1.0 + 1e-8
            assert mu.min() > 0


def test_near_kernel_span_c1():
    """Without the shift, ker(A~_ii) = {u : X_i [u; y] = 0} = range(A_ii^{-1} A(Omega_i, Delta_i));
    its D-image lies in the kept space for any practical threshold."""
    cfg = W.config_c1()
    A = O.as_scipy(cfg.A)
    sets = O.subdomain_sets(A, cfg.part, cfg.N, cfg.overlap)
    for i in (0, 1, 5):
        s = sets[i]
        Aii, Xi = O.extract(A, s)
        spl = O.local_splitting(Xi, s.I.size, s.Gamma.size)
        _, mu_keep, ZI = O.local_eigen(Aii, spl.S_I, s.I.size, cfg.tau)
        K = np.linalg.solve(Aii, Xi[:, Aii.shape[0]:])[: s.I.size]
        Uk, sk, _ = np.linalg.svd(K, full_matrices=False)
        Uk = Uk[:, sk > 1e-10 * sk[0]]
        ang = sla.subspace_angles(Uk, ZI)
        assert ang.max() < 1e-8
        # for the constant-coefficient Poisson subdomains the two spaces coincide
        assert Uk.shape[1] == ZI.shape[1]


# ---------------------------------------------------------------------------
# (2.1), E, kappa bound, special cases  (PIN-4, PIN-7, PIN-8, PIN-9, PIN-11, PIN-12)
# ---------------------------------------------------------------------------
def test_bound_multiplicity_and_E_spd_tiny():
    for A, part, N, d in _tiny_cases():
        for tau in (0.1, 0.5):
            pre = O.build(A, part, N, d, tau)
            if pre.nC:
                assert np.linalg.eigvalsh(pre.E).min() > 0
            dg = O.diagnostics(A, pre, tau)
            assert dg["k_m"] <= N + 1e-10
            assert dg["lambda_max"] <= dg["k_c"] + 1 + 1e-8
            assert dg["kappa"] <= dg["bound"]


def test_apply_against_dense_definition():
    """M^{-1} = R_0^T E^{-1} R_0 + sum R_i^T A_ii^{-1} R_i with dense matrices."""
    A = W.poisson2d(8)
    part = W.grid2d_partition(8, 2, 2)
    pre = O.build(A, part, 4, 1, 0.1)
    Ad = A.to_scipy().toarray()
    n = Ad.shape[0]
    Minv = np.zeros((n, n))
    for L in pre.locals:
        R = np.eye(n)[L.sets.Omega]
        Minv += R.T @ np.linalg.inv(R @ Ad @ R.T) @ R
    Z = pre.Z.toarray()
    if Z.shape[1]:
        Minv += Z @ np.linalg.inv(Z.T @ Ad @ Z) @ Z.T
    r = np.random.default_rng(0).standard_normal(n)
    np.testing.assert_allclose(pre.apply(r), Minv @ r, rtol=1e-12, atol=1e-12)


def test_single_subdomain_reduces_to_exact_solve():
    """N = 1: Omega = all, Gamma = Delta = empty; A~ = (A^2)^{1/2} + sI = A + sI,
    every mu = lambda(A)/(lambda(A)+s) ~ 1 so nothing is kept for tau < 1;
    M^{-1} = A^{-1} and PCG stops after one iteration."""
    A = W.random_spd(40, 3, seed=9)
    part = np.zeros(40, dtype=np.int32)
    s = O.subdomain_sets(A, part, 1, 1)[0]
    assert s.Gamma.size == 0 and s.Delta.size == 0
    Aii, Xi = O.extract(A, s)
    spl = O.local_splitting(Xi, 40, 0)
    Ad = O.as_scipy(A).toarray()
    np.testing.assert_allclose(spl.Atilde_ii, Ad + spl.s * np.eye(40), atol=1e-12 * spl.sigma1)
    pre = O.build(A, part, 1, 1, 0.5)
    assert pre.nC == 0
    b = W.rhs(40, 1)
    x, its, rr = O.pcg(A, b, pre.apply, rtol=1e-12)
    assert its == 1 and rr < 1e-12


def test_tau_to_zero_gives_one_level_asm():
    cfg = W.config_c1()
    A = W.poisson2d(16)
    part = W.grid2d_partition(16, 2, 2)
    pre = O.build(A, part, 4, 1, 1e-30)
    assert pre.nC == 0
    Ad = A.to_scipy().toarray()
    r = W.rhs(256, 3)
    z = np.zeros(256)
    for L in pre.locals:
        Om = L.sets.Omega
        z[Om] += np.linalg.solve(Ad[np.ix_(Om, Om)], r[Om])
    np.testing.assert_allclose(pre.apply(r), z, rtol=1e-12)


def test_pcg_solution_against_dense_solve():
    A = W.diffusion3d(6, seed=3)
    part = O.ggg_partition(A, 5, 0)
    pre = O.build(A, part, 5, 2, 0.02)
    b = W.rhs(A.n, 2)
    x, its, rr = O.pcg(A, b, pre.apply, rtol=1e-13)
    xd = np.linalg.solve(A.to_scipy().toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert rr <= 1e-13


def test_three_level_flexible_cg_converges():
    """Nested coarse solve (multilevel remark, Sec. 4 nested case): outer flexible
    CG with an inner PCG at 1e-4 reaches 1e-8."""
    A = W.poisson2d(24)
    part = W.grid2d_partition(24, 4, 4)
    pre = O.build(A, part, 16, 1, 0.1, levels=3, coarsen=4)
    assert hasattr(pre, "inner")
    b = W.rhs(A.n, 0)
    x, its, rr = O.flexible_pcg(A, b, pre.apply, rtol=1e-8)
    assert rr <= 1e-8
    pre2 = O.build(A, part, 16, 1, 0.1)
    _, its2, _ = O.pcg(A, b, pre2.apply, rtol=1e-8)
    assert its <= its2 + 3
