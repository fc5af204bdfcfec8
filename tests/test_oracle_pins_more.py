"""More pins of the CPU oracle (CPU only): the flexible CG of the nested case,
the block graph and partition of the next level, the nev cap, and the C1
condition-number constants.

Every expected value comes from mathematics or a brute-force restatement in
this file, never from the GPU path.  Each test names the passage it checks.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
import workloads as W
from test_oracle_pins import _ggg_bruteforce, _read_golden

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# flexible CG (multilevel remark of Sec. 3.2, nested case of Sec. 4)
# ---------------------------------------------------------------------------
def _record(store):
    def cb(k, x, r, p):
        store.append((k, x.copy(), r.copy(), p.copy()))
    return cb


def test_flexible_cg_equals_pcg_for_fixed_spd_preconditioner():
    """For a fixed SPD M, z_{k+1}^T r_k = 0, so the Polak-Ribiere beta equals
    the usual one and flexible CG produces the PCG iterates one by one."""
    A = W.diffusion3d(6, seed=3)
    part = O.ggg_partition(A, 5, 0)
    pre = O.build(A, part, 5, 2, 0.02)
    b = W.rhs(A.n, 2)
    h1, h2 = [], []
    _, its1, _ = O.pcg(A, b, pre.apply, rtol=1e-12, callback=_record(h1))
    _, its2, _ = O.flexible_pcg(A, b, pre.apply, rtol=1e-12, callback=_record(h2))
    assert its1 == its2 and len(h1) == len(h2) == its1
    xs = np.linalg.norm(h1[-1][1])
    for (k1, x1, r1, p1), (k2, x2, r2, p2) in zip(h1, h2):
        assert k1 == k2
        assert np.linalg.norm(x1 - x2) <= 1e-9 * xs, k1
        assert np.linalg.norm(p1 - p2) <= 1e-8 * np.linalg.norm(p1), k1


def _varying_preconditioner(A, pre):
    """M_k alternates between the two-level preconditioner and Jacobi, each
    scaled by a factor that changes with every call: SPD for every k, not
    the same operator twice in a row."""
    d = A.diagonal()
    state = {"k": 0}

    def Minv(r):
        k = state["k"]
        state["k"] += 1
        f = 1.0 + 0.5 * math.sin(1.7 * k)
        return f * (pre.apply(r) if k % 2 == 0 else r / d)
    return Minv


def _fr_flexible_cg(A, b, Minv, maxit):
    """Negative control: the same loop with the Fletcher-Reeves beta
    r_{k+1}^T z_{k+1} / r_k^T z_k, which loses local A-orthogonality when M varies."""
    x = np.zeros_like(b)
    r = b.copy()
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    ps = []
    for _ in range(maxit):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        ps.append(p.copy())
        z = Minv(r)
        rzn = r @ z
        p = z + (rzn / rz) * p
        rz = rzn
    return ps


def test_flexible_cg_local_conjugacy_with_varying_preconditioner():
    """Flexible CG with beta_k = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k): since
    r_{k+1} - r_k = -alpha_k A p_k, every new direction is A-orthogonal to the
    previous one, p_{k+1}^T A p_k = 0, and the residual is orthogonal to the
    last direction, r_{k+1}^T p_k = 0, whatever M_k is.  A Fletcher-Reeves beta,
    a wrong sign or a swapped update order breaks the first identity."""
    A = O.as_scipy(W.diffusion3d(6, seed=3))
    part = O.ggg_partition(A, 5, 0)
    pre = O.build(A, part, 5, 2, 0.02)
    b = W.rhs(A.shape[0], 2)
    hist = []
    x, its, rr = O.flexible_pcg(A, b, _varying_preconditioner(A, pre), rtol=1e-10, callback=_record(hist))
    assert rr <= 1e-10 and its >= 6
    for (_, _, r1, p0), (_, _, _, p1) in zip(hist[:-1], hist[1:]):
        Ap0 = A @ p0
        conj = abs(p1 @ Ap0) / math.sqrt((p1 @ (A @ p1)) * (p0 @ Ap0))
        assert conj <= 1e-10, conj
        assert abs(r1 @ p0) <= 1e-10 * np.linalg.norm(r1) * np.linalg.norm(p0)
    # the identity discriminates: Fletcher-Reeves violates it on the same M_k
    ps = _fr_flexible_cg(A, b, _varying_preconditioner(A, pre), 6)
    worst = max(abs(p1 @ (A @ p0)) / math.sqrt((p1 @ (A @ p1)) * (p0 @ (A @ p0))) for p0, p1 in zip(ps[:-1], ps[1:]))
    assert worst > 1e-3, worst


# ---------------------------------------------------------------------------
# next level: block graph and partition (multilevel remark of Sec. 3.2)
# ---------------------------------------------------------------------------
def _block_graph_bruteforce(A, sets):
    """i ~ j iff A(Omega_Ii, Omega_Ij) != 0, entry by entry."""
    Ad = O.as_scipy(A).toarray()
    N = len(sets)
    G = np.zeros((N, N), dtype=bool)
    for i in range(N):
        for j in range(N):
            G[i, j] = bool(np.any(Ad[np.ix_(sets[i].I, sets[j].I)] != 0))
    return G


def _overlap_graph_bruteforce(A, sets):
    Ad = O.as_scipy(A).toarray()
    N = len(sets)
    return np.array([[bool(np.any(Ad[np.ix_(sets[i].Omega, sets[j].Omega)] != 0)) for j in range(N)]
                     for i in range(N)])


def test_next_level_graph_and_partition_bruteforce():
    """The nodes of the next level are the fine subdomains and E's block (i, j)
    is Z_i^T A(Omega_Ii, Omega_Ij) Z_j, so E's nonzero blocks are exactly the
    pairs with A(Omega_Ii, Omega_Ij) != 0.  The graph the oracle partitions
    must be that one (not the overlapping Omega_i adjacency, which here has
    the corner neighbours in addition), and its partition must be the
    brute-force growing rule into ceil(N / coarsen) parts, each fine
    subdomain's coarse dofs kept together."""
    m, N, coarsen = 24, 16, 4
    A = W.poisson2d(m)
    part = W.grid2d_partition(m, 4, 4)
    pre = O.build(A, part, N, 1, 0.1, levels=3, coarsen=coarsen)
    sets = [L.sets for L in pre.locals]
    G = _block_graph_bruteforce(A, sets)
    Go = pre.block_graph.toarray() != 0
    np.testing.assert_array_equal(Go, G)
    # E's actual block pattern
    off = pre.coarse_offsets
    Eb = np.array([[np.abs(pre.E[off[i]:off[i + 1], off[j]:off[j + 1]]).max() > 1e-12 * np.abs(pre.E).max()
                    for j in range(N)] for i in range(N)])
    np.testing.assert_array_equal(Eb, G)
    assert (_overlap_graph_bruteforce(A, sets) & ~G).any()  # the plausible misreading differs here
    # partition of the block graph
    N2 = math.ceil(N / coarsen)
    Gcsr = sp.csr_matrix(G.astype(float))
    np.testing.assert_array_equal(pre.block_part, _ggg_bruteforce(Gcsr, N2, 0))
    for i in range(N):
        blk = pre.coarse_part[off[i]:off[i + 1]]
        assert np.all(blk == blk[0]) if blk.size else True
    assert len(pre.inner.locals) == np.unique(pre.coarse_part).size <= N2


def test_next_level_partition_count_default_coarsening():
    """N_2 = ceil(N / 64) with the default coarsening (Sec. 4: 256 -> 4)."""
    m = 32
    A = W.poisson2d(m)
    part = W.grid2d_partition(m, 8, 8)
    pre = O.build(A, part, 64, 1, 0.1, levels=3)
    assert int(pre.block_part.max()) + 1 == 1
    assert len(pre.inner.locals) == 1


# ---------------------------------------------------------------------------
# nev cap (3.3) against the full pencil by brute force
# ---------------------------------------------------------------------------
def test_nev_cap_is_the_nev_largest_lambda_above_threshold():
    """The cap keeps, among the eigenpairs of D_i A_ii D_i u = lambda A~_ii u with
    lambda > 1/tau, the nev with the largest lambda.  Brute force: A~_ii as the
    explicit Schur complement of (X^T X)^{1/2} + s I onto Omega_i (a test shift
    s = 1e-3 sigma_1 keeps it well conditioned), then the generalized symmetric
    eigenproblem of the full pencil on Omega_i."""
    m = 12
    A = W.poisson2d(m)
    part = W.grid2d_partition(m, 2, 2)
    sets = O.subdomain_sets(A, part, 4, 1)
    s = sets[3]
    Aii, Xi = O.extract(A, s)
    nI, ni = s.I.size, s.Omega.size
    _, sig, Vt = np.linalg.svd(Xi, full_matrices=False)  # (X^T X)^{1/2} = V Sigma V^T
    shift = 1e-3 * sig[0]
    M = (Vt.T * sig) @ Vt + shift * np.eye(Xi.shape[1])
    At = M[:ni, :ni] - M[:ni, ni:] @ np.linalg.solve(M[ni:, ni:], M[ni:, :ni])
    DAD = np.zeros((ni, ni))
    DAD[:nI, :nI] = Aii[:nI, :nI]
    lam, U = sla.eigh(DAD, 0.5 * (At + At.T))
    tau = 0.5
    above = np.flatnonzero(lam > 1.0 / tau)
    assert above.size >= 6
    nev = 4
    sel = above[np.argsort(lam[above])[::-1][:nev]]
    spl = O.local_splitting(Xi, nI, s.Gamma.size, shift=shift)
    _, mu_keep, ZI = O.local_eigen(Aii, spl.S_I, nI, tau, nev)
    np.testing.assert_allclose(mu_keep, np.sort(1.0 / lam[sel]), rtol=1e-9)
    gap = np.sort(lam[above])[::-1]
    assert gap[nev - 1] > 1.01 * gap[nev]  # the kept block is separated
    ang = sla.subspace_angles(ZI, U[:nI, sel])
    assert ang.max() <= 1e-7, ang.max()
    # without the cap every lambda > 1/tau is kept
    _, mu_all, _ = O.local_eigen(Aii, spl.S_I, nI, tau)
    np.testing.assert_allclose(mu_all, np.sort(1.0 / lam[above]), rtol=1e-9)


# ---------------------------------------------------------------------------
# C1: condition number, constants and iteration counts (Sec. 3.2 bound)
# ---------------------------------------------------------------------------
def test_c1_condition_number_constants_and_iterations():
    """64^2 Poisson in 4x4 parts, overlap 1, lambda > 10: values computed
    independently from the paper's definitions (tests/golden/c1_constants.txt,
    a throwaway dense probe, not the paper's numbers): n_C, kappa(M^{-1}A),
    k_m, k_c, PCG iterations to 1e-8; and the one-level method (no coarse
    space) for contrast."""
    g = {r[0]: float(r[1]) for r in _read_golden("c1_constants.txt")}
    cfg = W.config_c1()
    b = W.rhs(cfg.A.n, 0)
    pre = O.build(cfg.A, cfg.part, 16, 1, 0.1)
    d = O.diagnostics(cfg.A, pre, 0.1)
    _, its, rr = O.pcg(cfg.A, b, pre.apply, rtol=1e-8)
    assert pre.nC == int(g["n_C"])
    assert abs(d["kappa"] - g["kappa"]) <= 1e-3
    assert abs(d["k_m"] - g["k_m"]) <= 1e-3
    assert d["k_c"] == int(g["k_c"])
    assert its == int(g["pcg_its"]) and rr <= 1e-8
    assert d["kappa"] <= d["bound"]
    one = O.build(cfg.A, cfg.part, 16, 1, 1e-30)
    d1 = O.diagnostics(cfg.A, one, 1e-30)
    _, its1, _ = O.pcg(cfg.A, b, one.apply, rtol=1e-8)
    assert one.nC == 0
    assert abs(d1["kappa"] - g["kappa_one_level"]) <= 0.1
    assert its1 == int(g["pcg_its_one_level"])
