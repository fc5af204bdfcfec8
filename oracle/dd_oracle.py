"""FP64 CPU oracle — test infrastructure only (see package docstring).

Each function follows one step of the method in the order the paper gives it,
in the paper's notation.  Citations name the paper's sections, equations,
lemmas and remarks:

* Sec. 2 (Domain decomposition): nonoverlapping sets Omega_Ii, overlap
  Gamma_i, extended layer Delta_i, restrictions R_i, one-level ASM, the
  two-level additive preconditioner (2.1), the algebraic partition of unity.
* Sec. 2.2: local SPSD splittings and the multiplicity constant k_m (2.2).
* Sec. 3.1: X_i = R_i A R~_i^T (3.1); the square root lemma for A^2
  splittings; the Schur complement lemma (3.2); the shift remark.
* Sec. 3.2: the coarse space (3.3) with threshold lambda > 1/tau, the
  condition-number bound, the SVD route and the inverse formula (3.4); the
  multilevel extension.
* Sec. 4: exact local and coarse Cholesky, tolerance 1e-8, nested levels.

Readings where the paper is silent or ambiguous (each one is listed in the
design notes):
* R1  Boolean partition of unity: D_i = 1 on Omega_Ii, 0 on Gamma_i.
* R2  Overlap delta >= 1: Gamma_i = BFS layers 1..delta of Omega_Ii in G(A),
      Delta_i = layer delta+1; each set in ascending global index.
* R3  eps = 2^-52 in the shift s_i = sigma_1i * eps (shift remark, Sec. 3.1).
* R4  The Schur complement (3.2) is evaluated through the triangular factor of
      a QR factorisation of a factor of the shifted square root, never through
      the explicit inverse of its (2,2) block or through (3.4), which cancel
      catastrophically at a shift of relative size eps.
* R5  The eigenproblem (3.3) with Boolean D_i is solved in its reciprocal
      form S_I w = mu A_I w (mu = 1/lambda), S_I the Schur complement of the
      splitting onto Omega_Ii; keep mu < tau (strict), optionally only the
      nev smallest.
* R6  PCG with the additive preconditioner (2.1) (the bound in Sec. 3.2 is
      proved for it), x0 = 0, stop on ||r_k||_2 <= rtol ||b||_2.
* R7  Seeded greedy graph growing partition (SplitMix64 seeds, level-
      synchronous BFS with minimum-id conflict resolution).
* R8  Levels >= 3: coarse graph blocks = fine subdomains, N_2 = ceil(N/64),
      inner PCG on E to 1e-4, outer flexible CG.
* R12 The deflated variant of Sec. 4, M_deflated = R_0^T E^{-1} R_0 +
      M_RAS (I - A R_0^T E^{-1} R_0), with the one-level restricted additive
      Schwarz M_RAS = sum_i R_i^T D_i A_ii^{-1} R_i and the Boolean D_i of R1,
      under right-preconditioned GMRES(30) from x0 = 0, Arnoldi by modified
      Gram-Schmidt, stopping when the Arnoldi estimate of the unpreconditioned
      residual reaches rtol ||b||_2 (the true residual is recomputed at every
      restart).  With levels >= 3 the coarse systems are solved by right-
      preconditioned GMRES(30) to 1e-4 with the next level's M_deflated, and
      the outer solver is flexible GMRES(30).

Parity for the finite-precision near-kernel cluster (lambda >~ 1e6) is only
meaningful as a subspace; its individual values are parity unpinned.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

EPS = 2.0 ** -52

__all__ = [
    "EPS", "splitmix64", "ggg_partition", "Sets", "subdomain_sets", "extract",
    "Splitting", "local_splitting", "schur_via_qr", "local_eigen", "LocalResult",
    "TwoLevel", "build", "pcg", "flexible_pcg", "gmres", "coloring_kc", "diagnostics",
    "coarse_partition", "as_scipy", "build_locals",
]


def as_scipy(A):
    """Accept a workloads.CSR or a scipy sparse matrix; return scipy CSR."""
    if sp.issparse(A):
        return sp.csr_matrix(A)
    return sp.csr_matrix((A.val, A.colind, A.rowptr), shape=(A.n, A.n))


# ---------------------------------------------------------------------------
# R7: seeded greedy graph growing (the partition is an input of the method,
# Sec. 2: "a graph partitioning algorithm can be used")
# ---------------------------------------------------------------------------
_M64 = (1 << 64) - 1


def splitmix64(seed: int, count: int) -> list[int]:
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): state += golden gamma,
    then two xor-shift-multiply mixing rounds and a final xor-shift."""
    out = []
    state = seed & _M64
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & _M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out.append(z ^ (z >> 31))
    return out


def ggg_partition(A, N: int, seed: int) -> np.ndarray:
    """Seeded greedy graph growing into N parts.

    1. Seeds: draw SplitMix64 values x_1, x_2, ... from ``seed``; vertex
       v = x mod n; skip vertices already chosen; the k-th distinct vertex
       becomes part k (k = 0..N-1).
    2. Level-synchronous BFS: in each round every unassigned vertex with at
       least one neighbour assigned in the previous round takes the minimum
       part id among those neighbours.
    3. Vertices never reached (other components) all go to the part with the
       fewest vertices (ties: lowest id).
    """
    A = as_scipy(A)
    n = A.shape[0]
    if not (1 <= N <= n):
        raise ValueError("need 1 <= N <= n")
    part = np.full(n, -1, dtype=np.int64)
    chosen = 0
    k = 0
    while chosen < N:
        # k-th SplitMix64 output of the stream started at ``seed``
        v = splitmix64((seed + k * 0x9E3779B97F4A7C15) & _M64, 1)[0] % n
        k += 1
        if part[v] < 0:
            part[v] = chosen
            chosen += 1
    rowptr, colind = A.indptr, A.indices
    frontier = np.flatnonzero(part >= 0)
    r = 0
    while frontier.size:
        r += 1
        # every unassigned neighbour of the frontier takes the min part id
        # among its frontier neighbours
        starts, ends = rowptr[frontier], rowptr[frontier + 1]
        lens = ends - starts
        src = np.repeat(frontier, lens)
        idx = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)]) if frontier.size else np.array([], int)
        dst = colind[idx]
        m = (part[dst] < 0) & (dst != src)
        dst, src = dst[m], src[m]
        if dst.size == 0:
            break
        best = np.full(n, np.iinfo(np.int64).max)
        np.minimum.at(best, dst, part[src])
        newv = np.flatnonzero(best != np.iinfo(np.int64).max)
        part[newv] = best[newv]
        frontier = newv
    rest = part < 0
    if rest.any():
        sizes = np.bincount(part[~rest], minlength=N)
        part[rest] = int(np.argmin(sizes))  # argmin returns the lowest id on ties
    return part.astype(np.int32)


# ---------------------------------------------------------------------------
# Sec. 2: subdomains Omega_Ii, Gamma_i, Delta_i
# ---------------------------------------------------------------------------
@dataclass
class Sets:
    I: np.ndarray      # Omega_Ii, ascending global indices
    Gamma: np.ndarray  # Gamma_i  (layers 1..delta), ascending
    Delta: np.ndarray  # Delta_i  (layer delta+1), ascending

    @property
    def Omega(self):   # Omega_i = [Omega_Ii, Gamma_i]
        return np.concatenate([self.I, self.Gamma])

    @property
    def Omega_ext(self):  # extended Omega~_i = [Omega_Ii, Gamma_i, Delta_i]
        return np.concatenate([self.I, self.Gamma, self.Delta])


def _neighbours(A: sp.csr_matrix, S: np.ndarray) -> np.ndarray:
    """N(S) = {c : a_rc stored, r in S, c != r} (the graph G(A) as stored)."""
    if S.size == 0:
        return S
    rows = A[S]
    cols = np.unique(rows.indices)
    return cols


def subdomain_sets(A, part: np.ndarray, N: int, delta: int) -> list[Sets]:
    """Omega_Ii = {j : part_j = i}; layer_0 = Omega_Ii; layer_k = N(union of
    earlier layers) minus those layers; Gamma_i = layers 1..delta,
    Delta_i = layer delta+1 (Sec. 2, generalised to delta >= 1)."""
    A = as_scipy(A)
    n = A.shape[0]
    part = np.asarray(part)
    if part.shape != (n,) or part.min() < 0 or part.max() >= N:
        raise ValueError("partition ids must lie in [0, N)")
    out = []
    order = np.argsort(part, kind="stable")
    counts = np.bincount(part, minlength=N)
    if (counts == 0).any():
        raise ValueError("empty subdomain")
    starts = np.concatenate([[0], np.cumsum(counts)])
    for i in range(N):
        I = np.sort(order[starts[i]:starts[i + 1]])
        visited = np.zeros(n, dtype=bool)
        visited[I] = True
        layers = []
        cur = I
        for _k in range(delta + 1):
            nb = _neighbours(A, cur)
            new = nb[~visited[nb]]
            new = np.unique(new)
            visited[new] = True
            layers.append(new)
            cur = np.flatnonzero(visited)
        Gamma = np.sort(np.concatenate(layers[:delta])) if delta else np.array([], dtype=np.int64)
        Delta = np.sort(layers[delta])
        out.append(Sets(I.astype(np.int64), Gamma.astype(np.int64), Delta.astype(np.int64)))
    return out


def extract(A, s: Sets):
    """A_ii = A(Omega_i, Omega_i) and X_i = A(Omega_i, Omega~_i) (3.1), dense."""
    A = as_scipy(A)
    Om, Omx = s.Omega, s.Omega_ext
    rows = A[Om]
    Aii = rows[:, Om].toarray()
    Xi = rows[:, Omx].toarray()
    return Aii, Xi


# ---------------------------------------------------------------------------
# Sec. 3.1-3.2: local SPSD splitting
# ---------------------------------------------------------------------------
def schur_via_qr(F: np.ndarray, keep: np.ndarray) -> np.ndarray:
    """Schur complement of M = F^T F onto the columns ``keep``.

    With the eliminated columns c placed first, QR of F[:, [c, keep]] gives
    M[keep,keep] - M[keep,c] M[c,c]^{-1} M[c,keep] = R22^T R22 (the residual of
    F[:, keep] after projection on range(F[:, c])).  This is reading R4.
    """
    ncol = F.shape[1]
    keep = np.asarray(keep)
    mask = np.ones(ncol, dtype=bool)
    mask[keep] = False
    elim = np.flatnonzero(mask)
    nk = keep.size
    if elim.size == 0:
        return F[:, keep].T @ F[:, keep]
    G = F[:, np.concatenate([elim, keep])]
    if G.shape[0] < G.shape[1]:
        G = np.vstack([G, np.zeros((G.shape[1] - G.shape[0], G.shape[1]))])
    R = np.linalg.qr(G, mode="r")
    R22 = R[elim.size:elim.size + nk, elim.size:]
    return R22.T @ R22


@dataclass
class Splitting:
    sigma: np.ndarray       # singular values of X_i (descending)
    sigma1: float           # largest singular value
    s: float                # shift sigma_1 * eps (shift remark)
    Fhat: np.ndarray        # factor with Fhat^T Fhat = underline{A~}_ii (shifted square root)
    Atilde_ii: np.ndarray   # Schur complement onto Omega_i, (3.2)
    S_I: np.ndarray         # Schur complement onto Omega_Ii (reciprocal eigenproblem)


def local_splitting(Xi: np.ndarray, nI: int, nG: int, shift: float | None = None) -> Splitting:
    """Sec. 3.2 practical construction.

    Economic SVD X_i = U Sigma V^T with complement V_perp; the shifted square
    root of X_i^T X_i is V (Sigma + s I) V^T + s V_perp V_perp^T with
    s = sigma_1 eps (shift remark).  Represented by its factor
    Fhat = diag(sqrt(sigma_j + s), sqrt(s)) [V, V_perp]^T.  Then (3.2) gives
    A~_ii as the Schur complement onto Omega_i (the first nI+nG columns),
    and S_I the Schur complement onto Omega_Ii (first nI columns) — the
    latter equals the Schur complement of A~_ii onto Omega_Ii (quotient
    property).  ``shift`` overrides s for tests only.
    """
    ni, nt = Xi.shape
    assert ni == nI + nG and nt >= ni
    U, sig, Vt = np.linalg.svd(Xi, full_matrices=True)
    sigma1 = float(sig[0]) if sig.size else 0.0
    s = sigma1 * EPS if shift is None else shift
    d = np.concatenate([sig + s, np.full(nt - ni, s)])
    Fhat = np.sqrt(d)[:, None] * Vt
    Atil = schur_via_qr(Fhat, np.arange(ni))
    S_I = schur_via_qr(Fhat, np.arange(nI))
    return Splitting(sig, sigma1, s, Fhat, 0.5 * (Atil + Atil.T), 0.5 * (S_I + S_I.T))


# ---------------------------------------------------------------------------
# Sec. 3.2: the local generalized eigenproblem (3.3), Boolean D_i
# ---------------------------------------------------------------------------
@dataclass
class LocalResult:
    sets: Sets
    Aii: np.ndarray
    split: Splitting | None
    mu_all: np.ndarray      # all mu = 1/lambda, ascending
    mu_keep: np.ndarray     # kept (mu < tau, optionally the nev smallest)
    Z_I: np.ndarray         # orthonormal basis of D_i Z_i restricted to Omega_Ii  (nI x p_i)


def local_eigen(Aii: np.ndarray, S_I: np.ndarray, nI: int, tau: float, nev: int | None = None):
    """(3.3) with Boolean D_i: D_i A_ii D_i = blkdiag(A_I, 0), so the nonzero
    eigenvalues are those of A_I w = lambda S_I w (eliminate the Gamma rows).
    Solve S_I w = mu A_I w, keep mu < tau (lambda > 1/tau), optionally only
    the nev smallest mu; D_i u = [w; 0]; orthonormalise the kept w."""
    A_I = Aii[:nI, :nI]
    mu, W = sla.eigh(S_I, A_I)
    keep = np.flatnonzero(mu < tau)
    if nev is not None:
        keep = keep[:nev]
    if keep.size:
        Q, _ = np.linalg.qr(W[:, keep])
    else:
        Q = np.zeros((nI, 0))
    return mu, mu[keep], Q


# ---------------------------------------------------------------------------
# Sec. 2.1: the two-level additive Schwarz preconditioner (2.1)
# ---------------------------------------------------------------------------
class TwoLevel:
    """M^{-1} = R_0^T E^{-1} R_0 + sum_i R_i^T A_ii^{-1} R_i  (2.1),
    R_0^T = [R_1^T D_1 Z_1, ..., R_N^T D_N Z_N], E = R_0 A R_0^T.
    variant "deflated": M_deflated of Sec. 4 (R12) from the same parts."""

    def __init__(self, A, locals_: list[LocalResult], coarse_solver=None, variant="additive"):
        if variant not in ("additive", "deflated"):
            raise ValueError("variant is 'additive' or 'deflated'")
        self.variant = variant
        self.A = as_scipy(A)
        self.n = self.A.shape[0]
        self.locals = locals_
        self.chol = [sla.cho_factor(L.Aii, lower=True) for L in locals_]
        self.omega = [L.sets.Omega for L in locals_]
        cols, rows, vals = [], [], []
        off = 0
        self.coarse_offsets = [0]
        for L in locals_:
            p = L.Z_I.shape[1]
            if p:
                rr, cc = np.meshgrid(L.sets.I, np.arange(off, off + p), indexing="ij")
                rows.append(rr.ravel())
                cols.append(cc.ravel())
                vals.append(L.Z_I.ravel())
            off += p
            self.coarse_offsets.append(off)
        self.nC = off
        if off:
            self.Z = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                   shape=(self.n, off))
            self.E = (self.Z.T @ (self.A @ self.Z)).toarray()
            self.E = 0.5 * (self.E + self.E.T)
            if coarse_solver is None:
                self.E_chol = sla.cho_factor(self.E, lower=True)  # raises if E is not SPD
            self.coarse_solver = coarse_solver
        else:
            self.Z = None
            self.E = np.zeros((0, 0))
            self.coarse_solver = None

    def apply_local(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros_like(r)
        for Om, c in zip(self.omega, self.chol):
            z[Om] += sla.cho_solve(c, r[Om])
        return z

    def apply_coarse(self, r: np.ndarray) -> np.ndarray:
        if self.nC == 0:
            return np.zeros_like(r)
        y = self.Z.T @ r
        if self.coarse_solver is not None:
            y = self.coarse_solver(y)
        else:
            y = sla.cho_solve(self.E_chol, y)
        return self.Z @ y

    def apply_ras(self, r: np.ndarray) -> np.ndarray:
        """M_RAS r = sum_i R_i^T D_i A_ii^{-1} R_i r (Sec. 4), Boolean D_i (R1):
        of each local solution on Omega_i = [Omega_Ii, Gamma_i] only the
        Omega_Ii part is kept, so every dof takes the value of its own part."""
        z = np.zeros_like(r)
        for L, Om, c in zip(self.locals, self.omega, self.chol):
            zi = sla.cho_solve(c, r[Om])
            z[L.sets.I] = zi[:L.sets.I.size]
        return z

    def apply_deflated(self, r: np.ndarray) -> np.ndarray:
        """M_deflated r = y + M_RAS (r - A y), y = R_0^T E^{-1} R_0 r (Sec. 4)."""
        y = self.apply_coarse(r)
        return y + self.apply_ras(r - self.A @ y)

    def apply(self, r: np.ndarray) -> np.ndarray:
        if self.variant == "deflated":
            return self.apply_deflated(r)
        return self.apply_coarse(r) + self.apply_local(r)

    @property
    def grid_complexity(self) -> float:  # (n + n_C) / n, Sec. 4
        return (self.n + self.nC) / self.n


def build_locals(A, part, N, delta, tau, nev=None, shift=None, keep_split=True):
    A = as_scipy(A)
    sets = subdomain_sets(A, part, N, delta)
    out = []
    for s in sets:
        Aii, Xi = extract(A, s)
        spl = local_splitting(Xi, s.I.size, s.Gamma.size, shift=shift)
        mu, mu_keep, Z_I = local_eigen(Aii, spl.S_I, s.I.size, tau, nev)
        out.append(LocalResult(s, Aii, spl if keep_split else None, mu, mu_keep, Z_I))
    return out


def coarse_partition(offsets: list[int], part_fine_graph: np.ndarray) -> np.ndarray:
    """Expand a partition of the subdomain graph to the coarse dofs (R8)."""
    nC = offsets[-1]
    out = np.empty(nC, dtype=np.int32)
    for i in range(len(offsets) - 1):
        out[offsets[i]:offsets[i + 1]] = part_fine_graph[i]
    return out


def _subdomain_graph(A, locals_: list[LocalResult]) -> sp.csr_matrix:
    """Block graph of E: i ~ j iff A(Omega_Ii, Omega_Ij) != 0 (coarse blocks)."""
    A = as_scipy(A)
    n = A.shape[0]
    owner = np.empty(n, dtype=np.int64)
    for i, L in enumerate(locals_):
        owner[L.sets.I] = i
    coo = A.tocoo()
    G = sp.csr_matrix((np.ones(coo.nnz), (owner[coo.row], owner[coo.col])), shape=(len(locals_),) * 2)
    G.data[:] = 1.0
    return G


def build(A, part, N, delta, tau, levels=2, nev=None, inner_rtol=1e-4, shift=None, coarsen=64,
          variant="additive"):
    """Full setup (Sec. 3.2), recursively for levels >= 3 (multilevel remark,
    R8); variant "deflated" for M_deflated and GMRES coarse solves (R12)."""
    if levels < 2:
        raise ValueError("levels >= 2")
    locs = build_locals(A, part, N, delta, tau, nev, shift)
    if levels == 2:
        return TwoLevel(A, locs, variant=variant)
    pre = TwoLevel(A, locs, coarse_solver=lambda y: y, variant=variant)  # E assembled, solver set below
    E = pre.E
    if pre.nC == 0:
        pre.coarse_solver = None
        return pre
    # coarse block graph -> partition with N_2 = ceil(N / coarsen) parts
    nb = [L.Z_I.shape[1] for L in locs]
    G = _subdomain_graph(A, locs)
    active = np.array([p > 0 for p in nb])
    N2 = max(1, math.ceil(N / coarsen))
    Gs = sp.csr_matrix(G)
    part_blocks = ggg_partition(Gs, min(N2, G.shape[0]), 0)
    part2 = coarse_partition(pre.coarse_offsets, part_blocks)
    # remove empty parts (blocks with no coarse dofs may leave a part empty)
    used = np.unique(part2)
    remap = -np.ones(int(part_blocks.max()) + 1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    part2 = remap[part2].astype(np.int32)
    inner = build(sp.csr_matrix(E), part2, int(used.size), delta, tau, levels - 1, nev, inner_rtol, shift, coarsen,
                  variant)
    Esp = sp.csr_matrix(E)

    def coarse_solve(y):
        if variant == "deflated":
            x, its, rr = gmres(Esp, y, inner.apply, rtol=inner_rtol, restart=30, maxit=1000,
                               flexible=levels - 1 >= 3)
        else:
            x, its, rr = pcg(Esp, y, inner.apply, rtol=inner_rtol, maxit=1000)
        return x

    pre.coarse_solver = coarse_solve
    pre.inner = inner
    pre.block_graph = G            # for inspection: the graph the next level is partitioned on
    pre.block_part = part_blocks   # its partition into ceil(N / coarsen) parts
    pre.coarse_part = part2        # expanded to the coarse dofs, empty parts removed
    return pre


# ---------------------------------------------------------------------------
# Krylov solvers (R6, R8)
# ---------------------------------------------------------------------------
def pcg(A, b, Minv, rtol=1e-8, maxit=1000, x0=None, callback=None):
    """Preconditioned CG; stop when ||r_k||_2 <= rtol ||b||_2 (recurrence
    residual); return (x, iterations, true relative residual).  callback(k,
    x, r, p), if given, sees iteration k's iterate, residual and direction
    after the update (observation only)."""
    A = as_scipy(A)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0
    r = b - A @ x
    its = 0
    if np.linalg.norm(r) > rtol * bn:
        z = Minv(r)
        p = z.copy()
        rz = r @ z
        for its in range(1, maxit + 1):
            q = A @ p
            alpha = rz / (p @ q)
            x += alpha * p
            r -= alpha * q
            if callback is not None:
                callback(its, x, r, p)
            if np.linalg.norm(r) <= rtol * bn:
                break
            z = Minv(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
    return x, its, float(np.linalg.norm(b - A @ x) / bn)


def flexible_pcg(A, b, Minv, rtol=1e-8, maxit=1000, callback=None):
    """Flexible CG (Polak-Ribiere beta) for a variable preconditioner (R8):
    beta_k = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k).  callback as in pcg."""
    A = as_scipy(A)
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0.0
    r = b.copy()
    its = 0
    if np.linalg.norm(r) > rtol * bn:
        z = Minv(r)
        p = z.copy()
        rz = r @ z
        for its in range(1, maxit + 1):
            q = A @ p
            alpha = rz / (p @ q)
            x += alpha * p
            r_old = r.copy()
            r -= alpha * q
            if callback is not None:
                callback(its, x, r, p)
            if np.linalg.norm(r) <= rtol * bn:
                break
            z = Minv(r)
            beta = (z @ (r - r_old)) / rz
            rz = r @ z
            p = z + beta * p
    return x, its, float(np.linalg.norm(b - A @ x) / bn)


def gmres(A, b, Minv, rtol=1e-8, restart=30, maxit=1000, flexible=False):
    """Right-preconditioned GMRES(restart) (Saad & Schultz 1986) and its
    flexible form (Saad 1993), R12: x0 = 0; Arnoldi on A M by modified
    Gram-Schmidt; Givens rotations reduce the Hessenberg matrix; a cycle ends
    when the estimate |g_{j+1}| of ||b - A x_j||_2 reaches rtol ||b||_2, after
    `restart` steps, on breakdown (h_{j+1,j} = 0) or at maxit steps in total.
    At the end of a cycle x += M V_k y (flexible: x += [M_1 v_1 ... M_k v_k] y)
    and the true residual starts the next one.  Returns (x, Arnoldi steps,
    true relative residual)."""
    A = as_scipy(A)
    n = b.size
    x = np.zeros_like(b)
    bn = float(np.linalg.norm(b))
    if bn == 0.0:
        return x, 0, 0.0
    its = 0
    r = b.copy()
    beta = bn
    while beta > rtol * bn and its < maxit:
        m = restart
        V = np.zeros((n, m + 1))
        Zs = []
        Hm = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            zj = Minv(V[:, j])
            if flexible:
                Zs.append(zj)
            w = A @ zj
            for i in range(j + 1):
                Hm[i, j] = w @ V[:, i]
                w = w - Hm[i, j] * V[:, i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] > 0.0:
                V[:, j + 1] = w / Hm[j + 1, j]
            for i in range(j):  # earlier rotations on the new column
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            d = math.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j] = Hm[j, j] / d
            sn[j] = Hm[j + 1, j] / d
            Hm[j, j] = d
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            if abs(g[j + 1]) <= rtol * bn or its >= maxit or sn[j] == 0.0:
                break
        y = sla.solve_triangular(Hm[:k, :k], g[:k])
        if flexible:
            x = x + np.column_stack(Zs) @ y
        else:
            x = x + Minv(V[:, :k] @ y)
        r = b - A @ x
        beta = float(np.linalg.norm(r))
    return x, its, beta / bn


# ---------------------------------------------------------------------------
# Sec. 3.2: constants of the condition-number bound (diagnostics, tiny inputs)
# ---------------------------------------------------------------------------
def coloring_kc(A, locals_: list[LocalResult]) -> int:
    """Greedy colouring in index order of the subdomain graph i ~ j iff
    A(Omega_i, Omega_j) != 0; returns the number of colours k_c."""
    A = as_scipy(A)
    N = len(locals_)
    n = A.shape[0]
    memb = sp.lil_matrix((N, n))
    for i, L in enumerate(locals_):
        memb[i, L.sets.Omega] = 1.0
    memb = sp.csr_matrix(memb)
    Apat = A.copy()
    Apat.data[:] = 1.0
    G = (memb @ Apat @ memb.T).toarray() != 0
    colors = -np.ones(N, dtype=int)
    for i in range(N):
        used = {colors[j] for j in np.flatnonzero(G[i]) if j != i and colors[j] >= 0}
        c = 0
        while c in used:
            c += 1
        colors[i] = c
    return int(colors.max() + 1)


def diagnostics(A, pre: TwoLevel, tau: float) -> dict:
    """kappa(M^{-1}A), lambda_min/max, k_m (2.2), k_c and the bound
    (k_c + 1)(2 + (2 k_c + 1) k_m / tau) (Sec. 3.2).  Dense; tiny inputs only."""
    A = as_scipy(A)
    Ad = A.toarray()
    n = Ad.shape[0]
    if pre.coarse_solver is None:  # linear: the whole identity in one block apply
        Minv = pre.apply(np.eye(n))
    else:
        Minv = np.column_stack([pre.apply(e) for e in np.eye(n)])
    Minv = 0.5 * (Minv + Minv.T)
    CA = np.linalg.cholesky(Ad)
    lam = np.linalg.eigvalsh(CA.T @ Minv @ CA)
    # k_m: largest eigenvalue of the pencil (sum_i R_i^T A~_ii R_i, A)
    S = np.zeros((n, n))
    for L in pre.locals:
        Om = L.sets.Omega
        S[np.ix_(Om, Om)] += L.split.Atilde_ii
    CAi = np.linalg.inv(CA)
    km = float(np.linalg.eigvalsh(CAi @ S @ CAi.T).max())
    kc = coloring_kc(A, pre.locals)
    return {
        "lambda_min": float(lam.min()), "lambda_max": float(lam.max()),
        "kappa": float(lam.max() / lam.min()), "k_m": km, "k_c": kc,
        "bound": (kc + 1) * (2 + (2 * kc + 1) * km / tau),
        "n_C": pre.nC,
    }
