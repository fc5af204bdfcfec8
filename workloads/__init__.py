"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input generation only: sparse SPD test matrices in CSR form
(full symmetric storage, sorted unique column indices per row), geometric
partitions and right-hand sides.  It contains none of the preconditioner's
arithmetic.  The matrices stand in for the paper's workloads (SuiteSparse SPD
matrices and FreeFEM diffusion / elasticity problems, Section 4), which are
not available here.

Conventions
-----------
* A matrix is returned as ``CSR(n, rowptr int32[n+1], colind int32[nnz], val f64[nnz])``.
* Stencils are unscaled (no h^2 factor); Dirichlet neighbours are eliminated,
  so boundary rows keep their full diagonal.
* Every random draw comes from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class CSR:
    n: int
    rowptr: np.ndarray  # int32[n+1]
    colind: np.ndarray  # int32[nnz]
    val: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))


def _from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    """Sum duplicates, sort by (row, col) and return CSR with int32 indices."""
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if len(vals) else vals
    r = (uniq // n).astype(np.int64)
    c = (uniq % n).astype(np.int32)
    counts = np.bincount(r, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    return CSR(n, rowptr.astype(np.int32), c, summed.astype(np.float64))


# --------------------------------------------------------------------------
# 2-D Poisson, 5-point finite differences
# --------------------------------------------------------------------------
def poisson2d(m: int) -> CSR:
    """5-point Laplacian [-1,-1,4,-1,-1] on an m x m grid, node k = iy*m + ix.

    Dirichlet neighbours are eliminated, so every row has diagonal 4 and the
    matrix is integer valued.
    """
    n = m * m
    iy, ix = np.divmod(np.arange(n, dtype=np.int64), m)
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [np.full(n, 4.0)]
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        jy, jx = iy + dy, ix + dx
        ok = (jy >= 0) & (jy < m) & (jx >= 0) & (jx < m)
        rows.append(np.arange(n)[ok])
        cols.append((jy * m + jx)[ok])
        vals.append(np.full(int(ok.sum()), -1.0))
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def diffusion2d(coeff: np.ndarray) -> CSR:
    """5-point finite differences of -div(c grad u) on an m x m grid with the
    node coefficients c (m x m, node k = iy*m + ix): the face coefficient is the
    harmonic mean of its two nodes, a Dirichlet face adds the node's own c to
    the diagonal.  With c = 1 this is poisson2d(m)."""
    m = coeff.shape[0]
    c = np.asarray(coeff, dtype=np.float64).reshape(-1)
    n = m * m
    k = np.arange(n, dtype=np.int64)
    iy, ix = np.divmod(k, m)
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        jy, jx = iy + dy, ix + dx
        ok = (jy >= 0) & (jy < m) & (jx >= 0) & (jx < m)
        nb = jy * m + jx
        face = np.where(ok, 2.0 * c * c[np.where(ok, nb, 0)] / (c + c[np.where(ok, nb, 0)]), c)
        diag += face
        rows.append(k[ok])
        cols.append(nb[ok])
        vals.append(-face[ok])
    rows.append(k)
    cols.append(k)
    vals.append(diag)
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def poisson2d_stiff_pair(m: int = 64, node: int = 24 * 64 + 24, kappa: float = 1e9) -> CSR:
    """diffusion2d with c = 1 except two horizontally adjacent nodes (node,
    node + 1) with c = kappa: a stiff inclusion that floats in its subdomain."""
    c = np.ones((m, m))
    c.reshape(-1)[[node, node + 1]] = kappa
    return diffusion2d(c)


def grid2d_partition(m: int, px: int, py: int) -> np.ndarray:
    """Geometric partition of an m x m grid into py x px blocks.

    part(k) = (iy // (m/py)) * px + (ix // (m/px)) for node k = iy*m + ix.
    """
    iy, ix = np.divmod(np.arange(m * m, dtype=np.int64), m)
    by = (iy * py) // m
    bx = (ix * px) // m
    return (by * px + bx).astype(np.int32)


# --------------------------------------------------------------------------
# 1-D Laplacian (tiny pins)
# --------------------------------------------------------------------------
def laplace1d(n: int) -> CSR:
    """Tridiagonal [-1, 2, -1] with Dirichlet ends eliminated."""
    i = np.arange(n)
    rows = np.concatenate([i, i[1:], i[:-1]])
    cols = np.concatenate([i, i[1:] - 1, i[:-1] + 1])
    vals = np.concatenate([np.full(n, 2.0), np.full(n - 1, -1.0), np.full(n - 1, -1.0)])
    return _from_coo(n, rows, cols, vals)


def contiguous_partition(n: int, N: int) -> np.ndarray:
    """part(k) = floor(k*N/n): N contiguous blocks of nearly equal size."""
    return ((np.arange(n, dtype=np.int64) * N) // n).astype(np.int32)


# --------------------------------------------------------------------------
# Random sparse SPD matrix with an unstructured pattern
# --------------------------------------------------------------------------
def random_spd(n: int, avg_deg: int, seed: int, positive_offdiag: bool = False) -> CSR:
    """Unstructured sparse SPD matrix.

    A random symmetric pattern with about ``avg_deg`` off-diagonal entries per
    row; off-diagonal values uniform in [-1, 1] (or [0, 1] when
    ``positive_offdiag``), diagonal = 1 + row sum of |off-diagonal|, which
    makes the matrix strictly diagonally dominant and therefore SPD.
    """
    rng = np.random.default_rng(seed)
    m = n * avg_deg // 2
    r = rng.integers(0, n, size=m)
    c = rng.integers(0, n, size=m)
    keep = r != c
    r, c = r[keep], c[keep]
    v = rng.uniform(0.0 if positive_offdiag else -1.0, 1.0, size=r.size)
    rows = np.concatenate([r, c])
    cols = np.concatenate([c, r])
    vals = np.concatenate([v, v])
    off = _from_coo(n, rows, cols, vals)
    offrows = np.repeat(np.arange(n), np.diff(off.rowptr))
    absrow = np.bincount(offrows, weights=np.abs(off.val), minlength=n)
    rows_all = np.concatenate([offrows, np.arange(n)])
    cols_all = np.concatenate([off.colind, np.arange(n)])
    vals_all = np.concatenate([off.val, 1.0 + absrow])
    return _from_coo(n, rows_all, cols_all, vals_all)


# --------------------------------------------------------------------------
# 3-D heterogeneous diffusion, 7-point finite volumes
# --------------------------------------------------------------------------
def diffusion3d_coefficient(m: int, seed: int, sigma: float = 2.0, channels: int = 8,
                            contrast: float = 1e6) -> np.ndarray:
    """Node coefficient c = exp(sigma*g), g iid N(0,1), then ``channels``
    axis-aligned straight channels of 2x2 nodes in cross-section, running the
    full length of the grid, set to ``contrast``.  Layout c[iz, iy, ix].
    All draws come from one default_rng(seed) stream: first the n normals,
    then for each channel its axis in {0,1,2} and two transverse offsets in
    [0, m-2].
    """
    rng = np.random.default_rng(seed)
    c = np.exp(sigma * rng.standard_normal((m, m, m)))
    for _ in range(channels):
        axis = int(rng.integers(0, 3))
        a, b = (int(t) for t in rng.integers(0, m - 1, size=2))
        if axis == 0:      # along x: fixed (iz, iy)
            c[a:a + 2, b:b + 2, :] = contrast
        elif axis == 1:    # along y: fixed (iz, ix)
            c[a:a + 2, :, b:b + 2] = contrast
        else:              # along z: fixed (iy, ix)
            c[:, a:a + 2, b:b + 2] = contrast
    return c


def diffusion3d(m: int, seed: int, sigma: float = 2.0, channels: int = 8,
                contrast: float = 1e6) -> CSR:
    """7-point finite-volume diffusion on an m^3 grid, node k = (iz*m+iy)*m+ix.

    Face coefficient = harmonic mean of the two node coefficients; a face on
    the Dirichlet boundary adds the node's own coefficient to the diagonal.
    """
    c = diffusion3d_coefficient(m, seed, sigma, channels, contrast).reshape(-1)
    n = m ** 3
    k = np.arange(n, dtype=np.int64)
    iz, rem = np.divmod(k, m * m)
    iy, ix = np.divmod(rem, m)
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for dz, dy, dx in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)):
        jz, jy, jx = iz + dz, iy + dy, ix + dx
        ok = (jz >= 0) & (jz < m) & (jy >= 0) & (jy < m) & (jx >= 0) & (jx < m)
        j = (jz * m + jy) * m + jx
        w = np.where(ok, 2.0 * c * c[np.where(ok, j, 0)] / (c + c[np.where(ok, j, 0)]), c)
        diag += w
        rows.append(k[ok])
        cols.append(j[ok])
        vals.append(-w[ok])
    rows.append(k)
    cols.append(k)
    vals.append(diag)
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


# --------------------------------------------------------------------------
# 3-D linear elasticity, trilinear hexahedra (Q1), 3 dofs per node
# --------------------------------------------------------------------------
def elasticity_element(young: float, poisson: float, h: float) -> np.ndarray:
    """24 x 24 stiffness of a cube of side h with trilinear shape functions,
    isotropic material, 2x2x2 Gauss quadrature (exact for this element).

    Local node a = dx + 2 dy + 4 dz sits at (dx, dy, dz) h; local dof 3a + c
    is displacement component c (x, y, z).  Strains in Voigt order
    (xx, yy, zz, yz, xz, xy) with engineering shears; lambda and mu from
    (E, nu).
    """
    lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson))
    mu = young / (2.0 * (1.0 + poisson))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] += 2.0 * mu
    C[1, 1] += 2.0 * mu
    C[2, 2] += 2.0 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    sgn = np.array([[(a & 1), (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=float) * 2.0 - 1.0
    g = 1.0 / math.sqrt(3.0)
    K = np.zeros((24, 24))
    for xi in (-g, g):
        for eta in (-g, g):
            for zeta in (-g, g):
                q = np.array([xi, eta, zeta])
                f = 1.0 + sgn * q                      # (8, 3) factors (1 + s_k q_k)
                dN = np.empty((8, 3))                  # dN_a / d(xi, eta, zeta)
                dN[:, 0] = sgn[:, 0] * f[:, 1] * f[:, 2] / 8.0
                dN[:, 1] = f[:, 0] * sgn[:, 1] * f[:, 2] / 8.0
                dN[:, 2] = f[:, 0] * f[:, 1] * sgn[:, 2] / 8.0
                dx = dN * (2.0 / h)                    # the map is x = (h/2)(xi + 1)
                B = np.zeros((6, 24))
                for a in range(8):
                    gx, gy, gz = dx[a]
                    B[0, 3 * a] = gx
                    B[1, 3 * a + 1] = gy
                    B[2, 3 * a + 2] = gz
                    B[3, 3 * a + 1] = gz
                    B[3, 3 * a + 2] = gy
                    B[4, 3 * a] = gz
                    B[4, 3 * a + 2] = gx
                    B[5, 3 * a] = gy
                    B[5, 3 * a + 1] = gx
                K += B.T @ C @ B * (h / 2.0) ** 3
    return K


def elasticity3d_stiffness(m: int, layer: int = 6, young=(1.0, 1e5), poisson=(0.3, 0.45)):
    """Assembled stiffness (scipy CSR, 3 m^3 dofs, no boundary conditions) of
    the unit cube meshed by (m-1)^3 trilinear hexahedra, node k =
    (iz*m+iy)*m+ix, dof 3k + component.  Elements are layered along z,
    ``layer`` elements thick, alternating between material 0 (young[0],
    poisson[0]) and material 1.  Every element coupling is kept in the pattern
    (the 3 x 3 blocks of all node pairs that share an element)."""
    import scipy.sparse as sp
    h = 1.0 / (m - 1)
    Ke = np.stack([elasticity_element(young[t], poisson[t], h) for t in range(2)])
    ne = m - 1
    e = np.arange(ne ** 3, dtype=np.int64)
    ez, rem = np.divmod(e, ne * ne)
    ey, ex = np.divmod(rem, ne)
    mat = (ez // layer) % 2
    nodes = np.stack([((ez + ((a >> 2) & 1)) * m + (ey + ((a >> 1) & 1))) * m + (ex + (a & 1)) for a in range(8)],
                     axis=1)
    dofs = (3 * nodes[:, :, None] + np.arange(3)).reshape(-1, 24)
    rows = np.repeat(dofs, 24, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, 24)).reshape(-1)
    vals = Ke[mat].reshape(-1)
    nd = 3 * m ** 3
    K = sp.coo_matrix((vals, (rows, cols)), shape=(nd, nd)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return K


def elasticity3d(m: int, layer: int = 6, young=(1.0, 1e5), poisson=(0.3, 0.45)) -> CSR:
    """3-D linear elasticity on an m^3-node grid (see ``elasticity3d_stiffness``)
    with the face x = 0 clamped: its dofs are removed, leaving n = 3 m^2 (m-1)
    unknowns in the original order."""
    K = elasticity3d_stiffness(m, layer, young, poisson)
    nd = 3 * m ** 3
    keep = np.nonzero((np.arange(nd) // 3) % m > 0)[0]
    A = K[keep][:, keep].tocsr()
    A.sort_indices()
    if A.nnz >= 2 ** 31:
        raise ValueError("nnz exceeds int32 range")
    return CSR(A.shape[0], A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


def elasticity3d_partition(m: int, p: int) -> np.ndarray:
    """Geometric p x p x p partition by node (all three dofs of a node in one
    part) for ``elasticity3d(m)``: part = (bz p + by) p + bx with b = i p // m."""
    nd = 3 * m ** 3
    node = np.arange(nd) // 3
    iz, rem = np.divmod(node, m * m)
    iy, ix = np.divmod(rem, m)
    part = ((iz * p // m) * p + (iy * p // m)) * p + (ix * p // m)
    return part[ix > 0].astype(np.int32)


# --------------------------------------------------------------------------
# Right-hand sides and configuration helpers
# --------------------------------------------------------------------------
def rhs(n: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """b iid N(0,1) from default_rng(seed); shape (n,) or column-major (n, nrhs)."""
    rng = np.random.default_rng(seed)
    if nrhs == 1:
        return rng.standard_normal(n)
    return np.asfortranarray(rng.standard_normal((nrhs, n)).T)


@dataclass(frozen=True)
class Config:
    name: str
    A: CSR
    part: np.ndarray | None   # None: seeded greedy graph growing (computed by the method)
    N: int
    overlap: int
    tau: float                # the paper's tau: keep lambda > 1/tau
    levels: int
    ggg_seed: int = 0
    nev_cap: int = 0          # > 0: keep at most the nev_cap smallest mu below tau per subdomain


def config_c1() -> Config:
    """2-D Poisson 64x64, 4x4 geometric subdomains, overlap 1, lambda > 10, 2 levels."""
    m = 64
    return Config("poisson2d_64x64_N16", poisson2d(m), grid2d_partition(m, 4, 4), 16, 1, 0.1, 2)


def config_c2(m: int = 64, N: int = 256, seed: int = 0) -> Config:
    """3-D log-normal diffusion with 1e6 channels, GGG partition, overlap 2, lambda > 50."""
    return Config(f"diffusion3d_{m}^3_N{N}", diffusion3d(m, seed), None, N, 2, 0.02, 2, ggg_seed=0)


def config_small3d(m: int = 16, N: int = 16, seed: int = 0) -> Config:
    """Down-scaled version of the 3-D diffusion workload (oracle-sized)."""
    return Config(f"diffusion3d_{m}^3_N{N}", diffusion3d(m, seed), None, N, 2, 0.02, 2, ggg_seed=0)


def config_c3(m: int = 48, p: int = 8, nev_cap: int = 20) -> Config:
    """3-D layered linear elasticity (E 1 / 1e5, nu 0.3 / 0.45, layers 6
    elements thick), 48^3 nodes, face x = 0 clamped (n = 324864), 8x8x8
    geometric parts, overlap 1, lambda > 10, 3 levels, at most nev_cap kept
    modes per subdomain."""
    return Config(f"elasticity3d_{m}^3_N{p ** 3}", elasticity3d(m), elasticity3d_partition(m, p), p ** 3, 1, 0.1, 3,
                  nev_cap=nev_cap)


def config_small_elasticity(m: int = 10, p: int = 2, levels: int = 2, nev_cap: int = 0) -> Config:
    """Down-scaled layered elasticity (oracle-sized): 10^3 nodes, 2x2x2 parts."""
    return Config(f"elasticity3d_{m}^3_N{p ** 3}", elasticity3d(m, layer=3), elasticity3d_partition(m, p), p ** 3, 1,
                  0.1, levels, nev_cap=nev_cap)


def log_uniform_sizes(count: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))


# --------------------------------------------------------------------------
# Batch of independent systems of uneven size (the many-systems workload)
# --------------------------------------------------------------------------
C5_KINDS = ("poisson2d_5pt", "diffusion3d_7pt_contrast1e6", "elasticity3d_layered")


def batch_system(kind: str, n_target: float, seed: int) -> CSR:
    """One system of the batch, sized as close to n_target unknowns as its grid allows:
    the 5-point Laplacian on an m x m grid, the 7-point log-normal diffusion with 1e6
    channels on m^3 nodes (coefficient seed `seed`), or the layered elasticity on m^3
    nodes (3 m^2 (m-1) unknowns after the clamped face)."""
    if kind == "poisson2d_5pt":
        return poisson2d(max(8, int(round(math.sqrt(n_target)))))
    if kind == "diffusion3d_7pt_contrast1e6":
        return diffusion3d(max(6, int(round(n_target ** (1.0 / 3.0)))), seed)
    if kind == "elasticity3d_layered":
        m = max(6, int(round((n_target / 3.0) ** (1.0 / 3.0))))
        while m > 6 and 3 * m * m * (m - 1) > 1.05 * n_target:
            m -= 1
        return elasticity3d(m)
    raise ValueError(kind)


def batch_plan(count: int = 64, lo: float = 2e4, hi: float = 5e5, seed: int = 0) -> list[tuple[str, float, int]]:
    """(kind, target size, coefficient seed) of every system: sizes log-uniform in [lo, hi]
    (seeded), kinds in turn 2-D 5-point, 3-D high-contrast 7-point, 3-D elasticity."""
    sizes = log_uniform_sizes(count, lo, hi, seed)
    return [(C5_KINDS[j % 3], float(sizes[j]), 1000 + j) for j in range(count)]

