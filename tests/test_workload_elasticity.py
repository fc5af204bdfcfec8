"""Pins of the elasticity workload generator (the stand-in for the paper's
linear elasticity problems, Section 4) against mechanics fixed independently
of its code:

* the trilinear element stiffness is symmetric positive semidefinite with
  exactly the six rigid-body motions (3 translations, 3 infinitesimal
  rotations) as its null space;
* for a linear displacement u = G x the element energy u^T K u equals
  h^3 (lambda (tr eps)^2 + 2 mu eps:eps), eps = sym(G), written here in
  tensor form (the generator uses Voigt notation), since trilinear functions
  reproduce linear fields and 2x2x2 Gauss integrates the constant exactly;
* the assembled stiffness annihilates the rigid motions, and with one
  material a linear field leaves zero residual at interior nodes (patch
  test);
* after clamping the face x = 0 the matrix is SPD with n = 3 m^2 (m - 1);
* the geometric partition keeps the three dofs of a node together.
"""
import numpy as np

import workloads as W


def _rigid_modes(X):
    """(3k, 6) rigid motions at the points X (k x 3), dof 3a + c."""
    k = X.shape[0]
    R = np.zeros((3 * k, 6))
    for c in range(3):
        R[c::3, c] = 1.0
    # rotations about x, y, z: u = w x X
    for j, w in enumerate(np.eye(3)):
        R[:, 3 + j] = np.cross(np.broadcast_to(w, X.shape), X).reshape(-1)
    return R


def _element_nodes(h):
    return np.array([[(a & 1) * h, ((a >> 1) & 1) * h, ((a >> 2) & 1) * h] for a in range(8)])


def test_element_null_space_is_rigid_motions():
    h = 0.37
    for E, nu in ((1.0, 0.3), (1e5, 0.45), (2.5, 0.0)):
        K = W.elasticity_element(E, nu, h)
        assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
        R = _rigid_modes(_element_nodes(h))
        assert np.abs(K @ R).max() <= 1e-12 * np.abs(K).max()
        ev = np.linalg.eigvalsh(K)
        assert ev.min() >= -1e-12 * ev.max()
        assert int((ev <= 1e-10 * ev.max()).sum()) == 6


def test_element_uniform_strain_energy():
    rng = np.random.default_rng(3)
    h = 0.25
    X = _element_nodes(h)
    for E, nu in ((1.0, 0.3), (1e5, 0.45)):
        lam = E * nu / ((1 + nu) * (1 - 2 * nu))
        mu = E / (2 * (1 + nu))
        K = W.elasticity_element(E, nu, h)
        for _ in range(5):
            G = rng.standard_normal((3, 3))
            u = (X @ G.T).reshape(-1)       # u(x) = G x at each node
            eps = 0.5 * (G + G.T)
            expect = h ** 3 * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
            assert abs(u @ K @ u - expect) <= 1e-12 * abs(expect)


def test_assembled_rigid_motions_and_patch():
    m = 5
    h = 1.0 / (m - 1)
    g = np.arange(m) * h
    iz, iy, ix = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    X = np.stack([g[ix.ravel()], g[iy.ravel()], g[iz.ravel()]], axis=1)  # node k = (iz m + iy) m + ix
    K = W.elasticity3d_stiffness(m, layer=2)
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()
    R = _rigid_modes(X)
    assert np.abs(K @ R).max() <= 1e-10 * abs(K).max()
    # patch test with one material: interior residual of a linear field is zero
    Kh = W.elasticity3d_stiffness(m, layer=2, young=(3.0, 3.0), poisson=(0.25, 0.25))
    G = np.random.default_rng(5).standard_normal((3, 3))
    r = Kh @ (X @ G.T).reshape(-1)
    inner = ((ix > 0) & (ix < m - 1) & (iy > 0) & (iy < m - 1) & (iz > 0) & (iz < m - 1)).ravel()
    dof_inner = np.repeat(inner, 3)
    assert np.abs(r[dof_inner]).max() <= 1e-11 * abs(Kh).max()
    assert np.abs(r[~dof_inner]).max() > 1e-3 * abs(Kh).max()


def test_clamped_matrix_spd_and_size():
    m = 4
    A = W.elasticity3d(m, layer=1)
    assert A.n == 3 * m * m * (m - 1)
    S = A.to_scipy().toarray()
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    assert np.linalg.eigvalsh(S).min() > 0
    # rows/columns sorted and unique
    for i in range(A.n):
        c = A.colind[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_partition_groups_node_dofs():
    m, p = 12, 3
    part = W.elasticity3d_partition(m, p)
    assert part.size == 3 * m * m * (m - 1)
    assert np.all(part[0::3] == part[1::3]) and np.all(part[0::3] == part[2::3])
    counts = np.bincount(part, minlength=p ** 3)
    assert counts.min() > 0 and counts.sum() == part.size
