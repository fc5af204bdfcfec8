"""Pins of the CPU reference of the learned start (CPU only).

* the network's gradient against central finite differences;
* the boundary features against values worked out by hand on the 1-D
  Laplacian, where every entry is known;
* the training target depends only on the kept span (invariant under a
  rotation of Z_i), its squares sum to |Delta_i| (the leverages of an
  orthonormal basis of rank p sum to p);
* the range start with the whole boundary data spans the near kernel of the
  splitting, which at C1 is exactly the kept space (Sec. 3.2; the near-kernel
  identity pinned in test_oracle_pins).
"""
import math

import numpy as np
import scipy.linalg as sla

import oracle as O
from oracle import warm_start as WS
import workloads as W


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(WS.NPARAM) * 0.3
    X = rng.standard_normal((40, WS.F)) * 2.0 + 1.0
    mean, std = X.mean(0), X.std(0) + 0.1
    t = np.abs(rng.standard_normal(40)) + 0.2
    c = rng.uniform(0.1, 1.0, 40)
    loss, g = WS.mlp_loss_grad(p, mean, std, X, t, c)
    assert math.isclose(loss, float(np.sum(c * (WS.mlp_forward(p, mean, std, X) - t) ** 2)), rel_tol=1e-14)
    h = 1e-6
    idx = rng.choice(WS.NPARAM, 60, replace=False)
    for k in list(idx) + [WS.NPARAM - 1, 0, WS.F * WS.H]:
        e = np.zeros(WS.NPARAM)
        e[k] = h
        fd = (WS.mlp_loss_grad(p + e, mean, std, X, t, c)[0] - WS.mlp_loss_grad(p - e, mean, std, X, t, c)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_features_on_the_1d_laplacian_by_hand():
    """1-D Laplacian [-1 2 -1], n = 12, two parts of 6, overlap 1: subdomain 0
    has Omega = {0..6} and Delta = {7}.  Node 7 has diagonal 2, one neighbour
    inside (6, link 1) and one outside (8); node 6's other link inside is to 5
    (strength 1); every diagonal is 2, so s_0 = log 2."""
    A = W.laplace1d(12)
    part = W.contiguous_partition(12, 2)
    s = O.subdomain_sets(A, part, 2, 1)[0]
    assert list(s.Delta) == [7]
    f = WS.features(A.to_scipy(), s)[0]
    l2 = math.log(2.0)
    expect = [0.0, -l2, -l2, 0.5, 0.0, 0.0, -l2, 0.0]
    np.testing.assert_allclose(f, expect, atol=1e-15)


def test_target_is_a_function_of_the_span():
    cfg = W.config_c1()
    A = cfg.A.to_scipy()
    locs = O.build_locals(cfg.A, cfg.part, 16, 1, 0.1, nev=12, keep_split=False)
    for i in (0, 5):
        L = locs[i]
        t = WS.targets(A, L.sets, L.Aii, L.Z_I)
        assert math.isclose(float(np.sum(t ** 2)), L.sets.Delta.size, rel_tol=1e-10)
        Q = np.linalg.qr(np.random.default_rng(i).standard_normal((12, 12)))[0]
        np.testing.assert_allclose(WS.targets(A, L.sets, L.Aii, L.Z_I @ Q), t, atol=1e-10)


def test_range_start_spans_the_kept_space_at_c1():
    cfg = W.config_c1()
    A = cfg.A.to_scipy()
    locs = O.build_locals(cfg.A, cfg.part, 16, 1, 0.1, keep_split=False)
    for i in (0, 5):
        L = locs[i]
        nD = L.sets.Delta.size
        X = WS.range_start(A, L.sets, L.Aii, np.ones(nD), np.eye(nD))
        U, sv, _ = np.linalg.svd(X, full_matrices=False)
        r = int(np.sum(sv > 1e-10 * sv[0]))
        assert r == L.Z_I.shape[1]
        ang = sla.subspace_angles(U[:, :r], L.Z_I)
        assert ang.max() <= 1e-8, ang.max()
