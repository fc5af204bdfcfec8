"""The reading behind the polar iteration's switch (CPU, numpy): dynamically
weighted Halley iterations (QDWH, Nakatsukasa, Bai & Gygi 2010) that take
the Cholesky form from c <= 2e4 instead of the customary c <= 100 still give
the square root H = (R^T R)^{1/2} to within 1e-12 relative of the SVD's, and
its eigenvalues within 1e-13 of sigma_1, for condition numbers 1e6 to 1e12.
The weights are the published ones; nothing here is the GPU code."""
import math

import numpy as np
import pytest
import scipy.linalg as sla


def weights(l):
    d = (4.0 * (1.0 - l * l) / l ** 4) ** (1.0 / 3.0)
    a = math.sqrt(1.0 + d) + 0.5 * math.sqrt(8.0 - 4.0 * d + 8.0 * (2.0 - l * l) / (l * l * math.sqrt(1.0 + d)))
    b = (a - 1.0) ** 2 / 4.0
    return a, b, a + b - 1.0


def polar_sqrt(R, switch):
    n = R.shape[0]
    alpha = 1.01 * np.linalg.norm(R, 2)
    l = 0.9 / (alpha * np.linalg.norm(np.linalg.inv(R), 2))
    X = R / alpha
    while abs(1.0 - l) >= 1e-14:
        a, b, c = weights(l)
        if c > switch:
            Q, _ = np.linalg.qr(np.vstack([math.sqrt(c) * X, np.eye(n)]))
            X = b / c * X + (a - b / c) / math.sqrt(c) * Q[:n] @ Q[n:].T
        else:
            L = np.linalg.cholesky(np.eye(n) + c * X.T @ X)
            W = sla.solve_triangular(L.T, sla.solve_triangular(L, X.T, lower=True), lower=False)
            X = b / c * X + (a - b / c) * W.T
        l = l * (a + b * l * l) / (1.0 + c * l * l)
    H = X.T @ R
    return 0.5 * (H + H.T)


@pytest.mark.parametrize("kappa", [1e6, 1e8, 1e10, 1e12])
def test_cholesky_form_from_c_2e4_keeps_h_accurate(kappa):
    rng = np.random.default_rng(int(math.log10(kappa)))
    n = 160
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0, -math.log10(kappa), n)
    R = np.linalg.qr(U @ np.diag(s) @ V.T, mode="r")
    _, sv, Vt = np.linalg.svd(R)
    H_svd = Vt.T @ np.diag(sv) @ Vt
    for switch in (100.0, 2e4):
        H = polar_sqrt(R, switch)
        assert np.linalg.norm(H - H_svd) <= 1e-12 * np.linalg.norm(H_svd)
        ev = np.sort(np.linalg.eigvalsh(H))[::-1]
        assert np.max(np.abs(ev - sv)) <= 1e-13 * sv[0]
