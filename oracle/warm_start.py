"""FP64 CPU reference of the learned start of the local eigensolver -- test
infrastructure only (only tests/, the smoke check and the benchmark's CPU
baseline may import it; the product path never does).

What it computes, from the definitions:

* the near kernel of the splitting (Sec. 3.2, the kernel of the SPSD splitting
  is the range of A_ii^{-1} A(Omega_i, Delta_i) applied to data on Delta_i), so a
  start block for the eigenproblem (3.3) is X = [A_ii^{-1} A(Omega_i, Delta_i)
  diag(w) G]_{Omega_Ii}, G Gaussian on Delta_i, w >= 0 a weight per boundary node;
* eight features of every boundary node d, from A alone, relative to the mean
  log diagonal s_i of Omega_i: log a_dd - s_i; log(sum_in |a_dr|) - log a_dd;
  log(max_in |a_dr|) - s_i; (number of in-neighbours) / (number of neighbours);
  log(sum_all |a_du|) - s_i; mean_in log a_rr - s_i; log of the strongest link
  from an in-neighbour r to another node of Omega_i, minus s_i; log(max_in a_rr) - s_i
  ("in" = neighbours of d inside Omega_i, u ranges over all neighbours u != d);
* the training target of the weights: with Z_i the kept eigenvectors (D-image),
  B = A(Delta_i, Omega_i) A_ii^{-1} [Z_i; 0] is the boundary data that reproduces
  them; t(d)^2 = |Delta_i| / p_i * (row d of an orthonormal basis of range(B))^2,
  which depends only on the kept span;
* the network: 8 standardised inputs, two tanh layers of 32, softplus output;
  loss sum_s c_s (w_s - t_s)^2; its gradient by the chain rule.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

F, H = 8, 32
NPARAM = F * H + H + H * H + H + H + 1


def _log(x):
    return np.log(np.maximum(x, 1e-300))


def features(A, s) -> np.ndarray:
    """Features of the boundary nodes Delta_i of one subdomain (rows in Delta_i order)."""
    A = sp.csr_matrix(A)
    diag = np.abs(A.diagonal())
    om = np.concatenate([s.I, s.Gamma])
    inside = np.zeros(A.shape[0], dtype=bool)
    inside[om] = True
    si = float(np.mean(_log(diag[om]))) if om.size else 0.0
    out = np.zeros((s.Delta.size, F))
    for a, d in enumerate(s.Delta):
        cols = A.indices[A.indptr[d]:A.indptr[d + 1]]
        vals = np.abs(A.data[A.indptr[d]:A.indptr[d + 1]])
        off = cols != d
        add = float(vals[~off].sum()) if (~off).any() else 0.0
        nb, nv = cols[off], vals[off]
        m = inside[nb]
        rin, vin = nb[m], nv[m]
        hop = 0.0
        for r in rin:
            c2 = A.indices[A.indptr[r]:A.indptr[r + 1]]
            v2 = np.abs(A.data[A.indptr[r]:A.indptr[r + 1]])
            k = (c2 != r) & inside[c2]
            if k.any():
                hop = max(hop, float(v2[k].max()))
        out[a, 0] = _log(add) - si
        out[a, 1] = _log(vin.sum()) - _log(add)
        out[a, 2] = _log(vin.max() if vin.size else 0.0) - si
        out[a, 3] = rin.size / nb.size if nb.size else 0.0
        out[a, 4] = _log(nv.sum()) - si
        out[a, 5] = float(np.mean(_log(diag[rin]))) - si if rin.size else 0.0
        out[a, 6] = _log(hop) - si
        out[a, 7] = _log(diag[rin].max() if rin.size else 0.0) - si
    return out


def targets(A, s, Aii: np.ndarray, Z_I: np.ndarray) -> np.ndarray:
    """t(d) for the boundary nodes of one subdomain from its kept vectors Z_I (n_Ii x p)."""
    A = sp.csr_matrix(A)
    p = Z_I.shape[1]
    ni = s.Omega.size
    U = np.zeros((ni, p))
    U[:s.I.size] = Z_I
    U = np.linalg.solve(Aii, U)
    B = A[s.Delta][:, s.Omega].toarray() @ U
    Q, R = np.linalg.qr(B)
    keep = np.abs(np.diag(R)) > 1e-13 * max(1e-300, np.abs(np.diag(R)).max())
    Q = Q[:, keep]
    return np.sqrt((Q ** 2).sum(1) * s.Delta.size / p)


def range_start(A, s, Aii: np.ndarray, w: np.ndarray, G: np.ndarray) -> np.ndarray:
    """[A_ii^{-1} A(Omega_i, Delta_i) diag(w) G]_{Omega_Ii} (pencil variables)."""
    A = sp.csr_matrix(A)
    Bd = A[s.Omega][:, s.Delta].toarray()
    return np.linalg.solve(Aii, Bd @ (w[:, None] * G))[:s.I.size]


def _unpack(p):
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def _softplus(o):
    return np.where(o > 0, o + np.log1p(np.exp(-np.abs(o))), np.log1p(np.exp(np.minimum(o, 0))))


def mlp_forward(params, mean, std, X) -> np.ndarray:
    W1, b1, W2, b2, w3, b3 = _unpack(np.asarray(params, dtype=np.float64))
    Xs = (X - mean) / std
    h1 = np.tanh(Xs @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return _softplus(h2 @ w3 + b3)


def mlp_loss_grad(params, mean, std, X, t, c):
    """loss = sum_s c_s (w_s - t_s)^2 and d loss / d params (chain rule, layer by layer)."""
    W1, b1, W2, b2, w3, b3 = _unpack(np.asarray(params, dtype=np.float64))
    Xs = (X - mean) / std
    h1 = np.tanh(Xs @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    o = h2 @ w3 + b3
    w = _softplus(o)
    diff = w - t
    loss = float(np.sum(c * diff * diff))
    do = 2.0 * c * diff / (1.0 + np.exp(-o))       # dL/do, softplus' = logistic
    gw3 = h2.T @ do
    gb3 = do.sum()
    dz2 = np.outer(do, w3) * (1.0 - h2 ** 2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (1.0 - h1 ** 2)
    gW1 = dz1.T @ Xs
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return loss, g
