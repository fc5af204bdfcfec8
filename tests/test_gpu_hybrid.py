"""Composability, the hybrid case of Sec. 4: the preconditioner solves the
coarse systems of another multilevel method, set up from that method's coarse
operator alone (no near-nullspace handed over).

The other method here is a two-grid smoothed-aggregation cycle written in
this test (it stands in for the GAMG / GenEO hierarchies the paper couples
with): aggregates of 2 x 2 x 2 grid nodes, the tentative prolongator P0
smoothed once by damped Jacobi, P = (I - w D^{-1} A) P0, the coarse operator
A_c = P^T A P, and one pre- and one post-smoothing Jacobi step.  The library
is set up on A_c with its own seeded graph-growing partition and the deflated
variant, and each coarse system is solved by right-preconditioned GMRES(30)
to 1e-4, as the paper's inner solves; the outer solver on A is flexible
GMRES(30).  The oracle runs the same composition with its own preconditioner
of A_c: outer iteration counts within 1 and solutions within 1e-8 at an
outer tolerance of 1e-10.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import DD_SCHWARZ_DEFLATED, DeviceCSR, Preconditioner, partition_ggg  # noqa: E402

OMEGA = 2.0 / 3.0


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _smoothed_aggregation(A, m):
    n = A.shape[0]
    k = np.arange(n)
    ix, iy, iz = k % m, (k // m) % m, k // (m * m)
    h = m // 2
    agg = (iz // 2 * h + iy // 2) * h + ix // 2
    P0 = sp.csr_matrix((np.ones(n), (k, agg)), shape=(n, h ** 3))
    Dinv = 1.0 / A.diagonal()
    P = (P0 - OMEGA * sp.diags(Dinv) @ (A @ P0)).tocsr()
    Ac = (P.T @ A @ P).tocsr()
    Ac = ((Ac + Ac.T) * 0.5).tocsr()
    Ac.sort_indices()
    return P, Ac, Dinv


def _two_grid(A, P, Dinv, coarse):
    def apply(r):
        x = OMEGA * Dinv * r
        x = x + P @ coarse(P.T @ (r - A @ x))
        return x + OMEGA * Dinv * (r - A @ x)
    return apply


def test_hybrid_two_grid_with_coarse_solves_by_the_preconditioner():
    m = 24
    A = W.diffusion3d(m, seed=1).to_scipy().tocsr()
    P, Ac, Dinv = _smoothed_aggregation(A, m)
    nc = Ac.shape[0]
    Nc, tau = 8, 0.1
    dAc = DeviceCSR(nc, Ac.indptr, Ac.indices, Ac.data)
    part = partition_ggg(dAc, Nc, 0)
    np.testing.assert_array_equal(part.cpu().numpy(), O.ggg_partition(Ac, Nc, 0))
    pre = Preconditioner(dAc, part, Nc, 1, tau, schwarz=DD_SCHWARZ_DEFLATED)
    ora = O.build(Ac, part.cpu().numpy(), Nc, 1, tau, variant="deflated")
    log(f"[hybrid] n={A.shape[0]}, coarse operator n_C2={nc} (aggregation), our coarse space n_C3="
        f"{pre.info()['n_C']} (oracle {ora.nC})")
    inner = {"gpu": [], "oracle": []}

    def coarse_gpu(y):
        x, its, rr, code = pre.gmres(torch.as_tensor(y, device="cuda"), rtol=1e-4, restart=30)
        assert code == 0
        inner["gpu"].append(its[0])
        return x.cpu().numpy()

    def coarse_oracle(y):
        x, its, _ = O.gmres(Ac, y, ora.apply, rtol=1e-4, restart=30)
        inner["oracle"].append(its)
        return x

    b = W.rhs(A.shape[0], 3)
    xg, itg, rrg = O.gmres(A, b, _two_grid(A, P, Dinv, coarse_gpu), rtol=1e-10, restart=30, flexible=True)
    xo, ito, rro = O.gmres(A, b, _two_grid(A, P, Dinv, coarse_oracle), rtol=1e-10, restart=30, flexible=True)
    log(f"[hybrid] outer FGMRES its: with the library {itg} (relres {rrg:.2e}), oracle {ito}; "
        f"mean inner GMRES its {np.mean(inner['gpu']):.1f} / {np.mean(inner['oracle']):.1f}")
    assert rrg <= 1e-10 and abs(itg - ito) <= 1
    assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)
