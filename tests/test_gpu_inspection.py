"""Inspection and failure paths through the C-ABI, against the oracle:

* the dense blocks A_ii = A(Omega_i, Omega_i) and X_i = A(Omega_i, Omega~_i) of
  (3.1) as the setup extracts them are bit-exact against the oracle's
  extraction (the values are copies, so nothing may differ);
* dd_info's colouring constant k_c equals the oracle's greedy colouring of
  the subdomain graph (Sec. 3.2 bound), and its p_i histogram counts every
  subdomain once in the right bin;
* a matrix whose local block is indefinite is refused with DD_ERR_NOT_SPD
  (local Cholesky breakdown, Sec. 4 exact local solver) and no handle;
* PCG stopped by maxit returns DD_WARN_MAXIT with the true residual of the
  iterate it reached, which equals the oracle's iterate after as many steps.
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

from paper_2109_05908_amd import DDError, DeviceCSR, Preconditioner, extract_local  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cases():
    c1 = W.config_c1()
    s3 = W.config_small3d()
    r = W.random_spd(600, 5, seed=1)
    return [
        ("c1", c1.A, c1.part, 16, 1),
        ("small3d", s3.A, O.ggg_partition(s3.A, s3.N, 0), s3.N, 2),
        ("rand", r, W.contiguous_partition(600, 6), 6, 2),
    ]


@pytest.mark.parametrize("case", range(3))
def test_extracted_blocks_bit_exact(case):
    name, A, part, N, delta = _cases()[case]
    dA = DeviceCSR.from_workload(A)
    sets = O.subdomain_sets(A, part, N, delta)
    for i in sorted({0, N // 2, N - 1}):
        log(f"[inspect] extraction {name} subdomain {i}")
        sz, Aii, X = extract_local(dA, part, N, delta, i)
        s = sets[i]
        assert sz == (s.I.size, s.Gamma.size, s.Delta.size)
        Ao, Xo = O.extract(A, s)
        assert np.array_equal(Aii, Ao)
        assert np.array_equal(X, Xo)


def test_kc_and_histogram_match_oracle():
    for name, A, part, N, delta in _cases():
        pre = Preconditioner(DeviceCSR.from_workload(A), part, N, delta, 0.1)
        inf = pre.info()
        locs = O.build_locals(A, part, N, delta, 0.1, keep_split=False)
        kc = O.coloring_kc(A, locs)
        log(f"[inspect] {name}: k_c GPU {inf['k_c']} oracle {kc}; p_hist {inf['p_hist']}")
        assert inf["k_c"] == kc
        p = pre.sizes()[:, 3]
        hist = np.zeros(16, dtype=int)
        for v in p:
            b = 0 if v == 0 else min(15, int(v).bit_length())
            hist[b] += 1
        assert list(hist) == inf["p_hist"]
        assert sum(inf["p_hist"]) == N


def test_indefinite_local_block_is_refused():
    A = W.poisson2d(16).to_scipy().tolil()
    A[37, 37] = -6.0  # symmetric, indefinite: A_ii of the part holding node 37 has no Cholesky factor
    A = sp.csr_matrix(A)
    A.sort_indices()
    part = W.grid2d_partition(16, 2, 2)
    log("[inspect] indefinite local block")
    with pytest.raises(DDError) as e:
        Preconditioner(DeviceCSR(A.shape[0], A.indptr, A.indices, A.data), part, 4, 1, 0.1)
    assert e.value.code == -2


def test_pcg_maxit_returns_warning_and_the_iterate():
    cfg = W.config_c1()  # GPU and oracle applies agree to 1e-10 here, so early iterates do as well
    part = cfg.part
    pre = Preconditioner(DeviceCSR.from_workload(cfg.A), part, cfg.N, cfg.overlap, cfg.tau)
    b = W.rhs(cfg.A.n, 0)
    x, its, rr, code = pre.pcg(torch.as_tensor(b, device="cuda"), rtol=1e-12, maxit=3)
    ora = O.build(cfg.A, part, cfg.N, cfg.overlap, cfg.tau)
    xo, itso, rro = O.pcg(cfg.A, b, ora.apply, rtol=1e-12, maxit=3)
    xg = x.cpu().numpy()
    Asc = cfg.A.to_scipy()
    true = np.linalg.norm(b - Asc @ xg) / np.linalg.norm(b)
    log(f"[inspect] maxit 3: code {code} its {its[0]} relres {rr[0]:.3e} (oracle {rro:.3e})")
    assert code == 1 and its[0] == 3 and itso == 3
    assert rr[0] > 1e-12
    assert abs(rr[0] - true) <= 1e-12 * max(1.0, true)
    assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo)
