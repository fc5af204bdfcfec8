"""Block eigensolver (LOBPCG, cap mode) and its learned start, through the C-ABI.

Parity of the block solver against the oracle's dense eigensolver of (3.3)
with the nev cap, explicit and matrix-free operator:
* kept counts equal; kept mu >= 1e-6 within 1e-4 relative (the kept-eigenvalue tolerance);
* which vectors of a near-kernel cluster the cap keeps is not fixed by the
  method, so the kept span is checked to lie in the oracle's cluster: the span
  of the pencil's eigenvectors with mu below 1e3 times the largest kept mu
  (a gap of three orders separates that cluster from the rest);
* PCG with the resulting preconditioner: iterations within max(3, 10 %) of
  the oracle's cap-mode run, x within 1e-10 at rtol 1e-13.

The network: forward and gradient equal the CPU reference to 1e-10 on random
inputs; the features and training targets the library computes from a setup
equal the CPU reference's (threshold mode at C1, where the kept span is
unique).  Training on a family of matrices lowers the loss, and on held-out
matrices the learned start needs fewer iterations than the random start and
leaves smaller eigen-residuals at a fixed small budget.
"""
import sys

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from oracle import warm_start as WS
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import (  # noqa: E402
    DD_EIG_LOBPCG, DD_EIG_LOBPCG_MATFREE, DD_SEL_THRESHOLD_CAP, DD_START_MODEL, DD_START_RANDOM, DD_START_RANGE,
    DeviceCSR, Preconditioner, WarmStartModel,
)

MU_FLOOR = 1e-6
MU_RTOL = 1e-4


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(name):
    if name == "c1":
        c = W.config_c1()
        return c.A, c.part, 16, 1, 0.1
    if name == "small3d":
        c = W.config_small3d()
        return c.A, O.ggg_partition(c.A, c.N, 0), c.N, 2, 0.02
    if name == "rand":
        A = W.random_spd(600, 5, seed=1)
        return A, W.contiguous_partition(600, 6), 6, 2, 0.1
    c = W.config_small_elasticity()
    return c.A, c.part, c.N, c.overlap, c.tau


@pytest.mark.parametrize("mode", [DD_EIG_LOBPCG, DD_EIG_LOBPCG_MATFREE])
@pytest.mark.parametrize("name", ["c1", "small3d", "rand", "elast"])
def test_lobpcg_cap_parity(name, mode):
    A, part, N, delta, tau = _case(name)
    nev = 8
    log(f"[lobpcg] {name} mode {mode} nev {nev}")
    pre = Preconditioner(DeviceCSR.from_workload(A), part, N, delta, tau, select=DD_SEL_THRESHOLD_CAP, nev_cap=nev,
                         eig_solver=mode)
    locs = O.build_locals(A, part, N, delta, tau, nev=nev)
    sizes = pre.sizes()
    its_e, res_e = pre.eig_stats()
    # the matrix-free form resolves mu only to its absolute residual (1e-12): a kept vector may
    # hold components of size 1e-12 / mu along eigenvectors of eigenvalue mu, so its span is
    # checked against the cluster mu <= 1e-8 (components <= 1e-4)
    res_floor = 1e-8 if mode == DD_EIG_LOBPCG_MATFREE else 0.0
    worst_mu, worst_span = 0.0, 0.0
    for i, L in enumerate(locs):
        assert sizes[i, 3] == L.mu_keep.size, (i, sizes[i, 3], L.mu_keep.size)
        mu_g = pre.eigs(i)
        big = L.mu_keep >= MU_FLOOR
        if big.any():
            worst_mu = max(worst_mu, float(np.max(np.abs(mu_g[big] - L.mu_keep[big]) / L.mu_keep[big])))
        if L.mu_keep.size:
            nI = L.sets.I.size
            mu, Wv = sla.eigh(L.split.S_I, L.Aii[:nI, :nI])
            clus = mu <= max(1e3 * L.mu_keep.max(), res_floor)
            Qc = np.linalg.qr(Wv[:, clus])[0]
            Zg = pre.basis(i)
            r = Zg - Qc @ (Qc.T @ Zg)
            worst_span = max(worst_span, float(np.linalg.norm(r) / np.linalg.norm(Zg)))
    log(f"[lobpcg] {name}: worst kept-mu rel {worst_mu:.2e}, worst span residual {worst_span:.2e}, "
        f"iterations max {its_e.max()} mean {its_e.mean():.1f}, residual max {res_e.max():.1e}")
    assert worst_mu <= MU_RTOL
    # the near-kernel vectors are determined only to about eps sigma_1 / lambda_min(A_I) (angles up
    # to ~1e-4 on the 3-D problems, as for the dense route); the matrix-free form's components of
    # up to 1e-4 along each eigenvector beyond its cluster add up to about 1e-3
    assert worst_span <= (1e-4 if mode == DD_EIG_LOBPCG else 1e-3)
    assert pre.info()["eig_maxit_hits"] == 0
    ora = O.build(A, part, N, delta, tau, nev=nev)
    b = W.rhs(A.n, 0)
    x, its, rr, code = pre.pcg(torch.as_tensor(b, device="cuda"), rtol=1e-13, maxit=2000)
    xo, itso, _ = O.pcg(A, b, ora.apply, rtol=1e-13, maxit=2000)
    log(f"[lobpcg] {name}: PCG its {its[0]} oracle (dense cap) {itso}")
    # which part of the near-kernel cluster the cap keeps is not fixed by the method (parity
    # unpinned); the matrix-free form, which cannot order it below 1e-7, may keep a weaker part
    slack = max(3, itso // 10) if mode == DD_EIG_LOBPCG else max(3, (3 * itso) // 10)
    assert code == 0 and abs(its[0] - itso) <= slack
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


def test_block_solver_requires_cap_mode():
    from paper_2109_05908_amd import DDError
    c = W.config_c1()
    dA = DeviceCSR.from_workload(c.A)
    for kw in ({}, {"select": DD_SEL_THRESHOLD_CAP, "nev_cap": 0}, {"select": DD_SEL_THRESHOLD_CAP, "nev_cap": 33}):
        with pytest.raises(DDError) as e:
            Preconditioner(dA, c.part, 16, 1, 0.1, eig_solver=DD_EIG_LOBPCG, **kw)
        assert e.value.code == -1


def test_network_forward_and_gradient_match_cpu():
    rng = np.random.default_rng(7)
    p = rng.standard_normal(WS.NPARAM) * 0.3
    X = rng.standard_normal((3000, WS.F)) * 1.5 + 0.5
    mean, std = X.mean(0), X.std(0) + 0.05
    t = np.abs(rng.standard_normal(3000)) + 0.1
    c = rng.uniform(0.1, 1.0, 3000)
    m = WarmStartModel(0)
    m.set_params(np.concatenate([p, mean, std]))
    wg = m.forward(X)
    wc = WS.mlp_forward(p, mean, std, X)
    assert np.max(np.abs(wg - wc)) <= 1e-12 * np.max(np.abs(wc))
    lg, gg = m.loss_grad(X, t, c)
    lc, gc = WS.mlp_loss_grad(p, mean, std, X, t, c)
    log(f"[lobpcg] network: loss {lg:.6e} vs {lc:.6e}, gradient rel diff {np.linalg.norm(gg - gc) / np.linalg.norm(gc):.1e}")
    assert abs(lg - lc) <= 1e-12 * abs(lc)
    assert np.linalg.norm(gg - gc) <= 1e-10 * np.linalg.norm(gc)


def test_samples_match_cpu_reference_c1():
    c = W.config_c1()
    pre = Preconditioner(DeviceCSR.from_workload(c.A), c.part, 16, 1, 0.1)
    m = WarmStartModel(0)
    m.add_samples(pre)
    f, t, w = m.samples()
    A = c.A.to_scipy()
    locs = O.build_locals(c.A, c.part, 16, 1, 0.1, keep_split=False)
    o = 0
    for L in locs:
        if not L.Z_I.shape[1] or not L.sets.Delta.size:
            continue
        nD = L.sets.Delta.size
        fo = WS.features(A, L.sets)
        to = WS.targets(A, L.sets, L.Aii, L.Z_I)
        assert np.max(np.abs(f[o:o + nD] - fo)) <= 1e-12
        assert np.max(np.abs(t[o:o + nD] - to)) <= 1e-6, np.max(np.abs(t[o:o + nD] - to))
        np.testing.assert_allclose(w[o:o + nD], 1.0 / nD, rtol=1e-15)
        o += nD
    assert o == f.shape[0]


def _family(seed):
    return W.diffusion3d(16, seed)


def test_learned_start_on_held_out_matrices():
    """Train on the kept eigenvectors (dense route, cap 16) of matrices 0..11 of a
    16^3 diffusion family, test on 12..15 against the random start.  Judged by
    the eigen-residual after two iterations, by the iterations to an eigen-
    residual of 1e-4 (the coarse space is as good as with converged vectors:
    PCG takes the same iterations) and by PCG with the resulting spaces."""
    nev, N = 16, 16
    A0 = _family(0)
    part = O.ggg_partition(A0, N, 0)
    m = WarmStartModel(1)
    for sd in range(12):
        P = Preconditioner(DeviceCSR.from_workload(_family(sd)), part, N, 2, 0.02, select=DD_SEL_THRESHOLD_CAP,
                           nev_cap=nev)
        m.add_samples(P)
        del P
    loss = m.train(400, 1e-2)
    log(f"[lobpcg] training loss {loss[0]:.4f} -> {loss[-1]:.4f}")
    assert loss[-1] < 0.7 * loss[0]
    stats = {}
    for sd in range(12, 16):
        dA = DeviceCSR.from_workload(_family(sd))
        b = torch.as_tensor(W.rhs(dA.n, 0), device="cuda")
        ref = Preconditioner(dA, part, N, 2, 0.02, select=DD_SEL_THRESHOLD_CAP, nev_cap=nev, eig_solver=DD_EIG_LOBPCG,
                             seed=sd)
        _, rits, _, _ = ref.pcg(b, rtol=1e-8, maxit=2000)
        for name, ws, model in (("random", DD_START_RANDOM, None), ("range", DD_START_RANGE, None),
                                ("model", DD_START_MODEL, m)):
            kw = dict(select=DD_SEL_THRESHOLD_CAP, nev_cap=nev, eig_solver=DD_EIG_LOBPCG, warm_start=ws, model=model,
                      seed=sd)
            P = Preconditioner(dA, part, N, 2, 0.02, lobpcg_tol=1e-4, **kw)
            its, _ = P.eig_stats()
            _, pits, _, _ = P.pcg(b, rtol=1e-8, maxit=2000)
            Pb = Preconditioner(dA, part, N, 2, 0.02, lobpcg_maxit=2, **kw)
            _, rb = Pb.eig_stats()
            st = stats.setdefault(name, {"its": [], "res2": [], "pcg": [], "ref": []})
            st["its"].append(its.mean())
            st["res2"].append(np.median(rb))
            st["pcg"].append(pits[0])
            st["ref"].append(rits[0])
    for name, st in stats.items():
        log(f"[lobpcg] held-out {name}: LOBPCG iterations to 1e-4 {np.mean(st['its']):.2f}, median residual after 2 "
            f"{np.median(st['res2']):.2e}, PCG its {st['pcg']} (converged-space reference {st['ref']})")
    assert np.mean(stats["model"]["its"]) < np.mean(stats["random"]["its"])
    assert np.median(stats["model"]["res2"]) <= 0.2 * np.median(stats["random"]["res2"])
    for st in stats.values():
        assert all(abs(a - r) <= 2 for a, r in zip(st["pcg"], st["ref"]))
