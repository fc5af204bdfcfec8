"""Overlap sets (Sec. 2) and the extraction (3.1) at a subdomain count where a
table of one byte per (subdomain, node) pair could not be held: the 5-point
Laplacian on a 2048 x 2048 grid (n = 4,194,304) in 262,144 geometric blocks
of 4 x 4 nodes, overlap 2.  Such a table would take n * N = 1.1e12 bytes,
about four times the device memory; the frontier lists take space in
proportion to the sets times their row lengths.

Sampled subdomains (corners, the middle, seeded random ones) are compared bit
for bit with the oracle.  The oracle runs on a partition that keeps the
sampled parts and merges every other node into one part: the layers of a
part depend only on A and on that part's own nodes, so its sets and blocks
are those of the full partition."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2109_05908_amd import DeviceCSR  # noqa: E402
from paper_2109_05908_amd.binding import extract_local  # noqa: E402

M = 2048
BLOCKS = 512          # per direction: 4 x 4 nodes per subdomain
OVERLAP = 2


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_sets_and_blocks_at_262144_subdomains():
    A = W.poisson2d(M)
    part = W.grid2d_partition(M, BLOCKS, BLOCKS)
    N = BLOCKS * BLOCKS
    assert A.n * N > 1e12
    rng = np.random.default_rng(7)
    corners = [0, BLOCKS - 1, N // 2 + BLOCKS // 2, N - 1]
    sample = list(dict.fromkeys(corners + [int(v) for v in rng.integers(0, N, 4)]))
    log(f"[sets-scale] n={A.n} N={N} overlap={OVERLAP} sample={sample}")
    dA = DeviceCSR.from_workload(A)

    # the oracle on the sampled parts, the rest merged into part len(sample)
    part2 = np.full(A.n, len(sample), dtype=np.int32)
    for k, i in enumerate(sample):
        part2[part == i] = k
    sets = O.subdomain_sets(A, part2, len(sample) + 1, OVERLAP)

    for k, i in enumerate(sample):
        log(f"[sets-scale] subdomain {i}")
        sz, Aii, X = extract_local(dA, part, N, OVERLAP, i)
        s = sets[k]
        assert sz == (s.I.size, s.Gamma.size, s.Delta.size)
        Aii_o, X_o = O.extract(A, s)
        np.testing.assert_array_equal(Aii, Aii_o)
        np.testing.assert_array_equal(X, X_o)


@pytest.mark.parametrize("overlap", [1, 3])
def test_sets_bit_exact_at_overlap(overlap):
    """Gamma_i gathers layers 1..delta (merged and sorted again when delta >= 2): I, Gamma and Delta of every
    subdomain equal the oracle's on a random graph and on a 3-D diffusion problem."""
    from paper_2109_05908_amd import Preconditioner
    for A, N in ((W.random_spd(600, 6, seed=11), 8), (W.diffusion3d(12, seed=2), 12)):
        part = O.ggg_partition(A, N, 0)
        log(f"[sets-scale] n={A.n} N={N} overlap={overlap}")
        pre = Preconditioner(DeviceCSR.from_workload(A), part, N, overlap, 0.1)
        for i, s in enumerate(O.subdomain_sets(A, part, N, overlap)):
            I, G, D = pre.sets(i)
            np.testing.assert_array_equal(I, s.I)
            np.testing.assert_array_equal(G, s.Gamma)
            np.testing.assert_array_equal(D, s.Delta)
