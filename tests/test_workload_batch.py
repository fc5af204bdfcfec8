"""The many-systems workload's generator (CPU): a seeded plan of sizes in the
stated range with the three kinds in turn, and systems of about the planned
size that are symmetric with a positive diagonal."""
import numpy as np
import scipy.sparse as sp

import workloads as W


def test_plan_is_seeded_in_range_and_rotates_kinds():
    p1, p2 = W.batch_plan(64), W.batch_plan(64)
    assert p1 == p2 and len(p1) == 64
    sizes = np.array([n for _, n, _ in p1])
    assert sizes.min() >= 2e4 and sizes.max() <= 5e5
    assert [k for k, _, _ in p1[:6]] == list(W.C5_KINDS) * 2
    assert len({sd for _, _, sd in p1}) == 64
    assert W.batch_plan(64, seed=1) != p1


def test_systems_match_their_planned_size_and_are_symmetric():
    for kind in W.C5_KINDS:
        for target in (2e4, 6e4):
            A = W.batch_system(kind, target, seed=5)
            assert 0.8 * target <= A.n <= 1.2 * target, (kind, target, A.n)
            M = sp.csr_matrix((A.val, A.colind, A.rowptr), shape=(A.n, A.n))
            assert abs(M - M.T).max() <= 1e-12 * abs(M).max()
            assert (M.diagonal() > 0).all()
