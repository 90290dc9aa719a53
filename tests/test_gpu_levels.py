"""Level sets computed on the device (ilu_levels_device) against the oracle's
level schedule (Sec. II peeling of lower(S) or lower(S + S^T)): perm and the level
pointers bit for bit, on small structured and random patterns, degenerate cases
(one row, no dependencies, one long chain), ILU(1) fill patterns, both dependency
patterns, the full-size 128^3 Laplacian and random_1m, and the CSR errors; and the
upper pattern against the backward schedule of the permuted factor pattern and the
oracle's upper levels."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).cuda()


def run_pattern(jv, rp, ci, pattern):
    lp, perm, ip = jv.levels_device(dev(rp), dev(ci), pattern)
    return lp.cpu().numpy(), perm.cpu().numpy(), ip.cpu().numpy()


def run(jv, n, rp, ci, sym=True):
    return run_pattern(jv, rp, ci, "sym" if sym else "lower")


def check(jv, n, rp, ci, sym=True, k_max=0):
    an = O.analyze(n, rp, ci, k_max=k_max, sym=sym)
    srp, sci = (rp, ci) if k_max == 0 else (an.s_rp, an.s_ci)
    lp, perm, ip = run(jv, n, srp, sci, sym)
    np.testing.assert_array_equal(lp, an.level_ptr)
    np.testing.assert_array_equal(perm, an.perm)
    np.testing.assert_array_equal(ip, an.iperm)
    return an


CASES = {
    "laplace2d_64": lambda: synth.laplace2d(64),
    "laplace3d_20": lambda: synth.laplace3d(20),
    "convdiff3d_12": lambda: synth.convdiff3d(12),
    "random_nonsym": lambda: synth.random_sparse(3000, 2e-3, np.random.default_rng(7)),
    "random_missing_diag": lambda: synth.random_sparse(2500, 1.5e-3, np.random.default_rng(8), drop_diag_frac=0.3),
    "heavy_rows": lambda: synth.heavy_rows(4000, heavy_len=(64, 300), rng=np.random.default_rng(9)),
}


@pytest.mark.parametrize("sym", [True, False], ids=["lower_sym", "lower_a"])
@pytest.mark.parametrize("name", list(CASES))
def test_levels_match_oracle(jv, name, sym):
    A = CASES[name]()
    check(jv, A.n, A.row_ptr, A.col_idx, sym=sym)


@pytest.mark.parametrize("sym", [True, False], ids=["lower_sym", "lower_a"])
def test_levels_ilu1_pattern(jv, sym):
    A = synth.convdiff3d(10)
    check(jv, A.n, A.row_ptr, A.col_idx, sym=sym, k_max=1)
    B = synth.random_sparse(1500, 3e-3, np.random.default_rng(3))
    check(jv, B.n, B.row_ptr, B.col_idx, sym=sym, k_max=2)


def test_levels_degenerate(jv):
    # one row without entries
    lp, perm, ip = run(jv, 1, np.array([0, 0]), np.array([], np.int32))
    assert lp.tolist() == [0, 1] and perm.tolist() == [0] and ip.tolist() == [0]
    # diagonal only: a single level in input order
    n = 1000
    lp, perm, _ = run(jv, n, np.arange(n + 1), np.arange(n))
    assert lp.tolist() == [0, n] and perm.tolist() == list(range(n))
    # lower bidiagonal: one level per row, across many claimed blocks
    n = 3000
    rp = np.concatenate([[0, 1], 1 + 2 * np.arange(1, n)])
    ci = np.concatenate([[0], np.stack([np.arange(n - 1), np.arange(1, n)], 1).ravel()])
    lp, perm, _ = run(jv, n, rp, ci)
    np.testing.assert_array_equal(lp, np.arange(n + 1))
    # upper entries only: one level under lower(A), a chain under lower(A + A^T)
    rp = np.minimum(np.arange(n + 1), n - 1)
    ci = np.arange(1, n)
    lp, _, _ = run(jv, n, rp, ci, sym=False)
    assert lp.tolist() == [0, n]
    lp, _, _ = run(jv, n, rp, ci, sym=True)
    np.testing.assert_array_equal(lp, np.arange(n + 1))
    check(jv, n, rp, ci, sym=True)


def test_levels_csr_errors(jv):
    A = synth.laplace2d(8)
    bad = []
    ci = A.col_idx.copy()
    ci[[3, 4]] = ci[[4, 3]]                                     # unsorted row
    bad.append((A.row_ptr, ci))
    ci = A.col_idx.copy()
    ci[5] = ci[4]                                               # repeated column
    bad.append((A.row_ptr, ci))
    ci = A.col_idx.copy()
    ci[-1] = A.n                                                # out of range
    bad.append((A.row_ptr, ci))
    rp = A.row_ptr.copy()
    rp[10], rp[11] = rp[11], rp[10]                             # not monotone
    bad.append((rp, A.col_idx))
    rp = A.row_ptr.copy()
    rp[-1] -= 1                                                 # does not end at nnz
    bad.append((rp, A.col_idx))
    for rp, ci in bad:
        with pytest.raises(jv.IluError) as e:
            run(jv, A.n, rp, ci)
        assert e.value.status == "ILU_ERR_CSR"
    # a good call afterwards still matches
    check(jv, A.n, A.row_ptr, A.col_idx)


@pytest.mark.slow
def test_levels_laplace3d_128_full(jv):
    A, _ = synth.workload(2)
    an = check(jv, A.n, A.row_ptr, A.col_idx)
    assert an.n_levels == 382


@pytest.mark.slow
@pytest.mark.parametrize("sym", [True, False], ids=["lower_sym", "lower_a"])
def test_levels_random_1m_full(jv, sym):
    A, _ = synth.workload(4)
    check(jv, A.n, A.row_ptr, A.col_idx, sym=sym)


UPPER_CASES = ["laplace2d_64", "convdiff3d_12", "random_nonsym", "random_missing_diag", "heavy_rows"]


@pytest.mark.parametrize("name", UPPER_CASES)
def test_upper_levels_match_backward_schedule(jv, name):
    # the backward schedule of the permuted factor pattern, and the upper levels
    # of the input pattern as given
    A = CASES[name]()
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    lp, perm, ip = run_pattern(jv, an.lu_rp, an.lu_ci, "upper")
    np.testing.assert_array_equal(lp, an.ulevel_ptr)
    np.testing.assert_array_equal(perm, an.ulevel_rows)
    ulev, nul = O.upper_levels(A.n, A.row_ptr.astype(np.int32), A.col_idx.astype(np.int32))
    rperm, riperm, rptr = O.sort_by_key(ulev, nul)
    lp, perm, ip = run_pattern(jv, A.row_ptr, A.col_idx, "upper")
    np.testing.assert_array_equal(lp, rptr)
    np.testing.assert_array_equal(perm, rperm)
    np.testing.assert_array_equal(ip, riperm)


def test_upper_levels_chain_and_ilu1(jv):
    # upper bidiagonal: one level per row, the last row first
    n = 3000
    rp = np.concatenate([2 * np.arange(n), [2 * n - 1]])
    ci = np.concatenate([np.stack([np.arange(n - 1), np.arange(1, n)], 1).ravel(), [n - 1]])
    lp, perm, _ = run_pattern(jv, rp, ci, "upper")
    np.testing.assert_array_equal(lp, np.arange(n + 1))
    np.testing.assert_array_equal(perm, np.arange(n)[::-1])
    A = synth.convdiff3d(10)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    lp, perm, _ = run_pattern(jv, an.lu_rp, an.lu_ci, "upper")
    np.testing.assert_array_equal(lp, an.ulevel_ptr)
    np.testing.assert_array_equal(perm, an.ulevel_rows)


@pytest.mark.slow
def test_upper_levels_random_1m_full(jv):
    A, _ = synth.workload(4)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    lp, perm, _ = run_pattern(jv, an.lu_rp, an.lu_ci, "upper")
    np.testing.assert_array_equal(lp, an.ulevel_ptr)
    np.testing.assert_array_equal(perm, an.ulevel_rows)


def dev_perm(an):
    return dev(an.perm), dev(an.iperm)


def check_permute(jv, an, k0_src=True):
    p, ip = dev_perm(an)
    orp, oci, src, dp = [t.cpu().numpy() for t in jv.permute_device(dev(an.s_rp), dev(an.s_ci), p, ip)]
    np.testing.assert_array_equal(orp, an.lu_rp)
    np.testing.assert_array_equal(oci, an.lu_ci)
    np.testing.assert_array_equal(dp, an.diag_pos)
    if k0_src:
        # S is the canonical A: its entry map to A's input entries gives the factor's
        np.testing.assert_array_equal(np.asarray(an.a_src)[src], an.lu_src)


@pytest.mark.parametrize("name", list(CASES))
def test_permute_matches_oracle(jv, name):
    A = CASES[name]()
    check_permute(jv, O.analyze(A.n, A.row_ptr, A.col_idx))


def test_permute_fill_patterns_and_errors(jv):
    A = synth.convdiff3d(10)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    check_permute(jv, an, k0_src=False)
    # the level-ordered copy of A for spmv: the same call on A's canonical pattern
    p, ip = dev_perm(an)
    orp, oci, src, _ = [t.cpu().numpy() for t in jv.permute_device(dev(an.a_rp), dev(an.a_ci), p, ip)]
    np.testing.assert_array_equal(orp, an.b_rp)
    np.testing.assert_array_equal(oci, an.b_ci)
    np.testing.assert_array_equal(np.asarray(an.a_src)[src], an.b_src)
    B = synth.random_sparse(1500, 3e-3, np.random.default_rng(3))
    check_permute(jv, O.analyze(B.n, B.row_ptr, B.col_idx, k_max=2, sym=False), k0_src=False)
    # identity permutation on a pattern without some diagonals: diag_pos -1 there
    C = synth.random_sparse(800, 4e-3, np.random.default_rng(5), drop_diag_frac=0.5)
    ident = dev(np.arange(C.n))
    orp, oci, _, dp = [t.cpu().numpy() for t in jv.permute_device(dev(C.row_ptr), dev(C.col_idx), ident, ident)]
    np.testing.assert_array_equal(orp, C.row_ptr)
    np.testing.assert_array_equal(oci, C.col_idx)
    for r in range(C.n):
        cols = C.col_idx[C.row_ptr[r]:C.row_ptr[r + 1]]
        assert dp[r] == (C.row_ptr[r] + int(np.searchsorted(cols, r)) if r in cols else -1)
    # a perm that is not a permutation, and an iperm that is not its inverse
    bad = np.arange(C.n)
    bad[3] = 4
    with pytest.raises(jv.IluError) as e:
        jv.permute_device(dev(C.row_ptr), dev(C.col_idx), dev(bad), ident)
    assert e.value.status == "ILU_ERR_ARG"
    ci = C.col_idx.copy()
    ci[-1] = C.n
    with pytest.raises(jv.IluError) as e:
        jv.permute_device(dev(C.row_ptr), dev(ci), ident, ident)
    assert e.value.status == "ILU_ERR_CSR"


@pytest.mark.slow
@pytest.mark.parametrize("wid", [2, 4])
def test_device_schedule_pipeline_full(jv, wid):
    # levels, permuted factor pattern and backward schedule all on the device,
    # against the oracle's analysis (128^3 Laplacian, random_1m)
    A, _ = synth.workload(wid)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    srp, sci = dev(an.s_rp), dev(an.s_ci)
    lp, perm, iperm = jv.levels_device(srp, sci, "sym")
    np.testing.assert_array_equal(lp.cpu().numpy(), an.level_ptr)
    orp, oci, src, dp = jv.permute_device(srp, sci, perm, iperm)
    np.testing.assert_array_equal(orp.cpu().numpy(), an.lu_rp)
    np.testing.assert_array_equal(oci.cpu().numpy(), an.lu_ci)
    np.testing.assert_array_equal(dp.cpu().numpy(), an.diag_pos)
    np.testing.assert_array_equal(np.asarray(an.a_src)[src.cpu().numpy()], an.lu_src)
    ulp, urows, _ = jv.levels_device(orp, oci, "upper")
    np.testing.assert_array_equal(ulp.cpu().numpy(), an.ulevel_ptr)
    np.testing.assert_array_equal(urows.cpu().numpy(), an.ulevel_rows)


def check_transpose(jv, rp, ci):
    # the transpose of a pattern is unique: scipy's CSR transpose with sorted
    # columns, the entry map carried as the values
    import scipy.sparse as sp
    n = len(rp) - 1
    M = sp.csr_matrix((np.arange(1, len(ci) + 1, dtype=np.int64), np.asarray(ci), np.asarray(rp)), shape=(n, n))
    T = M.T.tocsr()
    T.sort_indices()
    trp, tci, tmap, tdg = [t.cpu().numpy() for t in jv.transpose_device(dev(rp), dev(ci))]
    np.testing.assert_array_equal(trp, T.indptr)
    np.testing.assert_array_equal(tci, T.indices)
    np.testing.assert_array_equal(tmap, T.data - 1)
    rows = np.repeat(np.arange(n), np.diff(trp))
    np.testing.assert_array_equal(np.asarray(ci)[tmap], rows)   # entry q of row j came from column j
    want = np.full(n, -1)
    hit = tci == rows
    want[rows[hit]] = np.nonzero(hit)[0]
    np.testing.assert_array_equal(tdg, want)


@pytest.mark.parametrize("name", ["laplace2d_64", "convdiff3d_12", "random_nonsym", "random_missing_diag",
                                  "heavy_rows"])
def test_transpose_matches_definition(jv, name):
    A = CASES[name]()
    check_transpose(jv, A.row_ptr, A.col_idx)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    check_transpose(jv, an.lu_rp, an.lu_ci)


def test_transpose_degenerate_and_errors(jv):
    check_transpose(jv, np.array([0, 0]), np.array([], np.int32))
    n = 500
    check_transpose(jv, np.minimum(np.arange(n + 1), n - 1), np.arange(1, n))   # upper shift only
    A = synth.laplace2d(8)
    ci = A.col_idx.copy()
    ci[[3, 4]] = ci[[4, 3]]
    with pytest.raises(jv.IluError) as e:
        jv.transpose_device(dev(A.row_ptr), dev(ci))
    assert e.value.status == "ILU_ERR_CSR"


@pytest.mark.slow
def test_transpose_random_1m_full(jv):
    A, _ = synth.workload(4)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    check_transpose(jv, an.lu_rp, an.lu_ci)
