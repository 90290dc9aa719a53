"""Pins for the CPU oracle: checks against what the paper and the mathematics fix.

None of these checks re-types the oracle's own formulas: they use closed forms,
hand-worked rational factors (tests/golden), invariants that characterise the
result uniquely, dense library routines (numpy/scipy/torch) and brute force on
tiny inputs.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(A):
    return synth.csr_to_dense(A)


def dense_pattern_of(an, rp, ci):
    n = an.n
    P = np.zeros((n, n), dtype=bool)
    for r in range(n):
        P[r, ci[rp[r]:rp[r + 1]]] = True
    return P


# --------------------------------------------------------------------------------------
# Hand-worked factors (Sec. III, Fig. 1)
# --------------------------------------------------------------------------------------

def load_cases():
    with open(os.path.join(GOLDEN, "hand_worked.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", load_cases(), ids=lambda c: c["name"])
def test_hand_worked(case):
    n = case["n"]
    rp = np.array(case["row_ptr"], np.int32)
    ci = np.array(case["col_idx"], np.int32)
    val = np.array(case["val"], np.float64)
    an = O.analyze(n, rp, ci, k_max=case["k"], sym=case["sym"])
    assert an.level.tolist() == case["level"]
    assert an.perm.tolist() == case["perm"]
    assert an.lu_ci.tolist() == case["lu_col_idx"]
    f = O.factor(an, val)
    assert f.status == O.OK
    expect = np.array([float(Fraction(s)) for s in case["lu_val"]])
    np.testing.assert_allclose(f.val, expect, rtol=4e-16, atol=0)


# --------------------------------------------------------------------------------------
# Closed forms and special cases of the factor
# --------------------------------------------------------------------------------------

def test_tridiagonal_closed_form():
    # tridiag(-1, 2, -1): exact LU with u_ii = (i+1)/i, l_{i,i-1} = -(i-1)/i (1-based)
    n = 60
    A = synth.tridiag(n)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    assert np.array_equal(an.perm, np.arange(n))          # a chain: one row per level
    assert an.n_levels == n
    f = O.factor(an, A.val)
    Lm, Um = O.dense_factors(an, f.val)
    i = np.arange(1, n + 1, dtype=np.float64)
    np.testing.assert_allclose(np.diag(Um), (i + 1) / i, rtol=1e-14)
    np.testing.assert_allclose(np.diag(Lm, -1), -(i[1:] - 1) / i[1:], rtol=1e-14)
    np.testing.assert_allclose(np.diag(Um, 1), -1.0, rtol=0)


@pytest.mark.parametrize("seed", range(4))
def test_dense_pattern_is_exact_lu(seed):
    # On a full pattern ILU(0) is Gaussian elimination without pivoting; with a
    # column diagonally dominant matrix partial pivoting does not swap, so LAPACK's
    # getrf (scipy.linalg.lu) returns the same factors with P = I.
    rng = np.random.default_rng(seed)
    A = synth.dense_pattern(14, rng)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    assert np.array_equal(an.perm, np.arange(A.n))
    f = O.factor(an, A.val)
    Lm, Um = O.dense_factors(an, f.val)
    P, Lr, Ur = scipy.linalg.lu(dense(A))
    assert np.array_equal(P, np.eye(A.n))
    np.testing.assert_allclose(Lm, Lr, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Um, Ur, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_full_fill_level_is_exact_solve(seed):
    # k >= n-1 admits every fill entry of exact elimination in the input ordering.
    # With the lower(S+S^T) dependency pattern the level order keeps the relative
    # order of every pair joined by an entry of S, so no entry outside P S P^T can
    # fill in and M = A: M^{-1} b = A^{-1} b (numpy.linalg.solve).  (With lower(S)
    # an upper entry of S may turn lower and the factor is not exact.)
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(8, 40))
    A = synth.random_sparse(n, 0.12, rng, symmetric_pattern=bool(seed % 2))
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=n - 1, sym=True)
    f = O.factor(an, A.val)
    assert f.status == O.OK
    b = rng.uniform(-1, 1, n)
    x = O.apply(an, f.val, b)
    xr = np.linalg.solve(dense(A), b)
    np.testing.assert_allclose(x, xr, rtol=1e-10, atol=1e-12 * np.abs(xr).max())


@pytest.mark.parametrize("p", [1, 2, 3])
def test_banded_fill_is_exact(p):
    # A full band of half-width p has no fill outside the band, so ILU(0) is exact.
    rng = np.random.default_rng(p)
    A = synth.banded(30, p, rng)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    b = rng.uniform(-1, 1, A.n)
    np.testing.assert_allclose(O.apply(an, f.val, b), np.linalg.solve(dense(A), b), rtol=1e-11)


def _fixed_pattern_residual(an, A, f):
    """(LU - Atilde) on the permuted pattern, where Atilde is A with 0 on fill."""
    Lm, Um = O.dense_factors(an, f.val)
    D = dense(A)[np.ix_(an.perm, an.perm)]
    Pat = dense_pattern_of(an, an.lu_rp, an.lu_ci)
    return (Lm @ Um - D), Pat, D, Um


@pytest.mark.parametrize("seed", range(12))
def test_fixed_pattern_identity(seed):
    # The up-looking ILU on a fixed pattern S is characterised by (LU)_ij = A_ij for
    # every (i, j) in S (A_ij = 0 on fill): with nonzero pivots it has exactly one
    # solution.  Holds for every k and both dependency patterns.
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(5, 60))
    k = int(seed % 3)
    sym = bool(seed % 2)
    A = synth.random_sparse(n, float(rng.uniform(0.03, 0.2)), rng, symmetric_pattern=bool(seed % 4 == 0))
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k, sym=sym)
    f = O.factor(an, A.val)
    assert f.status == O.OK
    R, Pat, D, _ = _fixed_pattern_residual(an, A, f)
    scale = np.abs(D).max()
    assert np.abs(R[Pat]).max() <= 1e-12 * scale


@pytest.mark.parametrize("seed", range(6))
def test_tau_dropping_bounds(seed):
    # With drops, kept entries still satisfy the identity; a dropped U entry leaves a
    # residual equal to its value (< tau_r), a dropped L entry one equal to its value
    # times the pivot (< tau_r * |u_cc|).
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(10, 50))
    A = synth.random_sparse(n, 0.15, rng)
    tau = float(rng.choice([1e-3, 1e-2, 5e-2]))
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    f = O.factor(an, A.val, k=1, tau=tau)
    assert f.status == O.OK
    R, Pat, D, Um = _fixed_pattern_residual(an, A, f)
    rt = O.row_tau(an, A.val, tau)
    scale = np.abs(D).max()
    kept = np.zeros_like(Pat)
    for r in range(n):
        for p in range(an.lu_rp[r], an.lu_rp[r + 1]):
            c = an.lu_ci[p]
            if f.stat[p] == 0:
                kept[r, c] = True
            elif f.stat[p] == 1:
                if c > r:
                    assert abs(R[r, c]) < rt[r] * (1 + 1e-12) + 1e-14 * scale
                else:
                    assert abs(R[r, c]) < rt[r] * abs(Um[c, c]) * (1 + 1e-12) + 1e-14 * scale
                assert f.val[p] == 0.0
            assert not (c == r and f.stat[p] != 0)   # the diagonal is never dropped
    assert np.abs(R[kept]).max() <= 1e-12 * scale
    assert (f.stat == 1).any() or tau < 1e-2


def load_tau_cases():
    with open(os.path.join(GOLDEN, "tau_norm.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", load_tau_cases(), ids=lambda c: c["name"])
def test_tau_norm_hand_worked(case):
    # tau_r = tau * ||A(row,:)||_2 (reading of Sec. I's ILU(tau)); each case sits where
    # the 1-norm, the infinity norm or a pivot-only test would decide the other way.
    n = case["n"]
    rp = np.array(case["row_ptr"], np.int32)
    ci = np.array(case["col_idx"], np.int32)
    val = np.array(case["val"], np.float64)
    an = O.analyze(n, rp, ci)
    assert an.perm.tolist() == case["perm"]
    f = O.factor(an, val, tau=case["tau"])
    assert f.status == O.OK
    assert f.stat.tolist() == case["state"]
    expect = np.array([float(Fraction(s)) for s in case["lu_val"]])
    np.testing.assert_allclose(f.val, expect, rtol=4e-16, atol=0)


@pytest.mark.parametrize("seed", range(4))
def test_row_tau_is_two_norm_of_the_original_row(seed):
    # the threshold of permuted row r is tau times the Euclidean norm of row perm[r] of A
    # as given (LAPACK's norm, not a sum re-typed here)
    rng = np.random.default_rng(900 + seed)
    A = synth.random_sparse(int(rng.integers(20, 60)), 0.12, rng)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    tau = float(rng.uniform(1e-3, 1e-1))
    expect = tau * np.linalg.norm(dense(A)[an.perm], axis=1)
    np.testing.assert_allclose(O.row_tau(an, A.val, tau), expect, rtol=1e-15, atol=0)


def test_tau_infinite_is_jacobi():
    rng = np.random.default_rng(7)
    A = synth.random_sparse(40, 0.1, rng)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val, tau=1e300)
    b = rng.uniform(-1, 1, A.n)
    np.testing.assert_allclose(O.apply(an, f.val, b), b / np.diag(dense(A)), rtol=1e-15)


def test_lower_triangular_is_exact_integer():
    # ILU(0) of a lower-triangular A is L = A, U = I (no updates reach the upper part),
    # so an integer unit-lower system with integer b is solved exactly.
    rng = np.random.default_rng(11)
    A = synth.integer_unit_lower(50, 0.1, rng)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    b = rng.integers(-3, 4, A.n).astype(np.float64)
    x = O.apply(an, f.val, b)
    assert np.array_equal(np.round(x), x)
    assert np.array_equal(dense(A) @ x, b)


def test_k_restriction_matches_pattern_subset():
    # factor(k=0) on the ILU(1) structure: fill entries are absent (0.0) and the
    # identity holds on the level-0 pattern.
    rng = np.random.default_rng(12)
    A = synth.random_sparse(45, 0.1, rng)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    f = O.factor(an, A.val, k=0)
    absent = an.lu_lev > 0
    assert np.array_equal(f.stat == 2, absent)
    assert np.all(f.val[absent] == 0.0)
    Lm, Um = O.dense_factors(an, f.val)
    D = dense(A)[np.ix_(an.perm, an.perm)]
    Pat0 = np.zeros((A.n, A.n), bool)
    for r in range(A.n):
        for p in range(an.lu_rp[r], an.lu_rp[r + 1]):
            if an.lu_lev[p] == 0:
                Pat0[r, an.lu_ci[p]] = True
    assert np.abs((Lm @ Um - D)[Pat0]).max() <= 1e-12 * np.abs(D).max()


# --------------------------------------------------------------------------------------
# Modified ILU (Sec. I and Sec. III name it; the rule is the textbook one: what a row
# loses goes to its diagonal)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(10))
def test_milu_row_sums_and_offdiagonal_identity(seed):
    # The modified factor is characterised by two facts: every kept off-diagonal
    # entry of LU equals A's (as for plain ILU), and every row sum of LU equals the
    # row sum of A (what is lost is given back on the diagonal).  With tau drops the
    # row sums still hold.  Row by row the two fix L, the off-diagonal U and the
    # diagonal uniquely.
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(8, 60))
    k_max = int(seed % 3)
    k = k_max if seed % 5 else max(k_max - 1, 0)
    tau = 0.0 if seed < 6 else float(rng.choice([1e-3, 1e-2]))
    A = synth.random_sparse(n, float(rng.uniform(0.05, 0.2)), rng, symmetric_pattern=bool(seed % 2))
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k_max, sym=bool(seed % 3 == 0))
    f = O.factor(an, A.val, k=k, tau=tau, milu=True)
    assert f.status == O.OK
    Lm, Um = O.dense_factors(an, f.val)
    D = dense(A)[np.ix_(an.perm, an.perm)]
    LU = Lm @ Um
    scale = np.abs(D).max() * max(1.0, np.abs(LU).max() / np.abs(D).max())
    assert np.abs(LU.sum(axis=1) - D.sum(axis=1)).max() <= 1e-12 * scale * n
    kept_off = np.zeros((n, n), bool)
    for r in range(n):
        for p in range(an.lu_rp[r], an.lu_rp[r + 1]):
            if f.stat[p] == 0 and an.lu_ci[p] != r:
                kept_off[r, an.lu_ci[p]] = True
    assert np.abs((LU - D)[kept_off]).max() <= 1e-12 * scale
    # something was lost, so the diagonal differs from plain ILU's
    g = O.factor(an, A.val, k=k, tau=tau)
    dg = an.diag_pos
    assert not np.array_equal(f.val[dg], g.val[dg]) or np.array_equal(f.val, g.val)


def test_milu_5point_diagonal_recurrence():
    # 5-point Laplacian (4 on the diagonal, -1 to each neighbour), natural ordering:
    # eliminating the south neighbour (i, j-1) loses its east entry (i+1, j-1) and
    # eliminating the west neighbour (i-1, j) loses its north entry (i-1, j+1), each
    # worth (-1/d)(-1), so d_ij = 4 - (1 + [i+1 < nx]) / d_{i,j-1} - (1 + [j+1 < ny]) / d_{i-1,j}.
    # Plain ILU(0) has d_ij = 4 - 1/d_{i,j-1} - 1/d_{i-1,j}.
    nx, ny = 9, 7
    A = synth.laplace2d(nx, ny)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    for milu in (True, False):
        f = O.factor(an, A.val, milu=milu)
        d = np.zeros((nx, ny))
        for j in range(ny):
            for i in range(nx):
                v = 4.0
                if j > 0:
                    v -= (1 + (milu and i + 1 < nx)) / d[i, j - 1]
                if i > 0:
                    v -= (1 + (milu and j + 1 < ny)) / d[i - 1, j]
                d[i, j] = v
        got = f.val[an.diag_pos][an.iperm]       # original row order
        np.testing.assert_allclose(got, d.T.ravel(), rtol=1e-14)


def test_milu_equals_ilu_when_nothing_is_lost():
    # Tridiagonal ILU(0), a dense pattern and a lower-triangular matrix lose no
    # update, so the modified factor is the plain one bit for bit.
    rng = np.random.default_rng(31)
    mats = [synth.tridiag(40), synth.integer_unit_lower(30, 0.2, rng), synth.dense_pattern(12, rng)]
    for A in mats:
        an = O.analyze(A.n, A.row_ptr, A.col_idx)
        f = O.factor(an, A.val, milu=True)
        g = O.factor(an, A.val)
        assert f.status == O.OK and np.array_equal(f.val, g.val)


# --------------------------------------------------------------------------------------
# Reverse Cuthill-McKee preordering (Sec. VII compares orderings; textbook algorithm)
# --------------------------------------------------------------------------------------

def _sym_adj(A):
    D = dense(A) != 0
    G = (D | D.T)
    np.fill_diagonal(G, False)
    return [np.flatnonzero(G[i]) for i in range(A.n)]


def _bandwidth(adj, order):
    pos = np.empty(len(order), np.int64)
    pos[order] = np.arange(len(order))
    return max((abs(pos[i] - pos[j]) for i in range(len(adj)) for j in adj[i]), default=0)


def _bfs_depths(adj, root):
    d = {root: 0}
    frontier = [root]
    while frontier:
        nxt = []
        for u in frontier:
            for w in adj[u]:
                if w not in d:
                    d[w] = d[u] + 1
                    nxt.append(w)
        frontier = nxt
    return d


def _scramble(A, rng):
    p = rng.permutation(A.n)
    D = dense(A)[np.ix_(p, p)]
    r, c = np.nonzero(D)
    return synth.csr_from_coo(A.n, r, c, D[r, c])


def test_rcm_recovers_a_scrambled_path():
    rng = np.random.default_rng(41)
    B = _scramble(synth.tridiag(60), rng)
    order = O.rcm(B.n, B.row_ptr, B.col_idx)
    assert sorted(order) == list(range(B.n))
    assert _bandwidth(_sym_adj(B), order) == 1


@pytest.mark.parametrize("nx,ny", [(7, 11), (12, 5), (9, 9)])
def test_rcm_scrambled_grid_bandwidth(nx, ny):
    # from a corner the visit runs along anti-diagonals of at most min(nx, ny)
    # vertices, so no edge spans more than two of them
    B = _scramble(synth.laplace2d(nx, ny), np.random.default_rng(nx * ny))
    order = O.rcm(B.n, B.row_ptr, B.col_idx)
    adj = _sym_adj(B)
    assert _bandwidth(adj, order) <= 2 * min(nx, ny)
    assert len(adj[order[-1]]) == 2            # the visit starts at a corner


@pytest.mark.parametrize("seed", range(8))
def test_rcm_cuthill_mckee_properties(seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(20, 80))
    A = synth.random_sparse(n, float(rng.uniform(0.01, 0.06)), rng, symmetric_pattern=bool(seed % 2))
    adj = _sym_adj(A)
    deg = np.array([len(a) for a in adj])
    order = O.rcm(A.n, A.row_ptr, A.col_idx)
    assert sorted(order) == list(range(n))
    cm = list(order[::-1])
    pos = {v: i for i, v in enumerate(cm)}
    # components: contiguous, in order of their smallest vertex
    starts, seen_min = [], -1
    i = 0
    while i < n:
        comp = _bfs_depths(adj, cm[i])
        seg = cm[i:i + len(comp)]
        assert set(seg) == set(comp)
        assert min(comp) > seen_min
        seen_min = min(comp)
        starts.append((cm[i], comp))
        i += len(comp)
    for s0, comp in starts:
        # breadth first: every vertex after the start has its first-placed neighbour
        # (its parent) earlier, parents are non-decreasing, and siblings come in
        # (degree, index) order
        seg = sorted(comp, key=lambda v: pos[v])
        par = [min(pos[w] for w in adj[v]) for v in seg[1:]]
        assert all(par[k] < pos[seg[k + 1]] for k in range(len(par)))
        assert all(par[k] <= par[k + 1] for k in range(len(par) - 1))
        for k in range(len(par) - 1):
            if par[k] == par[k + 1]:
                a, b = seg[k + 1], seg[k + 2]
                assert (deg[a], a) < (deg[b], b)
        # the start ends the pseudo-peripheral search: the least-degree vertex of its
        # last level is no deeper, and the start is the search's seed (least degree,
        # smallest index) or deeper than it
        d = _bfs_depths(adj, s0)
        ecc = max(d.values())
        last = [v for v in comp if d[v] == ecc]
        x = min(last, key=lambda v: (deg[v], v))
        assert max(_bfs_depths(adj, x).values()) <= ecc
        m = min(comp, key=lambda v: (deg[v], v))
        assert s0 == m or ecc > max(_bfs_depths(adj, m).values())


def test_rcm_bandwidth_close_to_scipy():
    # a library RCM (different tie rules) as a yardstick on scrambled grids and bands
    import scipy.sparse.csgraph as csg
    rng = np.random.default_rng(77)
    for A in (synth.laplace2d(15, 9), synth.laplace3d(6), synth.banded(80, 3, rng)):
        B = _scramble(A, rng)
        adj = _sym_adj(B)
        ours = _bandwidth(adj, O.rcm(B.n, B.row_ptr, B.col_idx))
        M = scipy.sparse.csr_matrix((np.ones(B.nnz), B.col_idx, B.row_ptr), shape=(B.n, B.n))
        ref = _bandwidth(adj, csg.reverse_cuthill_mckee(M, symmetric_mode=False))
        assert ours <= 1.5 * ref + 1


def test_analyze_with_rcm_is_analysis_of_permuted_matrix():
    # the composed analysis equals the plain analysis of Q A Q^T, and the factor
    # reaches the same values through the composed entry maps
    rng = np.random.default_rng(55)
    A = synth.random_sparse(70, 0.05, rng, symmetric_pattern=True)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1, rcm_order=True)
    q = an.order
    D = dense(A)[np.ix_(q, q)]
    r, c = np.nonzero(D)
    Bq = synth.csr_from_coo(A.n, r, c, D[r, c])
    bn = O.analyze(Bq.n, Bq.row_ptr, Bq.col_idx, k_max=1)
    assert np.array_equal(an.lu_rp, bn.lu_rp) and np.array_equal(an.lu_ci, bn.lu_ci)
    assert np.array_equal(an.perm, q[bn.perm])
    fa = O.factor(an, A.val, tau=1e-3)
    fb = O.factor(bn, Bq.val, tau=1e-3)
    assert np.array_equal(fa.stat, fb.stat)
    np.testing.assert_allclose(fa.val, fb.val, rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------------------
# Errors (no pivoting, Sec. III)
# --------------------------------------------------------------------------------------

def test_zero_pivot_first_row():
    A = synth.csr_from_coo(3, [0, 0, 1, 1, 2, 2], [0, 1, 0, 1, 1, 2], [0.0, 1, 1, 2, 1, 3])
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    assert f.status == O.ERR_ZERO_PIVOT and an.perm[f.bad_row] == 0


def test_zero_pivot_later_row():
    # [[1,1],[1,1]]: u_11 = 1 - 1*1 = 0
    A = synth.csr_from_coo(2, [0, 0, 1, 1], [0, 1, 0, 1], [1.0, 1, 1, 1])
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    assert f.status == O.ERR_ZERO_PIVOT and f.bad_row == 1


def test_nonfinite_value():
    A = synth.laplace2d(4, 4)
    v = A.val.copy()
    v[7] = np.nan
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, v)
    assert f.status == O.ERR_NONFINITE


def test_missing_diagonal_inserted():
    A = synth.csr_from_coo(3, [0, 1, 1, 2], [1, 0, 2, 2], [1.0, 1.0, 2.0, 3.0])
    rp, ci, v, src = O.canonical(A.n, A.row_ptr, A.col_idx, A.val)
    assert rp.tolist() == [0, 2, 5, 6]
    assert ci.tolist() == [0, 1, 0, 1, 2, 2]
    assert v.tolist() == [0.0, 1.0, 1.0, 0.0, 2.0, 3.0]
    assert src.tolist() == [-1, 0, 1, -1, 2, 3]


@pytest.mark.parametrize("bad", ["unsorted", "duplicate", "range", "rowptr"])
def test_invalid_csr(bad):
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    if bad == "unsorted":
        ci = np.array([1, 0, 0, 1], np.int32)
    elif bad == "duplicate":
        ci = np.array([0, 0, 0, 1], np.int32)
    elif bad == "range":
        ci = np.array([0, 2, 0, 1], np.int32)
    else:
        rp = np.array([0, 3, 2], np.int32)
    with pytest.raises(O.OracleError):
        O.canonical(2, rp, ci)


# --------------------------------------------------------------------------------------
# Symbolic ILU(k): level of fill = shortest fill path - 1 (brute force)
# --------------------------------------------------------------------------------------

def brute_fill_levels(D):
    """lev(i,j) = (edges of the shortest path i -> j in the graph of A whose inner
    vertices are all < min(i, j)) - 1; inf when no such path exists."""
    n = D.shape[0]
    adj = [np.nonzero(D[u])[0] for u in range(n)]
    lev = np.full((n, n), np.inf)
    for i in range(n):
        for j in range(n):
            if i == j or D[i, j] != 0:
                lev[i, j] = 0
                continue
            lim = min(i, j)
            dist = {i: 0}
            frontier = [i]
            found = None
            while frontier and found is None:
                nxt = []
                for u in frontier:
                    for v in adj[u]:
                        if v == j:
                            found = dist[u] + 1
                            break
                        if v < lim and v not in dist:
                            dist[v] = dist[u] + 1
                            nxt.append(v)
                    if found is not None:
                        break
                frontier = nxt
            if found is not None:
                lev[i, j] = found - 1
    return lev


@pytest.mark.parametrize("seed", range(6))
def test_symbolic_fill_paths(seed):
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(6, 36))
    A = synth.random_sparse(n, float(rng.uniform(0.05, 0.2)), rng, symmetric_pattern=bool(seed % 2))
    Lb = brute_fill_levels(dense(A) != 0)
    for K in (0, 1, 2, n):
        srp, sci, slev = O.symbolic(n, *O.canonical(n, A.row_ptr, A.col_idx)[:2], K)
        got = np.full((n, n), np.inf)
        for i in range(n):
            got[i, sci[srp[i]:srp[i + 1]]] = slev[srp[i]:srp[i + 1]]
        want = np.where(Lb <= K, Lb, np.inf)
        assert np.array_equal(got, want), (K, np.argwhere(got != want)[:5])


def test_ilu1_5point_fill_diagonals():
    # 5-point ILU(1) adds exactly the diagonals +-(nx-1) (entries (i+1, j-1), (i-1, j+1))
    nx = ny = 9
    A = synth.laplace2d(nx, ny)
    srp, sci, slev = O.symbolic(A.n, A.row_ptr, A.col_idx, 1)
    rows = np.repeat(np.arange(A.n), np.diff(srp))
    fill = slev > 0
    assert set(np.abs(sci[fill] - rows[fill]).tolist()) == {nx - 1}
    # count: (nx-1)*(ny-1) in each of the two diagonals
    assert fill.sum() == 2 * (nx - 1) * (ny - 1)


@pytest.mark.parametrize("m", [5, 12])
def test_ilu1_7point_count(m):
    A = synth.laplace3d(m)
    srp, sci, slev = O.symbolic(A.n, A.row_ptr, A.col_idx, 1)
    assert srp[-1] == m**3 + 6 * m * m * (m - 1) + 6 * m * (m - 1) ** 2


# --------------------------------------------------------------------------------------
# Level sets (Sec. II, Sec. III) and the permutation
# --------------------------------------------------------------------------------------

def check_level_characterisation(n, rp, ci, level, sym):
    deps = [set() for _ in range(n)]
    for i in range(n):
        for j in ci[rp[i]:rp[i + 1]]:
            if j < i:
                deps[i].add(int(j))
            elif j > i and sym:
                deps[int(j)].add(i)
    for i in range(n):
        # (i) every dependency sits in a strictly earlier level
        assert all(level[j] < level[i] for j in deps[i])
        # (ii) a row above level 0 has a dependency exactly one level below
        if level[i] > 0:
            assert any(level[j] == level[i] - 1 for j in deps[i])
        else:
            assert not deps[i]


@pytest.mark.parametrize("seed", range(8))
def test_levels_characterisation(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(10, 120))
    A = synth.random_sparse(n, float(rng.uniform(0.01, 0.08)), rng)
    sym = bool(seed % 2)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=seed % 3, sym=sym)
    check_level_characterisation(n, an.s_rp, an.s_ci, an.level, sym)
    # permutation: stable sort by (level, index) -- numpy's stable argsort
    assert np.array_equal(an.perm, np.argsort(an.level, kind="stable"))
    assert np.array_equal(an.iperm[an.perm], np.arange(n))
    assert np.array_equal(an.level_ptr, np.concatenate([[0], np.cumsum(np.bincount(an.level))]))
    # every strictly lower entry of P S P^T points to an earlier level
    lv = an.level[an.perm]
    for r in range(n):
        for c in an.lu_ci[an.lu_rp[r]:an.lu_rp[r + 1]]:
            if c < r:
                assert lv[c] < lv[r]


def test_level_closed_forms():
    with open(os.path.join(GOLDEN, "level_stats.json")) as f:
        G = json.load(f)
    A = synth.laplace2d(64)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    i, j = np.meshgrid(np.arange(64), np.arange(64), indexing="xy")
    assert np.array_equal(an.level, (i + j).ravel())
    s = an.level_stats()
    g = G["laplace2d_64"]
    assert (s["levels"], s["min"], s["max"], s["median"]) == (g["levels"], g["min"], g["max"], g["median"])
    A = synth.laplace3d(10, 11, 12)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    k, j, i = np.meshgrid(np.arange(12), np.arange(11), np.arange(10), indexing="ij")
    assert np.array_equal(an.level, (i + j + k).ravel())
    an1 = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    assert np.array_equal(an1.level, (i + 2 * j + 3 * k).ravel())


@pytest.mark.slow
def test_level_stats_full_size():
    with open(os.path.join(GOLDEN, "level_stats.json")) as f:
        G = json.load(f)
    A, _ = synth.workload(2)
    s = O.analyze(A.n, A.row_ptr, A.col_idx).level_stats()
    g = G["laplace3d_128"]
    assert (s["levels"], s["min"], s["max"], s["median"]) == (g["levels"], g["min"], g["max"], g["median"])
    A, _ = synth.workload(3)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    s = an.level_stats()
    g = G["convdiff3d_96_ilu1"]
    assert (s["levels"], s["min"], s["max"], s["median"]) == (g["levels"], g["min"], g["max"], g["median"])
    assert an.nnz_lu == g["nnz_lu"]


@pytest.mark.parametrize("seed", range(4))
def test_permuted_structure_and_upper_schedule(seed):
    rng = np.random.default_rng(600 + seed)
    n = int(rng.integers(10, 60))
    A = synth.random_sparse(n, 0.08, rng, drop_diag_frac=0.2 if seed % 2 else 0.0)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=seed % 2, sym=bool(seed % 2))
    Sd = np.zeros((n, n), bool)
    for i in range(n):
        Sd[i, an.s_ci[an.s_rp[i]:an.s_rp[i + 1]]] = True
    # P S P^T as a dense boolean permutation
    assert np.array_equal(dense_pattern_of(an, an.lu_rp, an.lu_ci), Sd[np.ix_(an.perm, an.perm)])
    # factor values before factorisation: A on its pattern, 0 on fill and inserted diagonals
    D = dense(A)[np.ix_(an.perm, an.perm)]
    v0 = O.gather(an.lu_src, A.val)
    for r in range(n):
        for p in range(an.lu_rp[r], an.lu_rp[r + 1]):
            assert v0[p] == D[r, an.lu_ci[p]]
        assert an.lu_ci[an.diag_pos[r]] == r
    # permuted copy of A for spmv
    vb = O.b_values(an, A.val)
    Bd = np.zeros((n, n))
    for r in range(n):
        Bd[r, an.b_ci[an.b_rp[r]:an.b_rp[r + 1]]] = vb[an.b_rp[r]:an.b_rp[r + 1]]
    assert np.array_equal(Bd, D)
    # upper schedule: each upper dependency is in an earlier upper level, maximal
    ul = an.ulev
    for r in range(n):
        ups = [c for c in an.lu_ci[an.lu_rp[r]:an.lu_rp[r + 1]] if c > r]
        assert all(ul[c] < ul[r] for c in ups)
        assert (ul[r] == 0) == (not ups) and (not ups or max(ul[c] for c in ups) == ul[r] - 1)
    assert np.array_equal(an.ulevel_rows, np.argsort(ul, kind="stable"))


# --------------------------------------------------------------------------------------
# Apply, spmv, casts (Sec. VI)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_apply_dense_triangular(seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(5, 64))
    A = synth.random_sparse(n, 0.1, rng)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=seed % 2)
    f = O.factor(an, A.val)
    Lm, Um = O.dense_factors(an, f.val)
    nrhs = 1 + seed % 3
    b = rng.uniform(-1, 1, (n, nrhs)) if nrhs > 1 else rng.uniform(-1, 1, n)
    x, y = O.apply(an, f.val, b, want_y=True)
    bp = b[an.perm]
    yr = scipy.linalg.solve_triangular(Lm, bp, lower=True, unit_diagonal=True)
    zr = scipy.linalg.solve_triangular(Um, yr, lower=False)
    xr = np.empty_like(zr)
    xr[an.perm] = zr
    np.testing.assert_allclose(y, yr, rtol=1e-12, atol=1e-13 * np.abs(yr).max())
    np.testing.assert_allclose(x, xr, rtol=1e-12, atol=1e-13 * np.abs(xr).max())
    # permuted-space variant
    np.testing.assert_allclose(O.apply(an, f.val, bp, permuted=True), zr, rtol=1e-12,
                               atol=1e-13 * np.abs(zr).max())


def test_apply_lowp_bounds():
    # FP32 and BF16 factors: the result is close to the FP64 apply of the rounded
    # factor (FP32 arithmetic error only) -- checked against the dense solve.
    rng = np.random.default_rng(9)
    A = synth.laplace2d(12)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    b = rng.uniform(-1, 1, A.n)
    for prec, caster, widen in (("f32", O.cast_f32, lambda v: v.astype(np.float64)),
                                ("bf16", O.cast_bf16,
                                 lambda v: (v.astype(np.uint32) << 16).view(np.float32).astype(np.float64))):
        low = caster(f.val)
        x = O.apply(an, low, b, prec=prec)
        xr = O.apply(an, widen(low), b)
        assert np.abs(x - xr).max() <= 1e-5 * np.abs(xr).max()


def _exact_vec(strs, shape):
    return np.array([float(Fraction(s)) for s in strs], np.float64).reshape(shape)


def load_lowp_cases():
    with open(os.path.join(GOLDEN, "lowp_apply.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("case", load_lowp_cases(), ids=lambda c: c["name"])
def test_apply_lowp_hand_worked(case, prec):
    # FP32 arithmetic in ascending column order and a true FP32 division, bit for bit
    n, nrhs = case["n"], case["nrhs"]
    val = np.array([float(Fraction(s)) for s in case["val"]])
    an = O.analyze(n, np.array(case["row_ptr"], np.int32), np.array(case["col_idx"], np.int32))
    f = O.factor(an, val)
    assert f.status == O.OK
    low = O.cast_f32(f.val) if prec == "f32" else O.cast_bf16(f.val)
    b = _exact_vec(case["b"], (n, nrhs))
    x = O.apply(an, low, b if nrhs > 1 else b[:, 0], prec=prec).reshape(n, nrhs)
    expect = _exact_vec(case["x_f32"], (n, nrhs))
    assert np.array_equal(x.view(np.uint64), expect.view(np.uint64)), (x, expect)
    if "x_f64" in case:
        x64 = O.apply(an, f.val, b if nrhs > 1 else b[:, 0]).reshape(n, nrhs)
        assert np.array_equal(x64, _exact_vec(case["x_f64"], (n, nrhs)))
        assert not np.array_equal(x64, x)   # the case separates FP32 from FP64 arithmetic


def _serial_f32_apply(an, low32, b):
    # textbook forward and back substitution on numpy float32 scalars (every product,
    # sum and division rounded to FP32), columns ascending, in the level ordering
    n = an.n
    f = np.float32
    y = [f(0)] * n
    z = [f(0)] * n
    bp = b[an.perm]
    for r in range(n):
        acc = f(0)
        for p in range(an.lu_rp[r], an.diag_pos[r]):
            acc = f(acc + f(low32[p] * y[an.lu_ci[p]]))
        y[r] = f(f(bp[r]) - acc)
    for r in range(n - 1, -1, -1):
        acc = f(0)
        for p in range(an.diag_pos[r] + 1, an.lu_rp[r + 1]):
            acc = f(acc + f(low32[p] * z[an.lu_ci[p]]))
        z[r] = f(f(y[r] - acc) / low32[an.diag_pos[r]])
    x = np.empty(n, np.float64)
    x[an.perm] = np.array(z, np.float32).astype(np.float64)
    return x


@pytest.mark.parametrize("seed", range(4))
def test_apply_lowp_serial_float32(seed):
    # n <= 64: the oracle's FP32/BF16 apply equals a serial numpy.float32 substitution
    # bit for bit, on inputs with wide value ranges where FP32 and FP64 arithmetic
    # give visibly different results
    rng = np.random.default_rng(950 + seed)
    n = int(rng.integers(20, 65))
    A = synth.random_sparse(n, 0.15, rng)
    A.val[:] = A.val * np.exp(rng.uniform(-6, 6, A.nnz))
    for i in range(n):   # keep it factorable: dominant diagonal
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        d = s + int(np.searchsorted(A.col_idx[s:e], i))
        A.val[d] = 1.5 * np.abs(A.val[s:e]).sum() + 1.0
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    assert f.status == O.OK
    b = rng.uniform(-1, 1, n) * np.exp(rng.uniform(-8, 8, n))
    for prec in ("f32", "bf16"):
        low = O.cast_f32(f.val) if prec == "f32" else O.cast_bf16(f.val)
        w32 = low if prec == "f32" else (low.astype(np.uint32) << 16).view(np.float32)
        x = O.apply(an, low, b, prec=prec)
        xr = _serial_f32_apply(an, w32, b)
        assert np.array_equal(x.view(np.uint64), xr.view(np.uint64))
        x64 = O.apply(an, w32.astype(np.float64), b)
        assert np.abs(x64 - x).max() > 0.0   # FP64 arithmetic would be told apart


def test_spmv_library_and_integer_exact():
    rng = np.random.default_rng(13)
    A = synth.random_sparse(80, 0.05, rng)
    x = rng.uniform(-1, 1, (80, 3))
    y = O.spmv(A.n, A.row_ptr, A.col_idx, A.val, x)
    S = scipy.sparse.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(80, 80))
    np.testing.assert_allclose(y, S @ x, rtol=1e-14, atol=1e-14)
    Ai = rng.integers(-5, 6, A.nnz).astype(np.float64)
    xi = rng.integers(-5, 6, 80).astype(np.float64)
    assert np.array_equal(O.spmv(A.n, A.row_ptr, A.col_idx, Ai, xi), dense(synth.CSR(80, A.row_ptr, A.col_idx, Ai)) @ xi)


def test_casts_against_library_rounding():
    import torch
    rng = np.random.default_rng(14)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-40, 40, 4000),
                        [0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45, 3.4e38, 3.5e38, 1.0 + 2**-8,
                         1.0 + 3 * 2**-9, 1.0 + 2**-9, -(1.0 + 2**-9)]])
    f32 = O.cast_f32(x)
    assert np.array_equal(f32.view(np.uint32), x.astype(np.float32).view(np.uint32))
    bf = O.cast_bf16(x)
    tb = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    nan = np.isnan(x)
    assert np.array_equal(bf[~nan], tb[~nan])
    assert np.all(((bf[nan] >> 7) & 0xFF) == 0xFF) and np.all((bf[nan] & 0x7F) != 0)


# --------------------------------------------------------------------------------------
# Krylov consumers
# --------------------------------------------------------------------------------------

def test_pcg_exact_preconditioner_one_iteration():
    rng = np.random.default_rng(15)
    A = synth.laplace2d(6)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=A.n)
    f = O.factor(an, A.val)
    b = rng.uniform(-1, 1, A.n)
    x, it, rr, st = O.pcg(an, O.b_values(an, A.val), f.val, b)
    assert st == O.OK and it == 1 and rr <= 1e-10


def test_pcg_laplace2d_against_scipy():
    A, b = synth.workload(1)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    x, it, rr, st = O.pcg(an, O.b_values(an, A.val), f.val, b)
    assert st == O.OK and rr <= 1e-10
    S = scipy.sparse.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    np.testing.assert_allclose(x, scipy.sparse.linalg.spsolve(S.tocsc(), b), rtol=0, atol=1e-8)
    # scipy's PCG with the same preconditioner converges in the same number of steps (+-2)
    M = scipy.sparse.linalg.LinearOperator((A.n, A.n), matvec=lambda v: O.apply(an, f.val, v))
    count = [0]
    scipy.sparse.linalg.cg(S, b, rtol=1e-10, atol=0.0, M=M, maxiter=1000,
                           callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert abs(count[0] - it) <= 2, (count[0], it)


def test_fgmres_exact_and_convdiff():
    rng = np.random.default_rng(16)
    A = synth.convdiff3d(5)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=A.n)
    f = O.factor(an, A.val)
    b = rng.uniform(-1, 1, A.n)
    x, it, rr, st = O.fgmres(an, O.b_values(an, A.val), f.val, b)
    assert st == O.OK and it == 1 and rr <= 1e-10
    A = synth.convdiff3d(10)
    b = rng.uniform(-1, 1, A.n)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    f = O.factor(an, A.val, tau=1e-3)
    for prec in ("f64", "f32", "bf16"):
        low = None if prec == "f64" else (O.cast_f32(f.val) if prec == "f32" else O.cast_bf16(f.val))
        x, it, rr, st = O.fgmres(an, O.b_values(an, A.val), f.val, b, prec=prec, lu_low=low, restart=30)
        assert st == O.OK and rr <= 1e-10
        np.testing.assert_allclose(x, np.linalg.solve(dense(A), b), rtol=0, atol=1e-8)


# --------------------------------------------------------------------------------------
# Adjoint: finite differences and dense autograd
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_adjoint_finite_differences_and_autograd(seed):
    import torch
    rng = np.random.default_rng(800 + seed)
    n = int(rng.integers(10, 40))
    A = synth.random_sparse(n, 0.12, rng)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=seed % 2)
    f = O.factor(an, A.val)
    nrhs = 1 + seed
    b = rng.uniform(-1, 1, (n, nrhs))
    c = rng.uniform(-1, 1, (n, nrhs))      # loss = sum(c * x)
    x, y = O.apply(an, f.val, b, want_y=True)
    gb, glu = O.adjoint(an, f.val, c, x, y)

    def loss(lu, bb):
        return float(np.sum(c * O.apply(an, lu, bb)))

    h = 1e-6
    for _ in range(3):
        vb = rng.standard_normal(b.shape)
        fd = (loss(f.val, b + h * vb) - loss(f.val, b - h * vb)) / (2 * h)
        assert abs(fd - np.sum(gb * vb)) <= 1e-6 * max(1.0, abs(fd))
        vl = rng.standard_normal(f.val.shape)
        fd = (loss(f.val + h * vl, b) - loss(f.val - h * vl, b)) / (2 * h)
        assert abs(fd - np.dot(glu, vl)) <= 1e-6 * max(1.0, abs(fd))

    # dense FP64 autograd through triangular solves, gradients restricted to the pattern
    Lm, Um = O.dense_factors(an, f.val)
    Lt = torch.tensor(Lm, dtype=torch.float64, requires_grad=True)
    Ut = torch.tensor(Um, dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(b, dtype=torch.float64, requires_grad=True)
    P = torch.tensor(an.perm, dtype=torch.long)
    yt = torch.linalg.solve_triangular(Lt, bt[P], upper=False, unitriangular=True)
    zt = torch.linalg.solve_triangular(Ut, yt, upper=True)
    xt = torch.empty_like(zt)
    xt = xt.index_copy(0, P, zt)
    (xt * torch.tensor(c)).sum().backward()
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-10, atol=1e-12)
    gL, gU = Lt.grad.numpy(), Ut.grad.numpy()
    for r in range(n):
        for p in range(an.lu_rp[r], an.lu_rp[r + 1]):
            col = an.lu_ci[p]
            want = gL[r, col] if col < r else gU[r, col]
            assert abs(glu[p] - want) <= 1e-10 * max(1.0, abs(want))
