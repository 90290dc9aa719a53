"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: schedules, permutation, pattern and drop state bit-exact; factor values
bit-exact (expected; the contract is 1e-12 relative); FP64 solves and spmv within
1e-12 relative (inf-norm per right-hand side); integer-valued inputs bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

SCHEDS = [("level", "level"), ("syncfree", "syncfree")]
# solve schedules: the factor schedule is irrelevant to the apply; the tiled solve
# is built with small tiles so that test matrices span several tiles (ragged last)
SOLVE_SCHEDS = SCHEDS + [("syncfree", "tiled")]
# factor schedules: the tiled factor covers ILU(k, tau) and modified ILU(k, tau) with
# k = k_max and rows of at most 32 entries, and falls back to the sync-free factor otherwise
FACTOR_SCHEDS = SCHEDS + [("tiled", "tiled")]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def relerr(x, ref):
    x = np.asarray(x).reshape(len(x), -1)
    ref = np.asarray(ref).reshape(len(ref), -1)
    return float(max(np.abs(x[:, s] - ref[:, s]).max() / max(np.abs(ref[:, s]).max(), 1e-300)
                     for s in range(ref.shape[1])))


def make(jv, A, k_max=0, sym=True, sched=("syncfree", "syncfree"), tile_rows=256):
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k_max, pattern="sym" if sym else "a", tile_rows=tile_rows)
    ilu.set_schedule(*sched)
    return ilu


CASES = [
    ("laplace2d_64", lambda: synth.workload(1)[0], 0, 0.0),
    ("laplace3d_24", lambda: synth.laplace3d(24), 0, 0.0),
    ("convdiff3d_14_ilu1_tau", lambda: synth.convdiff3d(14), 1, 1e-3),
    ("convdiff3d_14_ilu1", lambda: synth.convdiff3d(14), 1, 0.0),
    ("random_3000", lambda: synth.random_banded(3000, rng=np.random.default_rng(5)), 0, 0.0),
    ("random_sparse_ragged", lambda: synth.random_sparse(333, 0.02, np.random.default_rng(6)), 0, 0.0),
    ("random_sparse_missing_diag", lambda: synth.random_sparse(333, 0.02, np.random.default_rng(6),
                                                               drop_diag_frac=0.1), 0, 0.0),
    ("random_sparse_ilu2", lambda: synth.random_sparse(300, 0.015, np.random.default_rng(7)), 2, 0.0),
]


@pytest.mark.parametrize("sched", FACTOR_SCHEDS, ids=lambda s: s[0])
@pytest.mark.parametrize("name,mk,k,tau", CASES, ids=[c[0] for c in CASES])
def test_factor_bit_exact(jv, name, mk, k, tau, sched):
    A = mk()
    for sym in (True, False):
        an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k, sym=sym)
        ilu = make(jv, A, k, sym, sched)
        f = O.factor(an, A.val, k=k, tau=tau)
        if f.status != O.OK:
            # the oracle stops at the first failing row: same status and row required
            with pytest.raises(jv.IluError) as e:
                ilu.factor(dev(A.val), k=k, tau=tau)
            want = "ILU_ERR_ZERO_PIVOT" if f.status == O.ERR_ZERO_PIVOT else "ILU_ERR_NONFINITE"
            assert e.value.status == want and e.value.info["bad_row"] == f.bad_row
            continue
        info = ilu.factor(dev(A.val), k=k, tau=tau)
        lu, st = ilu.factor_values()
        np.testing.assert_array_equal(st, f.stat)
        assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64)), \
            f"max diff {np.abs(lu - f.val).max()}"
        assert info["n_dropped"] == int((f.stat == 1).sum())


MILU_CASES = [
    ("laplace2d_64", lambda: synth.workload(1)[0], 0, 0.0),
    ("laplace3d_16", lambda: synth.laplace3d(16), 0, 0.0),
    ("convdiff3d_12_ilu1", lambda: synth.convdiff3d(12), 1, 0.0),
    ("convdiff3d_12_ilu1_tau", lambda: synth.convdiff3d(12), 1, 1e-3),
    ("random_sparse_ilu1_tau", lambda: synth.random_sparse(300, 0.02, np.random.default_rng(9)), 1, 1e-2),
    ("random_banded_1500", lambda: synth.random_banded(1500, rng=np.random.default_rng(10)), 0, 0.0),
]


@pytest.mark.parametrize("sched", FACTOR_SCHEDS, ids=lambda s: s[0])
@pytest.mark.parametrize("staged", [1, 0], ids=["staged", "unstaged"])
@pytest.mark.parametrize("name,mk,k,tau", MILU_CASES, ids=[c[0] for c in MILU_CASES])
def test_factor_modified_bit_exact(jv, name, mk, k, tau, staged, sched):
    # modified ILU: every lost update, dropped multiplier and dropped U entry goes to
    # the diagonal in the oracle's order, so the factor is bit for bit the oracle's
    A = mk()
    for sym in (True, False):
        an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k, sym=sym)
        ilu = make(jv, A, k, sym, sched)
        ilu.set_tuning("factor_staged", staged)
        f = O.factor(an, A.val, k=k, tau=tau, milu=True)
        if f.status != O.OK:
            with pytest.raises(jv.IluError) as e:
                ilu.factor(dev(A.val), k=k, tau=tau, milu=True)
            want = "ILU_ERR_ZERO_PIVOT" if f.status == O.ERR_ZERO_PIVOT else "ILU_ERR_NONFINITE"
            assert e.value.status == want and e.value.info["bad_row"] == f.bad_row
            continue
        info = ilu.factor(dev(A.val), k=k, tau=tau, milu=True)
        lu, st = ilu.factor_values()
        np.testing.assert_array_equal(st, f.stat)
        assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64)), \
            f"max diff {np.abs(lu - f.val).max()}"
        assert info["n_dropped"] == int((f.stat == 1).sum())
        # and the plain factor afterwards on the same handle is the plain one
        ilu.factor(dev(A.val), k=k, tau=tau)
        g = O.factor(an, A.val, k=k, tau=tau)
        lu2, _ = ilu.factor_values()
        assert np.array_equal(lu2.view(np.uint64), g.val.view(np.uint64))


@pytest.mark.parametrize("staged", [1, 0], ids=["staged", "unstaged"])
def test_factor_modified_k_below_kmax(jv, staged):
    # entries above fill level k are outside the kept pattern: their updates go to
    # the diagonal too
    A = synth.convdiff3d(10)
    ilu = make(jv, A, 2, True, ("syncfree", "syncfree"))
    ilu.set_tuning("factor_staged", staged)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=2)
    for k, tau in ((0, 0.0), (1, 1e-2), (2, 0.0)):
        ilu.factor(dev(A.val), k=k, tau=tau, milu=True)
        f = O.factor(an, A.val, k=k, tau=tau, milu=True)
        lu, st = ilu.factor_values()
        np.testing.assert_array_equal(st, f.stat)
        assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))


def _heavy(n, seed, lo=100, hi=400):
    return synth.heavy_rows(n, heavy_len=(lo, hi), heavy_frac=0.02, rng=np.random.default_rng(seed))


LONG_CASES = [
    ("heavy_2000_ilu0", lambda: _heavy(2000, 3), 0, 0, 0.0, False, True),
    ("heavy_2000_ilu0_tau_modified", lambda: _heavy(2000, 3), 0, 0, 1e-3, True, True),
    ("heavy_2000_ilu1_k0", lambda: _heavy(2000, 4), 1, 0, 0.0, False, True),
    ("heavy_2000_ilu1_tau", lambda: _heavy(2000, 4), 1, 1, 1e-3, False, True),
    ("heavy_1500_lower_a_modified", lambda: _heavy(1500, 5, 300, 900), 0, 0, 0.0, True, False),
]


@pytest.mark.parametrize("sched", FACTOR_SCHEDS, ids=lambda s: s[0])
@pytest.mark.parametrize("name,mk,kmax,k,tau,milu,sym", LONG_CASES, ids=[c[0] for c in LONG_CASES])
def test_factor_long_rows_bit_exact(jv, name, mk, kmax, k, tau, milu, sym, sched):
    # rows of more than 64 entries: one wave per row with the row in LDS; bit for
    # bit the oracle's factor, then applies, spmv and FGMRES on it
    A = mk()
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=kmax, sym=sym)
    assert np.diff(an.lu_rp).max() > 64
    ilu = make(jv, A, kmax, sym, sched)
    f = O.factor(an, A.val, k=k, tau=tau, milu=milu)
    assert f.status == O.OK
    info = ilu.factor(dev(A.val), k=k, tau=tau, milu=milu)
    lu, st = ilu.factor_values()
    np.testing.assert_array_equal(st, f.stat)
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64)), f"max diff {np.abs(lu - f.val).max()}"
    assert info["n_dropped"] == int((f.stat == 1).sum())
    b = synth.rhs(A.n, 2, np.random.default_rng(8))
    x = ilu.apply(dev(b)).cpu().numpy()
    assert relerr(x, O.apply(an, f.val, b)) <= 1e-12
    y = ilu.spmv(dev(b)).cpu().numpy()
    assert relerr(y, synth.csr_to_dense(A) @ b) <= 1e-12
    _, si = ilu.gmres(dev(b[:, 0].copy()), rtol=1e-10, restart=30, prec="f64")
    assert si["true_relres"] <= 1e-10


def test_factor_rows_beyond_long_limit_unsupported(jv):
    # one row of 5000 entries: beyond the long-row factor's LDS row buffer
    n = 5000
    A = synth.heavy_rows(n, heavy_frac=0.0, rng=np.random.default_rng(9))
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    keep = rows != 7
    r = np.concatenate([rows[keep], np.full(n, 7)])
    c = np.concatenate([A.col_idx[keep], np.arange(n)])
    v = np.concatenate([A.val[keep], np.where(np.arange(n) == 7, float(n), 0.5)])
    B = synth.csr_from_coo(n, r, c, v)
    assert np.diff(B.row_ptr)[7] == n
    ilu = jv.Ilu(B.n, B.row_ptr, B.col_idx)
    with pytest.raises(jv.IluError) as e:
        ilu.factor(dev(B.val))
    assert e.value.status == "ILU_ERR_UNSUPPORTED"


RCM_CASES = [
    ("random_banded_3000", lambda: synth.random_banded(3000, rng=np.random.default_rng(31)), 0, 0.0, True),
    ("convdiff3d_12_ilu1_tau", lambda: synth.convdiff3d(12), 1, 1e-3, True),
    ("random_sparse_ragged_lower_a", lambda: synth.random_sparse(500, 0.01, np.random.default_rng(32)), 0, 0.0,
     False),
]


@pytest.mark.parametrize("sched", FACTOR_SCHEDS, ids=lambda s: s[0])
@pytest.mark.parametrize("name,mk,k,tau,sym", RCM_CASES, ids=[c[0] for c in RCM_CASES])
def test_rcm_preorder_factor_apply_krylov(jv, name, mk, k, tau, sym, sched):
    # reverse Cuthill-McKee preorder: schedule, factor bits and applies equal the
    # oracle's composed analysis; callers keep the input ordering throughout
    A = mk()
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k, sym=sym, rcm_order=True)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k, pattern="sym" if sym else "a", ordering="rcm")
    ilu.set_schedule(*sched)
    s = ilu.schedule()
    np.testing.assert_array_equal(s["perm"], an.perm)
    np.testing.assert_array_equal(s["lu_col_idx"], an.lu_ci)
    f = O.factor(an, A.val, k=k, tau=tau)
    assert f.status == O.OK
    ilu.factor(dev(A.val), k=k, tau=tau)
    lu, st = ilu.factor_values()
    np.testing.assert_array_equal(st, f.stat)
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    b = synth.rhs(A.n, 3, np.random.default_rng(33))
    x = ilu.apply(dev(b)).cpu().numpy()
    assert relerr(x, O.apply(an, f.val, b)) <= 1e-12
    y = ilu.spmv(dev(b)).cpu().numpy()
    assert relerr(y, synth.csr_to_dense(A) @ b) <= 1e-12
    rhs = dev(b[:, 0].copy())
    xs, info = ilu.gmres(rhs, rtol=1e-10, restart=30, prec="f64")
    assert info["true_relres"] <= 1e-10


@pytest.mark.parametrize("sched", FACTOR_SCHEDS, ids=lambda s: s[0])
def test_factor_k_below_kmax(jv, sched):
    A = synth.convdiff3d(10)
    ilu = make(jv, A, 2, True, sched)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=2)
    for k, tau in ((0, 0.0), (1, 1e-2), (2, 0.0)):
        ilu.factor(dev(A.val), k=k, tau=tau)
        f = O.factor(an, A.val, k=k, tau=tau)
        lu, st = ilu.factor_values()
        np.testing.assert_array_equal(st, f.stat)
        assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))


@pytest.mark.parametrize("sched", FACTOR_SCHEDS, ids=lambda s: s[0])
@pytest.mark.parametrize("lanes", [0, 16, 64])
def test_factor_lane_counts_same_bits(jv, sched, lanes):
    A = synth.random_banded(2000, rng=np.random.default_rng(8))
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.set_schedule(sched[0], sched[1], lanes_factor=max(lanes, 32) if lanes else 0)
    ilu.factor(dev(A.val))
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))


@pytest.mark.parametrize("sched", FACTOR_SCHEDS, ids=lambda s: s[0])
def test_factor_errors(jv, sched):
    # zero pivot in the first row, zero pivot later, non-finite value
    A = synth.csr_from_coo(3, [0, 0, 1, 1, 2, 2], [0, 1, 0, 1, 1, 2], [0.0, 1, 1, 2, 1, 3])
    ilu = make(jv, A, sched=sched)
    with pytest.raises(jv.IluError) as e:
        ilu.factor(dev(A.val))
    assert e.value.status == "ILU_ERR_ZERO_PIVOT" and e.value.info["bad_row_original"] == 0
    A = synth.csr_from_coo(2, [0, 0, 1, 1], [0, 1, 0, 1], [1.0, 1, 1, 1])
    ilu = make(jv, A, sched=sched)
    with pytest.raises(jv.IluError) as e:
        ilu.factor(dev(A.val))
    assert e.value.status == "ILU_ERR_ZERO_PIVOT" and e.value.info["bad_row"] == 1
    A = synth.laplace2d(8)
    v = A.val.copy()
    v[40] = np.nan
    ilu = make(jv, A, sched=sched)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, v)
    with pytest.raises(jv.IluError) as e:
        ilu.factor(dev(v))
    assert e.value.status == "ILU_ERR_NONFINITE" and e.value.info["bad_row"] == f.bad_row
    # argument errors
    with pytest.raises(jv.IluError) as e:
        ilu.factor(dev(A.val), k=1)
    assert e.value.status == "ILU_ERR_ARG"
    with pytest.raises(jv.IluError) as e:
        ilu.factor(dev(A.val), tau=-1.0)
    assert e.value.status == "ILU_ERR_ARG"


def test_apply_before_factor_is_state_error(jv):
    A = synth.laplace2d(4)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    with pytest.raises(jv.IluError) as e:
        ilu.apply(dev(np.ones(A.n)))
    assert e.value.status == "ILU_ERR_STATE"
    with pytest.raises(jv.IluError) as e:
        ilu.spmv(dev(np.ones(A.n)))
    assert e.value.status == "ILU_ERR_STATE"


APPLY_CASES = [
    ("laplace2d_64", lambda: synth.workload(1)[0], 0, 0.0),
    ("laplace3d_20", lambda: synth.laplace3d(20), 0, 0.0),
    ("convdiff3d_12_ilu1_tau", lambda: synth.convdiff3d(12), 1, 1e-3),
    ("random_2500", lambda: synth.random_banded(2500, rng=np.random.default_rng(9)), 0, 0.0),
]


@pytest.mark.parametrize("sched", SOLVE_SCHEDS, ids=lambda s: s[1])
@pytest.mark.parametrize("name,mk,k,tau", APPLY_CASES, ids=[c[0] for c in APPLY_CASES])
@pytest.mark.parametrize("nrhs", [1, 3, 16])
def test_apply_f64(jv, name, mk, k, tau, sched, nrhs):
    A = mk()
    rng = np.random.default_rng(nrhs)
    ilu = make(jv, A, k, True, sched)
    ilu.factor(dev(A.val), k=k, tau=tau)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    f = O.factor(an, A.val, k=k, tau=tau)
    b = rng.uniform(-1, 1, (A.n, nrhs)) if nrhs > 1 else rng.uniform(-1, 1, A.n)
    xr = O.apply(an, f.val, b)
    assert relerr(ilu.apply(dev(b)).cpu().numpy(), xr) <= 1e-12
    # permuted space
    bp = b[an.perm]
    xpr = O.apply(an, f.val, bp, permuted=True)
    assert relerr(ilu.apply(dev(bp), permuted=True).cpu().numpy(), xpr) <= 1e-12
    # in place
    bt = dev(b)
    ilu.apply(bt, x=bt)
    assert relerr(bt.cpu().numpy(), xr) <= 1e-12
    # repeated calls keep the published-buffer protocol intact
    for _ in range(3):
        assert relerr(ilu.apply(dev(b)).cpu().numpy(), xr) <= 1e-12


@pytest.mark.parametrize("sched", SOLVE_SCHEDS, ids=lambda s: s[1])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("vec", ["f64", "f32"])
def test_apply_low_precision(jv, sched, prec, vec):
    # FP32 arithmetic on the rounded factor: compared with the oracle's FP32 apply.
    # Both sides accumulate n_row <= 7 products in FP32 in different orders and
    # divide by the pivot; the solve recurrences amplify the per-row rounding by at
    # most the growth of |L^{-1}| |U^{-1}|; the bound below is 2^-17 relative
    # (about 64 FP32 ulps), far below the BF16 factor error itself.
    A = synth.laplace3d(16)
    ilu = make(jv, A, 0, True, sched)
    ilu.factor(dev(A.val), casts=("f32", "bf16"))
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    low = O.cast_f32(f.val) if prec == "f32" else O.cast_bf16(f.val)
    b = np.random.default_rng(3).uniform(-1, 1, (A.n, 2))
    xr = O.apply(an, low, b, prec=prec)
    bt = dev(b) if vec == "f64" else dev(b.astype(np.float32))
    x = ilu.apply(bt, prec=prec).cpu().numpy().astype(np.float64)
    if vec == "f32":
        xr = O.apply(an, low, b.astype(np.float32).astype(np.float64), prec=prec)
    assert relerr(x, xr) <= 2.0 ** -17


TAIL_CASES = [
    ("random_banded_6000_all", lambda: synth.random_banded(6000, rng=np.random.default_rng(31)), 0, 65536),
    ("laplace2d_150_tail65", lambda: synth.laplace2d(150), 0, 65),
    ("heavy_4000_long_rows", lambda: synth.heavy_rows(4000, heavy_len=(150, 700), heavy_frac=0.03,
                                                      rng=np.random.default_rng(32)), 0, 65536),
    ("random_banded_3000_ilu1_all", lambda: synth.random_banded(3000, rng=np.random.default_rng(33)), 1, 65536),
]


FACTOR_TAIL_CASES = [
    ("random_banded_6000_all", lambda: synth.random_banded(6000, rng=np.random.default_rng(31)), 0, 65536),
    ("laplace2d_150_tail65", lambda: synth.laplace2d(150), 0, 65),
    ("tridiag_3000_chain", lambda: synth.tridiag(3000), 0, 65536),
    ("laplace2d_60_ilu1", lambda: synth.laplace2d(60), 1, 65536),
    ("random_banded_3000_ilu1_narrow", lambda: synth.random_banded(3000, band=2, rnd=2, rng=np.random.default_rng(6)),
     1, 65536),
]


@pytest.mark.parametrize("name,mk,k,M", FACTOR_TAIL_CASES, ids=[c[0] for c in FACTOR_TAIL_CASES])
def test_factor_tail_bit_exact(jv, name, mk, k, M):
    # the factor's lower stage (rows before the tail sync-free, the tail streamed by
    # one workgroup): the serial factor's bits, its FP32/BF16 copies and the spmv
    # operand as on the other schedules, every schedule of the handle alike
    A = mk()
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    f = O.factor(an, A.val, k=k)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k, tile_rows=128, tail_min_rows=M)
    assert ilu.factor_tail()["level0"] >= 0 and ilu.get_tuning("factor_lower_planned") == 1
    assert ilu.get_tuning("factor_lower_stage") == 0
    ilu.set_tuning("factor_lower_stage", 1)
    for sched in ("tiled", "syncfree", "level"):
        ilu.set_schedule(sched, "syncfree")
        for rep in range(2):
            ilu.factor(dev(A.val * (1.0 + rep)), k=k, casts=("f32", "bf16"))
            fr = f if rep == 0 else O.factor(an, A.val * 2.0, k=k)
            lu, _ = ilu.factor_values()
            assert np.array_equal(lu.view(np.uint64), fr.val.view(np.uint64)), (sched, rep)
            assert np.array_equal(ilu.factor_values_prec("f32").view(np.uint32), O.cast_f32(fr.val).view(np.uint32))
            assert np.array_equal(ilu.factor_values_prec("bf16"), O.cast_bf16(fr.val))
            x = np.random.default_rng(38).uniform(-1, 1, A.n)
            yr = O.spmv(A.n, A.row_ptr, A.col_idx, A.val * (1.0 + rep), x)
            assert relerr(ilu.spmv(dev(x)).cpu().numpy(), yr) <= 1e-12
    # a non-finite input value in the tail: the first bad row, as the serial factor
    v = A.val.copy()
    r_bad = A.n - A.n // 5
    v[A.row_ptr[r_bad]] = np.nan
    fb = O.factor(an, v, k=k)
    with pytest.raises(jv.IluError) as e:
        ilu.factor(dev(v), k=k)
    assert e.value.status == "ILU_ERR_NONFINITE" and e.value.info["bad_row"] == fb.bad_row
    ilu.factor(dev(A.val), k=k)
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    # the autotuner times it against the other schedules and keeps the faster
    res, _ = ilu.tune(dev(A.val), reps=2)
    planned = ilu.get_tuning("tail_min_rows") > 0 and ilu.get_tuning("factor_lower_planned") == 1
    assert ((res[:, 0] == 0) & (res[:, 1] == 10)).sum() == int(planned)
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))


@pytest.mark.parametrize("sched", ["tiled", "syncfree", "level"])
@pytest.mark.parametrize("name,mk,k,M", TAIL_CASES, ids=[c[0] for c in TAIL_CASES])
def test_tail_apply(jv, name, mk, k, M, sched):
    # the lower stage: the levels before it on the handle's schedule (sync-free or
    # level launches), the tail streamed by one workgroup per right-hand side
    A = mk()
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    f = O.factor(an, A.val, k=k)
    assert f.status == O.OK
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k, tile_rows=128, tail_min_rows=M)
    ilu.set_schedule("syncfree", sched)
    info = ilu.info()
    assert info["tail_rows"] > 0 and info["tail_urows"] > 0
    ilu.factor(dev(A.val), k=k, casts=("f32",))
    rng = np.random.default_rng(34)
    for nrhs in (1, 3):
        b = rng.uniform(-1, 1, (A.n, nrhs)) if nrhs > 1 else rng.uniform(-1, 1, A.n)
        x = ilu.apply(dev(b)).cpu().numpy()
        assert relerr(x, O.apply(an, f.val, b)) <= 1e-12
        b32 = b.astype(np.float32)
        x32 = ilu.apply(dev(b32), prec="f32").cpu().numpy().astype(np.float64)
        xr32 = O.apply(an, O.cast_f32(f.val), b32.astype(np.float64), prec="f32")
        assert relerr(x32, xr32) <= 2.0 ** -17
    bp = rng.uniform(-1, 1, A.n)
    xp = dev(bp)
    ilu.apply(xp, x=xp, permuted=True)   # in place, level ordering
    assert relerr(xp.cpu().numpy(), O.apply(an, f.val, bp, permuted=True)) <= 1e-12
    ilu.status()
    _, si = ilu.gmres(dev(rng.uniform(-1, 1, A.n)), rtol=1e-10, restart=30)
    assert si["true_relres"] <= 1e-10
    # and the same handle without the lower stage gives the same results
    ilu.set_tuning("tail_min_rows", 0)
    assert ilu.info()["tail_rows"] == 0
    x0 = ilu.apply(dev(bp)).cpu().numpy()
    ilu.set_tuning("tail_min_rows", M)
    x1 = ilu.apply(dev(bp)).cpu().numpy()
    assert relerr(x1, x0) <= 1e-12


@pytest.mark.parametrize("sched", FACTOR_SCHEDS, ids=lambda s: s[0])
@pytest.mark.parametrize("name,mk,k,tau,milu", [
    ("random_3000", lambda: synth.random_banded(3000, rng=np.random.default_rng(10)), 0, 0.0, False),
    ("convdiff3d_14_ilu1_tau", lambda: synth.convdiff3d(14), 1, 1e-3, False),
    ("laplace3d_20_modified", lambda: synth.laplace3d(20), 0, 0.0, True),
], ids=lambda v: v if isinstance(v, str) else "")
def test_casts_bit_exact(jv, name, mk, k, tau, milu, sched):
    # the FP32 and BF16 storage copies are the oracle's roundings of the oracle's
    # factor (dropped entries 0), whether cast kernels or the tiled factor write them
    A = mk()
    ilu = make(jv, A, k, True, sched, tile_rows=128)
    for rep in range(2):
        ilu.factor(dev(A.val), k=k, tau=tau, casts=("f32", "bf16"), milu=milu)
        an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
        f = O.factor(an, A.val, k=k, tau=tau, milu=milu)
        lu, _ = ilu.factor_values()
        assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
        assert np.array_equal(ilu.factor_values_prec("f32").view(np.uint32), O.cast_f32(f.val).view(np.uint32))
        assert np.array_equal(ilu.factor_values_prec("bf16"), O.cast_bf16(f.val))


@pytest.mark.parametrize("sched", FACTOR_SCHEDS, ids=lambda s: s[0])
@pytest.mark.parametrize("name,mk,k", [
    ("laplace3d_20", lambda: synth.laplace3d(20), 0),
    ("convdiff3d_12_ilu1", lambda: synth.convdiff3d(12), 1),
    ("random_sparse_missing_diag", lambda: synth.random_sparse(333, 0.02, np.random.default_rng(6),
                                                               drop_diag_frac=0.1), 0),
], ids=lambda v: v if isinstance(v, str) else "")
def test_spmv_values_from_factor(jv, name, mk, k, sched):
    # the spmv operand loaded by ilu_factor (the tiled factor writes it while it
    # stages the rows; other schedules gather it): equal to the oracle's copy
    A = mk()
    rng = np.random.default_rng(12)
    ilu = make(jv, A, k, True, sched, tile_rows=128)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    for rep in range(2):
        try:
            ilu.factor(dev(A.val * (1.0 + rep)), k=k)
        except jv.IluError as e:   # an inserted zero diagonal may be a zero pivot; the values are loaded
            assert e.status in ("ILU_ERR_ZERO_PIVOT", "ILU_ERR_NONFINITE")
        x = rng.integers(-4, 5, (A.n, 2)).astype(np.float64)
        want = O.spmv(A.n, an.b_rp, an.b_ci, O.b_values(an, A.val * (1.0 + rep)), x)
        got = ilu.spmv(dev(x), permuted=True).cpu().numpy()
        assert relerr(got, want) <= 1e-12
        xo = rng.uniform(-1, 1, A.n)
        yo = O.spmv(A.n, A.row_ptr, A.col_idx, A.val * (1.0 + rep), xo)
        assert relerr(ilu.spmv(dev(xo)).cpu().numpy(), yo) <= 1e-12


@pytest.mark.parametrize("name,mk,k,tau", APPLY_CASES, ids=[c[0] for c in APPLY_CASES])
def test_spmv(jv, name, mk, k, tau):
    A = mk()
    rng = np.random.default_rng(11)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k)
    ilu.set_values(dev(A.val))
    for nrhs in (1, 4):
        x = rng.uniform(-1, 1, (A.n, nrhs)) if nrhs > 1 else rng.uniform(-1, 1, A.n)
        yr = O.spmv(A.n, A.row_ptr, A.col_idx, A.val, x)
        assert relerr(ilu.spmv(dev(x)).cpu().numpy(), yr) <= 1e-12
        y0 = rng.uniform(-1, 1, x.shape)
        got = ilu.spmv(dev(x), y=dev(y0), alpha=2.0, beta=-0.5).cpu().numpy()
        assert relerr(got, 2.0 * yr - 0.5 * y0) <= 1e-12
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    xp = rng.uniform(-1, 1, A.n)
    yp = O.spmv(A.n, an.b_rp, an.b_ci, O.b_values(an, A.val), xp)
    assert relerr(ilu.spmv(dev(xp), permuted=True).cpu().numpy(), yp) <= 1e-12
    # integer-valued: exact regardless of summation order
    Ai = rng.integers(-4, 5, A.nnz).astype(np.float64)
    xi = rng.integers(-4, 5, A.n).astype(np.float64)
    ilu.set_values(dev(Ai))
    assert np.array_equal(ilu.spmv(dev(xi)).cpu().numpy(), O.spmv(A.n, A.row_ptr, A.col_idx, Ai, xi))


@pytest.mark.parametrize("name,mk,default", [
    ("laplace3d_20", lambda: synth.laplace3d(20), 1),
    ("random_sparse_ragged", lambda: synth.random_sparse(333, 0.05, np.random.default_rng(6)), 16),
    ("heavy_3000_short_and_long", lambda: synth.heavy_rows(3000, heavy_len=(65, 200), heavy_frac=0.05,
                                                           rng=np.random.default_rng(32)), 1),
], ids=lambda v: v if isinstance(v, str) else "")
def test_spmv_lanes_every_setting(jv, name, mk, default):
    # one row per lane (rows averaging at most 8 entries; longer rows in batches of
    # 8) and every lane-group size: the oracle's products to rounding, several
    # right-hand sides, alpha and beta, both orderings; long rows still go to the
    # one-wave pass
    A = mk()
    rng = np.random.default_rng(41)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.set_values(dev(A.val))
    assert ilu.get_tuning("spmv_lanes") == default
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    x3 = rng.uniform(-1, 1, (A.n, 3))
    y0 = rng.uniform(-1, 1, (A.n, 3))
    yr = O.spmv(A.n, A.row_ptr, A.col_idx, A.val, x3)
    xp = rng.uniform(-1, 1, A.n)
    yp = O.spmv(A.n, an.b_rp, an.b_ci, O.b_values(an, A.val), xp)
    for lanes in (1, 4, 8, 16, 32, 64):
        ilu.set_tuning("spmv_lanes", lanes)
        assert relerr(ilu.spmv(dev(x3)).cpu().numpy(), yr) <= 1e-12
        got = ilu.spmv(dev(x3), y=dev(y0), alpha=2.0, beta=-0.5).cpu().numpy()
        assert relerr(got, 2.0 * yr - 0.5 * y0) <= 1e-12
        assert relerr(ilu.spmv(dev(xp), permuted=True).cpu().numpy(), yp) <= 1e-12
    with pytest.raises(jv.IluError):
        ilu.set_tuning("spmv_lanes", 2)


@pytest.mark.parametrize("name,mk", [
    ("heavy_6000_rows_over_waves", lambda: synth.heavy_rows(6000, heavy_len=(900, 3500), heavy_frac=0.02,
                                                            rng=np.random.default_rng(31))),
    ("heavy_3000_short_and_long", lambda: synth.heavy_rows(3000, heavy_len=(65, 200), heavy_frac=0.05,
                                                           rng=np.random.default_rng(32))),
], ids=lambda v: v if isinstance(v, str) else "")
def test_spmv_nnz_balanced(jv, name, mk):
    # the nnz-balanced pass (rows cut across lanes and waves, the pieces of rows
    # over several waves added by the second kernel) against the oracle and the
    # row-per-group pass; integer values exactly; the same bits run after run
    A = mk()
    rng = np.random.default_rng(33)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.set_values(dev(A.val))
    ilu.set_tuning("spmv_nz", 1)
    assert ilu.get_tuning("spmv_nz") == 1
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    x = rng.uniform(-1, 1, A.n)
    y0 = rng.uniform(-1, 1, A.n)
    for permuted in (False, True):
        if permuted:
            yr = O.spmv(A.n, an.b_rp, an.b_ci, O.b_values(an, A.val), x)
        else:
            yr = O.spmv(A.n, A.row_ptr, A.col_idx, A.val, x)
        got = ilu.spmv(dev(x), permuted=permuted).cpu().numpy()
        assert relerr(got, yr) <= 1e-12
        again = ilu.spmv(dev(x), permuted=permuted).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), again.view(np.uint64))
        got2 = ilu.spmv(dev(x), y=dev(y0), alpha=-1.5, beta=0.25, permuted=permuted).cpu().numpy()
        assert relerr(got2, -1.5 * yr + 0.25 * y0) <= 1e-12
        ilu.set_tuning("spmv_nz", 0)
        assert ilu.get_tuning("spmv_nz") == 0
        assert relerr(ilu.spmv(dev(x), permuted=permuted).cpu().numpy(), yr) <= 1e-12
        ilu.set_tuning("spmv_nz", 1)
    Ai = rng.integers(-4, 5, A.nnz).astype(np.float64)
    xi = rng.integers(-4, 5, A.n).astype(np.float64)
    ilu.set_values(dev(Ai))
    assert np.array_equal(ilu.spmv(dev(xi)).cpu().numpy(), O.spmv(A.n, A.row_ptr, A.col_idx, Ai, xi))


def test_spmv_nnz_balanced_default_and_tuned(jv):
    # rows beyond 4096 entries take the nnz-balanced pass by default
    A = synth.heavy_rows(20000, heavy_len=(5000, 9000), heavy_frac=0.001, rng=np.random.default_rng(34))
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.set_values(dev(A.val))
    assert np.diff(A.row_ptr).max() > 4096 and ilu.get_tuning("spmv_nz") == 1
    x = np.random.default_rng(35).uniform(-1, 1, A.n)
    assert relerr(ilu.spmv(dev(x)).cpu().numpy(), O.spmv(A.n, A.row_ptr, A.col_idx, A.val, x)) <= 1e-12
    # shorter long rows: the row pass by default; the autotuner times both
    B = synth.heavy_rows(6000, heavy_len=(300, 1200), heavy_frac=0.02, rng=np.random.default_rng(36))
    ilu = jv.Ilu(B.n, B.row_ptr, B.col_idx)
    assert ilu.get_tuning("spmv_nz") == 0
    ilu.factor(dev(B.val))
    res, _ = ilu.tune(dev(B.val), reps=2)
    spmv_rows = res[res[:, 0] == 2]
    assert sorted(spmv_rows[spmv_rows[:, 1] == 20.0][:, 2].astype(int).tolist()) == [1, 4, 8, 16, 32, 64]
    assert (spmv_rows[:, 1] == 21.0).sum() == 1 and set(spmv_rows[:, 1].tolist()) == {20.0, 21.0}
    assert ilu.get_tuning("spmv_nz") == int(spmv_rows[np.argmin(spmv_rows[:, 3]), 1] == 21.0)
    xb = np.random.default_rng(37).uniform(-1, 1, B.n)
    assert relerr(ilu.spmv(dev(xb)).cpu().numpy(), O.spmv(B.n, B.row_ptr, B.col_idx, B.val, xb)) <= 1e-12


@pytest.mark.parametrize("sched", SOLVE_SCHEDS, ids=lambda s: s[1])
def test_apply_integer_exact(jv, sched):
    rng = np.random.default_rng(12)
    A = synth.integer_unit_lower(400, 0.01, rng)
    ilu = make(jv, A, sched=sched)
    ilu.factor(dev(A.val))
    b = rng.integers(-3, 4, (A.n, 4)).astype(np.float64)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    x = ilu.apply(dev(b)).cpu().numpy()
    assert np.array_equal(x, O.apply(an, f.val, b))


@pytest.mark.parametrize("sched", SOLVE_SCHEDS, ids=lambda s: s[1])
def test_pcg_and_gmres(jv, sched):
    A, b = synth.workload(1)
    ilu = make(jv, A, sched=sched)
    ilu.factor(dev(A.val), casts=("f32", "bf16"))
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    xr, itr, rr, st = O.pcg(an, O.b_values(an, A.val), f.val, b)
    x, info = ilu.pcg(dev(b))
    assert info["true_relres"] <= 1e-10 and abs(info["iters"] - itr) <= 1
    assert np.abs(x.cpu().numpy() - xr).max() <= 1e-8 * np.abs(xr).max()
    for prec in ("f32", "bf16"):
        x, info = ilu.pcg(dev(b), prec=prec)
        assert info["true_relres"] <= 1e-10
    A = synth.convdiff3d(12)
    b = np.random.default_rng(13).uniform(-1, 1, A.n)
    ilu = make(jv, A, 1, True, sched)
    ilu.factor(dev(A.val), k=1, tau=1e-3, casts=("f32", "bf16"))
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    f = O.factor(an, A.val, k=1, tau=1e-3)
    for prec in ("f64", "f32", "bf16"):
        low = None if prec == "f64" else (O.cast_f32(f.val) if prec == "f32" else O.cast_bf16(f.val))
        xr, itr, rr, st = O.fgmres(an, O.b_values(an, A.val), f.val, b, prec=prec, lu_low=low)
        x, info = ilu.gmres(dev(b), prec=prec)
        assert info["true_relres"] <= 1e-10 and abs(info["iters"] - itr) <= 1, (prec, info, itr)


def test_krylov_exact_preconditioner_and_noconv(jv):
    A = synth.laplace2d(6)
    b = np.random.default_rng(14).uniform(-1, 1, A.n)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=A.n)
    ilu.factor(dev(A.val), k=A.n)
    x, info = ilu.pcg(dev(b))
    assert info["iters"] == 1
    x, info = ilu.gmres(dev(b))
    assert info["iters"] == 1
    A, b = synth.workload(1)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.factor(dev(A.val))
    x, info = ilu.pcg(dev(b), maxit=3, raise_on_fail=False)
    assert info["status"] == "ILU_ERR_NOCONV" and info["iters"] == 3


@pytest.mark.parametrize("sched", SCHEDS, ids=lambda s: s[0])
def test_adjoint_against_oracle(jv, sched):
    rng = np.random.default_rng(15)
    A = synth.random_sparse(300, 0.02, rng)
    for k in (0, 1):
        ilu = make(jv, A, k, False, sched)
        ilu.factor(dev(A.val), k=k)
        an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k, sym=False)
        f = O.factor(an, A.val, k=k)
        b = rng.uniform(-1, 1, (A.n, 3))
        gx = rng.uniform(-1, 1, (A.n, 3))
        x, y = ilu.apply_ex(dev(b))
        xr, yr = O.apply(an, f.val, b, want_y=True)
        assert relerr(x.cpu().numpy(), xr) <= 1e-12 and relerr(y.cpu().numpy(), yr) <= 1e-12
        gb, glu = ilu.adjoint(dev(gx), x, y)
        gbr, glur = O.adjoint(an, f.val, gx, xr, yr)
        assert relerr(gb.cpu().numpy(), gbr) <= 1e-12
        g = glu.cpu().numpy()
        assert np.abs(g - glur).max() <= 1e-12 * np.abs(glur).max()


@pytest.mark.parametrize("tile_rows", [16, 100, 0])
@pytest.mark.parametrize("name,mk,k", [
    ("laplace2d_30", lambda: synth.laplace2d(30), 0),
    ("convdiff3d_8_ilu1", lambda: synth.convdiff3d(8), 1),
    ("random_sym_400", lambda: synth.random_sparse(400, 0.015, np.random.default_rng(17), symmetric_pattern=True), 0),
], ids=lambda v: v if isinstance(v, (str, int)) else "")
def test_adjoint_tiled_symmetric_pattern(jv, name, mk, k, tile_rows):
    # a symmetric factor pattern: the transposed solves of the adjoint run on the
    # forward and backward tiles, values through the transposed view's map
    A = mk()
    rng = np.random.default_rng(18)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k, tile_rows=tile_rows)
    ilu.set_schedule("syncfree", "tiled")
    ilu.factor(dev(A.val), k=k)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    f = O.factor(an, A.val, k=k)
    for nrhs in (1, 3):
        b = rng.uniform(-1, 1, (A.n, nrhs))
        gx = rng.uniform(-1, 1, (A.n, nrhs))
        x, y = ilu.apply_ex(dev(b))
        xr, yr = O.apply(an, f.val, b, want_y=True)
        assert relerr(x.cpu().numpy(), xr) <= 1e-12
        gb, glu = ilu.adjoint(dev(gx), x, y)
        gbr, glur = O.adjoint(an, f.val, gx, xr, yr)
        assert relerr(gb.cpu().numpy(), gbr) <= 1e-12
        g = glu.cpu().numpy()
        assert np.abs(g - glur).max() <= 1e-12 * np.abs(glur).max()


def test_autograd_finite_differences(jv):
    rng = np.random.default_rng(16)
    A = synth.convdiff3d(6)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.factor(dev(A.val))
    lu0 = ilu.factor_tensor()
    b = dev(rng.uniform(-1, 1, (A.n, 2))).requires_grad_(True)
    lu = lu0.clone().requires_grad_(True)
    c = dev(rng.uniform(-1, 1, (A.n, 2)))
    x = jv.IluApply.apply(ilu, b, lu)
    (x * c).sum().backward()
    h = 1e-6

    def loss(bb, ll):
        with torch.no_grad():
            return float((jv.IluApply.apply(ilu, bb, ll) * c).sum())

    for _ in range(3):
        vb = dev(rng.standard_normal((A.n, 2)))
        fd = (loss(b + h * vb, lu) - loss(b - h * vb, lu)) / (2 * h)
        assert abs(fd - float((b.grad * vb).sum())) <= 1e-6 * max(1.0, abs(fd))
        vl = dev(rng.standard_normal(ilu.nnz_lu))
        fd = (loss(b, lu + h * vl) - loss(b, lu - h * vl)) / (2 * h)
        assert abs(fd - float((lu.grad * vl).sum())) <= 1e-6 * max(1.0, abs(fd))


def test_batched_equals_singles(jv):
    mats, rhs = synth.workload(5, scale=0.12)
    mats, rhs = mats[:24], rhs[:24]
    hb = jv.Ilu.batched(mats)
    ro, zo = hb.batch_offsets()
    vals = np.concatenate([m.val for m in mats])
    b = np.concatenate(rhs)
    hb.factor(dev(vals), casts=("f32",))
    lu_b, _ = hb.factor_values()
    x_b = hb.apply(dev(b)).cpu().numpy()
    x_b32 = hb.apply(dev(b.astype(np.float32)), prec="f32").cpu().numpy()
    sb = hb.schedule()
    for i, M in enumerate(mats):
        an = O.analyze(M.n, M.row_ptr, M.col_idx)
        f = O.factor(an, M.val)
        xr = O.apply(an, f.val, rhs[i])
        assert relerr(x_b[ro[i]:ro[i + 1]], xr) <= 1e-12
        xr32 = O.apply(an, O.cast_f32(f.val), rhs[i].astype(np.float32).astype(np.float64), prec="f32")
        assert relerr(x_b32[ro[i]:ro[i + 1]].astype(np.float64), xr32) <= 2.0 ** -17
        # factor entries of matrix i (the batch keeps each matrix's rows and entries)
        rows = np.nonzero((sb["perm"] >= ro[i]) & (sb["perm"] < ro[i + 1]))[0]
        got = np.concatenate([lu_b[sb["lu_row_ptr"][r]:sb["lu_row_ptr"][r + 1]] for r in rows])
        want = np.concatenate([f.val[an.lu_rp[an.iperm[sb["perm"][r] - ro[i]]]:
                                     an.lu_rp[an.iperm[sb["perm"][r] - ro[i]] + 1]] for r in rows])
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def _stage_us(ilu, fn, reps, keys):
    fn()
    torch.cuda.synchronize()
    ilu.profile(True, 1 << 12)
    ilu.profile_read()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    p = ilu.profile_read()
    ilu.profile(False)
    return 1e3 * sum(p[k][0] for k in keys) / reps


@pytest.mark.parametrize("name,mk,k,tau,milu", [
    ("laplace3d_40_modified", lambda: synth.laplace3d(40), 0, 0.0, True),
    ("convdiff3d_20_ilu1_tau", lambda: synth.convdiff3d(20), 1, 1e-3, False),
], ids=lambda v: v if isinstance(v, str) else "")
def test_tune_no_slower_and_same_factor(jv, name, mk, k, tau, milu):
    # the tuner searches level / sync-free / tiled launches and the tile size (the
    # level-merge threshold); it re-runs the caller's factor (k, tau, modified) and
    # must leave its bits, and end no slower than the defaults it started from
    A = mk()
    a = dev(A.val)
    b = dev(np.random.default_rng(21).uniform(-1, 1, A.n))
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k)
    ilu.factor(a, k=k, tau=tau, casts=("f32",), milu=milu)
    t_fac0 = _stage_us(ilu, lambda: ilu.factor(a, k=k, tau=tau, casts=("f32",), milu=milu), 5, ("factor",))
    t_app0 = _stage_us(ilu, lambda: ilu.apply(b, permuted=True), 10, ("forward", "backward"))
    res, chosen = ilu.tune(a, reps=3)
    assert (res[:, 1] == 3).any(), "tiled candidates were timed"
    assert {128, 256, 512} <= set(res[res[:, 1] == 3][:, 2].astype(int))
    # the tiled factor's own tile size, when the tiled factor runs on the chosen tiling
    ft = res[(res[:, 0] == 0) & (res[:, 1] == 11)]
    if len(ft):
        assert len(set(ft[:, 2].astype(int))) == len(ft) and ilu.get_tuning("factor_tiled") == 1
    # the spmv's lanes per row: every setting timed, the fastest kept
    sp = res[(res[:, 0] == 2) & (res[:, 1] == 20)]
    assert sorted(sp[:, 2].astype(int).tolist()) == [1, 4, 8, 16, 32, 64]
    assert ilu.get_tuning("spmv_lanes") == int(sp[np.argmin(sp[:, 3]), 2])
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    f = O.factor(an, A.val, k=k, tau=tau, milu=milu)
    lu, st = ilu.factor_values()
    np.testing.assert_array_equal(st, f.stat)
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    bh = b.cpu().numpy()
    assert relerr(ilu.apply(b).cpu().numpy(), O.apply(an, f.val, bh)) <= 1e-12
    t_fac1 = _stage_us(ilu, lambda: ilu.factor(a, k=k, tau=tau, casts=("f32",), milu=milu), 5, ("factor",))
    t_app1 = _stage_us(ilu, lambda: ilu.apply(b, permuted=True), 10, ("forward", "backward"))
    assert t_app1 <= 1.25 * t_app0 + 20.0, (t_app0, t_app1, chosen)
    assert t_fac1 <= 1.25 * t_fac0 + 20.0, (t_fac0, t_fac1, chosen)


def test_tune_tries_the_lower_stage(jv):
    # narrow levels everywhere: the tuner times the lower stage next to the other
    # schedules, keeps whichever is faster, and the results stay the oracle's
    A = synth.random_banded(6000, rng=np.random.default_rng(35))
    a = dev(A.val)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.factor(a)
    res, chosen = ilu.tune(a, reps=3)
    assert (res[:, 1] == 10).any()
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    b = np.random.default_rng(36).uniform(-1, 1, A.n)
    assert relerr(ilu.apply(dev(b)).cpu().numpy(), O.apply(an, f.val, b)) <= 1e-12
    tail_rows = res[res[:, 1] == 10]
    best_other = res[(res[:, 0] == 1) & (res[:, 1] != 10)][:, 3].min()
    assert (ilu.get_tuning("tail_min_rows") > 0) == (tail_rows[:, 3].min() < best_other)


@pytest.mark.parametrize("sched", ["tiled", "syncfree", "level"])
def test_apply_timeout_reported_and_recovered(jv, sched):
    # failure path forced from the host: the abort flag raised inside an apply makes
    # every wait of its kernels give up within 64 polls (all kernels exit); the
    # status query reports ILU_ERR_TIMEOUT and re-arms, and the next apply is right
    A = synth.laplace3d(24)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, tile_rows=128)
    ilu.set_schedule("syncfree", sched)
    ilu.factor(dev(A.val))
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    b = np.random.default_rng(22).uniform(-1, 1, A.n)
    xr = O.apply(an, f.val, b)
    bd = dev(b)
    ilu.status()
    ilu.set_tuning("force_abort", 2)
    ilu.apply(bd)
    with pytest.raises(jv.IluError) as e:
        ilu.status()
    assert e.value.status == "ILU_ERR_TIMEOUT"
    ilu.status()   # reported once
    assert relerr(ilu.apply(bd).cpu().numpy(), xr) <= 1e-12
    ilu.status()
    # a flag left up by an unreported timeout: the next apply re-arms first, computes
    # the right result, and the timeout is still reported
    ilu.set_tuning("force_abort", 1)
    assert relerr(ilu.apply(bd).cpu().numpy(), xr) <= 1e-12
    with pytest.raises(jv.IluError) as e:
        ilu.status()
    assert e.value.status == "ILU_ERR_TIMEOUT"
    # the Krylov drivers stop with the status at their next readback
    ilu.set_tuning("force_abort", 2)
    with pytest.raises(jv.IluError) as e:
        ilu.pcg(bd, rtol=1e-10)
    assert e.value.status == "ILU_ERR_TIMEOUT"
    _, info = ilu.pcg(bd, rtol=1e-10)
    assert info["true_relres"] <= 1e-10
    # a factor after a pending timeout re-arms the intermediates first (the timeout
    # is still reported once), and the applies after it are right
    ilu.set_tuning("force_abort", 1)
    ilu.factor(dev(A.val))
    assert relerr(ilu.apply(bd).cpu().numpy(), xr) <= 1e-12
    with pytest.raises(jv.IluError) as e:
        ilu.status()
    assert e.value.status == "ILU_ERR_TIMEOUT"
    ilu.status()


def test_batched_adjoint_finite_differences(jv):
    # the adjoint of a batched handle (reduced batch, 4 right-hand sides per matrix)
    # against central differences along random directions, through IluApply
    mats, _ = synth.workload(5, scale=0.12)
    mats = mats[:8]
    hb = jv.Ilu.batched(mats)
    vals = np.concatenate([m.val for m in mats])
    hb.factor(dev(vals), casts=())
    rng = np.random.default_rng(23)
    lu0 = hb.factor_tensor()
    b = dev(rng.uniform(-1, 1, (hb.n, 4))).requires_grad_(True)
    lu = lu0.clone().requires_grad_(True)
    c = dev(rng.uniform(-1, 1, (hb.n, 4)))
    x = jv.IluApply.apply(hb, b, lu)
    (x * c).sum().backward()
    h = 1e-6

    def loss(bb, ll):
        with torch.no_grad():
            return float((jv.IluApply.apply(hb, bb, ll) * c).sum())

    for _ in range(3):
        vb = dev(rng.standard_normal((hb.n, 4)))
        fd = (loss(b + h * vb, lu) - loss(b - h * vb, lu)) / (2 * h)
        assert abs(fd - float((b.grad * vb).sum())) <= 1e-6 * max(1.0, abs(fd))
        vl = dev(rng.standard_normal(hb.nnz_lu))
        fd = (loss(b, lu + h * vl) - loss(b, lu - h * vl)) / (2 * h)
        assert abs(fd - float((lu.grad * vl).sum())) <= 1e-6 * max(1.0, abs(fd))


def test_tune_keeps_results(jv):
    A = synth.laplace3d(20)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    a = dev(A.val)
    ilu.factor(a, casts=("f32",))
    res, chosen = ilu.tune(a, reps=2)
    assert len(res) >= 4
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    b = np.random.default_rng(17).uniform(-1, 1, A.n)
    assert relerr(ilu.apply(dev(b)).cpu().numpy(), O.apply(an, f.val, b)) <= 1e-12
    x32 = ilu.apply(dev(b), prec="f32")   # FP32 copy survives tuning
    assert x32.shape == (A.n,)


def test_profile_counts(jv):
    A = synth.laplace3d(12)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.profile(True)
    ilu.factor(dev(A.val))
    b = dev(np.ones(A.n))
    ilu.apply(b)
    ilu.spmv(b)
    p = ilu.profile_read()
    assert p["factor"][1] == 1 and p["forward"][1] == 1 and p["backward"][1] == 1 and p["spmv"][1] == 1
    assert all(v[0] > 0 for v in p.values())


def test_multi_rhs_16_low_precision_vectors(jv):
    # 16 right-hand sides, FP32 factor and FP32 vectors (the random-matrix workload recipe)
    A = synth.random_banded(6000, rng=np.random.default_rng(18))
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.factor(dev(A.val), casts=("f32",))
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    b = np.random.default_rng(19).uniform(-1, 1, (A.n, 16)).astype(np.float32)
    x = ilu.apply(dev(b), prec="f32").cpu().numpy().astype(np.float64)
    xr = O.apply(an, O.cast_f32(f.val), b.astype(np.float64), prec="f32")
    assert relerr(x, xr) <= 2.0 ** -17
    x64 = ilu.apply(dev(b.astype(np.float64))).cpu().numpy()
    assert relerr(x64, O.apply(an, f.val, b.astype(np.float64))) <= 1e-12
    # 20 right-hand sides: one full batch of 16 and a partial one
    b20 = np.random.default_rng(20).uniform(-1, 1, (A.n, 20))
    assert relerr(ilu.apply(dev(b20)).cpu().numpy(), O.apply(an, f.val, b20)) <= 1e-12


@pytest.mark.parametrize("sched", SOLVE_SCHEDS, ids=lambda s: s[1])
def test_apply_graph_replays(jv, sched):
    # a captured apply replayed several times, with eager work and new inputs between
    # replays; every replay is checked against the eager result
    mats, rhs = synth.workload(5, scale=0.1)
    mats, rhs = mats[:16], rhs[:16]
    hb = jv.Ilu.batched(mats)
    hb.set_schedule(*sched)
    vals = np.concatenate([m.val for m in mats])
    hb.factor(dev(vals), casts=("f32",))
    b0 = np.concatenate(rhs).astype(np.float32)
    bt = dev(b0)
    xt = torch.empty_like(bt)
    g = hb.apply_graph(bt, xt, prec="f32")
    rng = np.random.default_rng(21)
    for it in range(4):
        bnew = rng.uniform(-1, 1, b0.shape).astype(np.float32)
        bt.copy_(dev(bnew))
        g.launch()
        torch.cuda.synchronize()
        got = xt.cpu().numpy().copy()
        want = hb.apply(dev(bnew), prec="f32").cpu().numpy()      # eager, in between replays
        hb.spmv(dev(bnew.astype(np.float64)))                      # unrelated eager work
        torch.cuda.synchronize()
        assert np.array_equal(got, want), it
    del g


@pytest.mark.parametrize("tile_rows", [16, 100, 256, 0])
@pytest.mark.parametrize("name,mk,k,sym", [
    ("laplace3d_20", lambda: synth.laplace3d(20), 0, True),
    ("convdiff3d_12_ilu1", lambda: synth.convdiff3d(12), 1, True),
    ("random_2500_lower_a", lambda: synth.random_banded(2500, rng=np.random.default_rng(9)), 0, False),
    ("tridiag_777", lambda: synth.tridiag(777), 0, True),
    # two tiles: the larger (512 rows) imports nothing, the other does -- the LDS
    # room for the import list must follow the most imports of any tile
    ("laplace2d_30", lambda: synth.laplace2d(30), 0, True),
], ids=lambda v: v if isinstance(v, (str, int)) else "")
def test_apply_tiled_tile_sizes(jv, name, mk, k, sym, tile_rows):
    # tiles from 16 rows (most dependencies cross tiles) to one tile for the whole
    # matrix (every dependency in LDS); FP64, one and five right-hand sides
    A = mk()
    ilu = make(jv, A, k, sym, ("syncfree", "tiled"), tile_rows=tile_rows)
    ilu.factor(dev(A.val), k=k)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k, sym=sym)
    f = O.factor(an, A.val, k=k)
    rng = np.random.default_rng(tile_rows)
    for nrhs in (1, 5):
        b = rng.uniform(-1, 1, (A.n, nrhs)) if nrhs > 1 else rng.uniform(-1, 1, A.n)
        xr = O.apply(an, f.val, b)
        for _ in range(2):
            assert relerr(ilu.apply(dev(b)).cpu().numpy(), xr) <= 1e-12


def test_apply_tiled_retune_and_lds_limit(jv):
    A = synth.laplace3d(20)
    ilu = make(jv, A, 0, True, ("syncfree", "tiled"), tile_rows=512)
    ilu.factor(dev(A.val))
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    b = np.random.default_rng(17).uniform(-1, 1, A.n)
    xr = O.apply(an, f.val, b)
    assert relerr(ilu.apply(dev(b)).cpu().numpy(), xr) <= 1e-12
    for t in (64, 700):
        ilu.set_tuning("tile_rows", t)
        assert ilu.get_tuning("tile_rows") == t and ilu.info()["tile_rows"] == t
        assert relerr(ilu.apply(dev(b)).cpu().numpy(), xr) <= 1e-12
    # a tile whose values do not fit the LDS budget is refused, not run
    big = synth.laplace3d(48)
    ilu = make(jv, big, 0, True, ("syncfree", "tiled"), tile_rows=65536)
    ilu.factor(dev(big.val))
    with pytest.raises(jv.IluError) as e:
        ilu.apply(dev(np.ones(big.n)))
    assert e.value.code == 10   # ILU_ERR_UNSUPPORTED


def test_apply_tiled_blocks_per_cu_same_bits(jv):
    # the cap on resident tiles changes only how many run at once: every setting
    # gives the same bits, in FP64 and with the FP32 factor
    A = synth.laplace3d(24)
    ilu = make(jv, A, 0, True, ("syncfree", "tiled"), tile_rows=512)
    ilu.factor(dev(A.val))
    assert ilu.get_tuning("solve_blocks_per_cu") == 2
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    b = np.random.default_rng(29).uniform(-1, 1, A.n)
    xr = O.apply(an, f.val, b)
    ref = {p: ilu.apply(dev(b), prec=p).cpu().numpy() for p in ("f64", "f32")}
    assert relerr(ref["f64"], xr) <= 1e-12
    for bpc in (0, 1, 3, 8):
        ilu.set_tuning("solve_blocks_per_cu", bpc)
        for p in ("f64", "f32"):
            assert np.array_equal(ilu.apply(dev(b), prec=p).cpu().numpy().view(np.uint64), ref[p].view(np.uint64))
    with pytest.raises(jv.IluError):
        ilu.set_tuning("solve_blocks_per_cu", 9)


@pytest.mark.parametrize("name,mk,k,tau,tile_rows", [
    ("convdiff3d_14_ilu1_tau", lambda: synth.convdiff3d(14), 1, 1e-3, 512),
    ("convdiff3d_17_ilu1", lambda: synth.convdiff3d(17), 1, 0.0, 128),
    ("laplace3d_20x12x9_ilu2", lambda: synth.laplace3d(20, 12, 9), 2, 0.0, 256),
    ("laplace2d_50", lambda: synth.laplace2d(50), 0, 0.0, 256),
], ids=["convdiff3d_14_ilu1_tau", "convdiff3d_17_ilu1", "laplace3d_20x12x9_ilu2", "laplace2d_50"])
def test_lattice_tiles_same_bits(jv, name, mk, k, tau, tile_rows):
    # box tiles of a grid (sheared once fill appears) against the greedy tiles: the
    # tiled factor is bit-exact with the oracle on both, and the tiled applies give
    # the same bits, FP64 and FP32
    A = mk()
    ilu = make(jv, A, k, True, ("tiled", "tiled"), tile_rows=tile_rows)
    assert ilu.get_tuning("tile_lattice") == 1 and ilu.get_tuning("factor_tiled") == 1
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    f = O.factor(an, A.val, k=k, tau=tau)
    b = np.random.default_rng(31).uniform(-1, 1, A.n)
    xr = O.apply(an, f.val, b)
    out = {}
    for lat in (1, 0):
        ilu.set_tuning("tile_lattice", lat)
        assert ilu.get_tuning("tile_lattice") == lat
        ilu.factor(dev(A.val), k=k, tau=tau)
        lu, st = ilu.factor_values()
        np.testing.assert_array_equal(st, f.stat)
        assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
        out[lat] = {p: ilu.apply(dev(b), prec=p).cpu().numpy() for p in ("f64", "f32")}
    assert relerr(out[1]["f64"], xr) <= 1e-12
    for p in ("f64", "f32"):
        assert np.array_equal(out[1][p].view(np.uint64), out[0][p].view(np.uint64))


@pytest.mark.parametrize("tile_rows", [16, 100, 512])
@pytest.mark.parametrize("name,mk,k,sym", [
    ("laplace3d_20", lambda: synth.laplace3d(20), 0, True),
    ("convdiff3d_12_ilu1", lambda: synth.convdiff3d(12), 1, True),
    ("laplace2d_40_lower_a", lambda: synth.laplace2d(40), 0, False),
    ("tridiag_777", lambda: synth.tridiag(777), 0, True),
    ("random_sparse_300", lambda: synth.random_sparse(300, 0.01, np.random.default_rng(23)), 0, False),
], ids=lambda v: v if isinstance(v, (str, int)) else "")
def test_factor_tiled_bit_exact(jv, name, mk, k, sym, tile_rows):
    # the tiled factor on tiles from 16 rows (most dependencies imported) to whole
    # matrices; bit for bit the serial factor, twice in a row (re-armed buffers),
    # plain and modified, alternating on one handle
    A = mk()
    ilu = make(jv, A, k, sym, ("tiled", "tiled"), tile_rows=tile_rows)
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k, sym=sym)
    cases = [(False, 0.0), (True, 0.0), (True, 1e-2), (False, 1e-2), (False, 0.0)]
    want = {c: O.factor(an, A.val, k=k, milu=c[0], tau=c[1]) for c in set(cases)}
    if np.diff(an.lu_rp).max() <= 16:
        assert ilu.get_tuning("factor_tiled") == 1
    for milu, tau in cases:
        f = want[(milu, tau)]
        info = ilu.factor(dev(A.val), k=k, milu=milu, tau=tau)
        lu, st = ilu.factor_values()
        np.testing.assert_array_equal(st, f.stat)
        assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64)), f"max diff {np.abs(lu - f.val).max()}"
        assert info["n_dropped"] == int((f.stat == 1).sum())
