"""Full-size GPU parity in the launch configuration bench.py times (the default
schedules -- tiled where they apply -- and default lanes): the whole factor against
the oracle bit for bit and whole solves against the oracle, on the full-size
workloads, and the modified factor, the RCM preorder and the long-row factor at
full size."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def relerr(x, ref):
    x = np.asarray(x).reshape(len(x), -1)
    ref = np.asarray(ref).reshape(len(ref), -1)
    return float(max(np.abs(x[:, s] - ref[:, s]).max() / np.abs(ref[:, s]).max() for s in range(ref.shape[1])))


def test_laplace3d_128_full(jv):
    A, b = synth.workload(2)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.factor(dev(A.val), casts=("f32",))
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    lu, st = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    bp = np.ascontiguousarray(b[an.perm])
    x = ilu.apply(dev(bp), permuted=True).cpu().numpy()
    assert relerr(x, O.apply(an, f.val, bp, permuted=True)) <= 1e-12
    y = ilu.spmv(dev(bp), permuted=True).cpu().numpy()
    assert relerr(y, O.spmv(A.n, an.b_rp, an.b_ci, O.b_values(an, A.val), bp)) <= 1e-12
    x, info = ilu.pcg(dev(b), rtol=1e-10)
    assert info["true_relres"] <= 1e-10


def test_convdiff3d_96_ilu1_full(jv):
    A, b = synth.workload(3)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=1)
    ilu.factor(dev(A.val), k=1, tau=1e-3, casts=("f32", "bf16"))
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=1)
    f = O.factor(an, A.val, k=1, tau=1e-3)
    lu, st = ilu.factor_values()
    np.testing.assert_array_equal(st, f.stat)
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    x = ilu.apply(dev(b)).cpu().numpy()
    assert relerr(x, O.apply(an, f.val, b)) <= 1e-12
    for prec in ("f64", "f32", "bf16"):
        x, info = ilu.gmres(dev(b), rtol=1e-10, restart=30, prec=prec)
        assert info["true_relres"] <= 1e-10, (prec, info)


def test_random_1m_16rhs_full(jv):
    A, B = synth.workload(4)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.factor(dev(A.val), casts=("f32",))
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    # 4 of the 16 right-hand sides through the FP64 oracle (one oracle solve each)
    x = ilu.apply(dev(B)).cpu().numpy()
    cols = [0, 5, 10, 15]
    xr = O.apply(an, f.val, np.ascontiguousarray(B[:, cols]))
    assert relerr(x[:, cols], xr) <= 1e-12
    B32 = B.astype(np.float32)
    x32 = ilu.apply(dev(B32), prec="f32").cpu().numpy().astype(np.float64)
    xr32 = O.apply(an, O.cast_f32(f.val), np.ascontiguousarray(B32[:, cols]).astype(np.float64), prec="f32")
    assert relerr(x32[:, cols], xr32) <= 2.0 ** -12


def test_random_1m_tail_full(jv):
    # every level of random_1m holds fewer than 15 rows: the whole matrix is the
    # lower stage, streamed by one workgroup per right-hand side (16 at once)
    A, B = synth.workload(4)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, tail_min_rows=64)
    assert ilu.info()["tail_rows"] == A.n
    ilu.factor(dev(A.val), casts=("f32",))
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    # the factor streamed as well (the lower stage of the factor): the serial bits
    assert ilu.factor_tail()["level0"] >= 0
    ilu.set_tuning("factor_lower_stage", 1)
    ilu.factor(dev(A.val), casts=("f32",))
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    cols = [0, 7, 15]
    x = ilu.apply(dev(B)).cpu().numpy()
    assert relerr(x[:, cols], O.apply(an, f.val, np.ascontiguousarray(B[:, cols]))) <= 1e-12
    B32 = B.astype(np.float32)
    x32 = ilu.apply(dev(B32), prec="f32").cpu().numpy().astype(np.float64)
    xr32 = O.apply(an, O.cast_f32(f.val), np.ascontiguousarray(B32[:, cols]).astype(np.float64), prec="f32")
    assert relerr(x32[:, cols], xr32) <= 2.0 ** -12
    ilu.status()


def test_heavy_1m_natural_tail_full(jv):
    # the irregular matrix in its natural order (322k forward levels): the lower
    # stage with rows of up to 2053 entries split over steps of one wave
    A = synth.heavy_rows(1_000_000, rng=np.random.default_rng([6, 0]))
    b = np.ascontiguousarray(synth.rhs(A.n, 1, np.random.default_rng([6, 1]))).reshape(-1)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, tail_min_rows=64)
    assert ilu.info()["tail_rows"] > 0.9 * A.n
    ilu.factor(dev(A.val), casts=())
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    x = ilu.apply(dev(b)).cpu().numpy()
    assert relerr(x, O.apply(an, f.val, b)) <= 1e-12
    ilu.status()


def test_batch512_full(jv):
    mats, rhs = synth.workload(5)
    hb = jv.Ilu.batched(mats)
    vals = np.concatenate([m.val for m in mats])
    hb.factor(dev(vals), casts=("f32",))
    ro, _ = hb.batch_offsets()
    b = np.concatenate(rhs)
    x = hb.apply(dev(b)).cpu().numpy()
    x32 = hb.apply(dev(b.astype(np.float32)), prec="f32").cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    for i in sorted(rng.choice(len(mats), 12, replace=False)):
        M = mats[i]
        an = O.analyze(M.n, M.row_ptr, M.col_idx)
        f = O.factor(an, M.val)
        assert relerr(x[ro[i]:ro[i + 1]], O.apply(an, f.val, rhs[i])) <= 1e-12
        xr32 = O.apply(an, O.cast_f32(f.val), rhs[i].astype(np.float32).astype(np.float64), prec="f32")
        assert relerr(x32[ro[i]:ro[i + 1]], xr32) <= 2.0 ** -12


def test_batch512_adjoint_full(jv):
    # the backward of the 512-matrix batch: b-bar and the L/U-value gradients of 12
    # sampled matrices against the oracle's adjoint of each matrix alone (4 RHS)
    mats, rhs = synth.workload(5)
    hb = jv.Ilu.batched(mats)
    vals = np.concatenate([m.val for m in mats])
    hb.factor(dev(vals), casts=())
    ro, _ = hb.batch_offsets()
    b = np.concatenate(rhs)
    gx = np.random.default_rng(31).uniform(-1, 1, b.shape)
    x, y = hb.apply_ex(dev(b))
    gb, glu = hb.adjoint(dev(gx), x, y)
    x, y, gb, glu = (t.cpu().numpy() for t in (x, y, gb, glu))
    sb = hb.schedule()
    perm, rp = sb["perm"], sb["lu_row_ptr"]
    rng = np.random.default_rng(0)
    for i in sorted(rng.choice(len(mats), 12, replace=False)):
        M = mats[i]
        an = O.analyze(M.n, M.row_ptr, M.col_idx)
        f = O.factor(an, M.val)
        xr, yr = O.apply(an, f.val, rhs[i], want_y=True)
        assert relerr(x[ro[i]:ro[i + 1]], xr) <= 1e-12
        gbr, glur = O.adjoint(an, f.val, gx[ro[i]:ro[i + 1]], xr, yr)
        assert relerr(gb[ro[i]:ro[i + 1]], gbr) <= 1e-12
        # the batch keeps each matrix's rows (in its level order) and their entries
        rows = np.nonzero((perm >= ro[i]) & (perm < ro[i + 1]))[0]
        loc = an.iperm[perm[rows] - ro[i]]
        assert relerr(y[rows], yr[loc]) <= 1e-12
        got = np.concatenate([glu[rp[r]:rp[r + 1]] for r in rows])
        want = np.concatenate([glur[an.lu_rp[q]:an.lu_rp[q + 1]] for q in loc])
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_laplace3d_128_modified_full(jv):
    # modified ILU(0) at full size: bit-exact with the oracle, and since L U has A's
    # row sums, M^{-1} (A 1) is the vector of ones up to rounding
    A, b = synth.workload(2)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    ilu.factor(dev(A.val), casts=(), milu=True)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val, milu=True)
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    ones = torch.ones(A.n, dtype=torch.float64, device="cuda")
    x = ilu.apply(ilu.spmv(ones)).cpu().numpy()
    assert np.abs(x - 1.0).max() <= 1e-9
    _, info = ilu.pcg(dev(b), rtol=1e-10)
    assert info["true_relres"] <= 1e-10 and info["iters"] < 120


def test_random_1m_rcm_full(jv):
    # the reverse Cuthill-McKee preorder at full size: the library's permutation and
    # factor equal the oracle's composed analysis; FGMRES converges in the input ordering
    A, B = synth.workload(4)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, ordering="rcm")
    an = O.analyze(A.n, A.row_ptr, A.col_idx, rcm_order=True)
    s = ilu.schedule()
    np.testing.assert_array_equal(s["perm"], an.perm)
    np.testing.assert_array_equal(s["level_ptr"], an.level_ptr)
    ilu.factor(dev(A.val), casts=())
    f = O.factor(an, A.val)
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    b = np.ascontiguousarray(B[:, 3])
    x = ilu.apply(dev(b)).cpu().numpy()
    assert relerr(x, O.apply(an, f.val, b)) <= 1e-12
    _, info = ilu.gmres(dev(b), rtol=1e-10, restart=30)
    assert info["true_relres"] <= 1e-10


def test_heavy_1m_long_rows_full(jv):
    # 10^6 irregular rows, 1% of them with 256..2048 entries: the long-row factor bit
    # for bit, the applies and the split spmv against the oracle
    A = synth.heavy_rows(1_000_000, rng=np.random.default_rng([6, 0]))
    b = np.ascontiguousarray(synth.rhs(A.n, 1, np.random.default_rng([6, 1]))).reshape(-1)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, ordering="rcm")
    an = O.analyze(A.n, A.row_ptr, A.col_idx, rcm_order=True)
    assert np.diff(an.lu_rp).max() > 64
    ilu.factor(dev(A.val), casts=())
    f = O.factor(an, A.val)
    lu, _ = ilu.factor_values()
    assert np.array_equal(lu.view(np.uint64), f.val.view(np.uint64))
    x = ilu.apply(dev(b)).cpu().numpy()
    assert relerr(x, O.apply(an, f.val, b)) <= 1e-12
    y = ilu.spmv(dev(b)).cpu().numpy()
    yr = O.spmv(A.n, A.row_ptr, A.col_idx, A.val, b)
    assert relerr(y, yr) <= 1e-12
