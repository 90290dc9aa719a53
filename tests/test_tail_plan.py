"""The lower stage of the solves (host plan, CPU): what the streaming kernel is told
to do, replayed step by step in numpy exactly as the kernel does it (ring of recent
results, values fetched from the published buffer, lane groups, carried partial
sums of split rows), must reproduce a serial substitution, read only values that
exist at that point, and cover every tail row and every dependency once."""
import numpy as np
import pytest

import oracle as O
import synth

W, Q, J = 2048, 24, 2   # ring slots, steps staged ahead, dependencies per lane


@pytest.fixture(scope="module")
def jv():
    import paper_1812_06160_amd as jv_mod
    jv_mod.load()
    return jv_mod


def serial(an, val, b, direction):
    """Forward (unit L) or backward (U) substitution in the level ordering."""
    n = an.n
    x = np.zeros(n)
    rows = range(n) if direction == 0 else range(n - 1, -1, -1)
    for r in rows:
        lo, hi = (an.lu_rp[r], an.diag_pos[r]) if direction == 0 else (an.diag_pos[r] + 1, an.lu_rp[r + 1])
        acc = float(np.dot(val[lo:hi], x[an.lu_ci[lo:hi]]))
        x[r] = b[r] - acc if direction == 0 else (b[r] - acc) / val[an.diag_pos[r]]
    return x


def replay(ilu, an, val, b, direction, upper_done):
    """The streaming kernel's arithmetic on the plan; upper_done holds the rows
    before the tail (solved by the upper stage), NaN elsewhere."""
    T = ilu.tail(direction)
    hdr, rec = T["hdr"], T["rec"]
    pub = upper_done.copy()
    emit_step = {}
    ring = np.full(W, np.nan)
    owner = np.full(W, -1)
    carry = 0.0
    seen = {}
    far = fetched = 0
    for s in range(T["nsteps"]):
        off, h, nent = int(hdr[s, 0]), int(hdr[s, 1]), int(hdr[s, 2])
        assert off % 4 == 0
        nrows, nlanes, gmax, flags = h & 255, (h >> 8) & 255, (h >> 16) & 255, h >> 24
        assert nent == nlanes * J and 1 <= nrows <= 32 and nlanes <= 64
        rw = rec[off:off + 4 * nrows].reshape(nrows, 4)
        lanes = rec[off + 4 * nrows: off + 4 * nrows + nlanes]
        ep = rec[off + 4 * nrows + nlanes: off + 4 * nrows + nlanes + nent]
        ec = rec[off + 4 * nrows + nlanes + nent: off + 4 * nrows + nlanes + 2 * nent]
        lane_sum = np.zeros(64)
        for e in range(nent):
            if ep[e] < 0:
                assert ec[e] == -1
                continue
            lane = e % nlanes
            k = lanes[lane] & 255
            r = rw[k, 0]
            c = an.lu_ci[ep[e]]
            lo, hi = (an.lu_rp[r], an.diag_pos[r]) if direction == 0 else (an.diag_pos[r] + 1, an.lu_rp[r + 1])
            assert lo <= ep[e] < hi, "entry outside its row's part"
            seen.setdefault(int(r), []).append(int(ep[e]))
            if ec[e] >= W:
                assert ec[e] - W == c
                assert not np.isnan(pub[c]), "read of a value not yet computed"
                if c in emit_step:
                    assert emit_step[c] < s
                    far += emit_step[c] <= s - Q     # staged without waiting for it
                    fetched += 1
                x = pub[c]
            else:
                assert owner[ec[e]] == c, "ring slot holds another row"
                x = ring[ec[e]]
            lane_sum[lane] += val[ep[e]] * x
        # lane groups: aligned, packed, one leader each
        for k in range(nrows):
            members = [ln for ln in range(nlanes) if (lanes[ln] & 255) == k]
            g = (lanes[members[0]] >> 8) & 255
            assert len(members) == 1 << g and members[0] % (1 << g) == 0 and g <= gmax
            assert [(lanes[ln] >> 16) & 1 for ln in members] == [1] + [0] * (len(members) - 1)
            acc = float(sum(lane_sum[ln] for ln in members))
            r = int(rw[k, 0])
            if flags & 1:
                acc += carry
            if not flags & 2:
                assert nrows == 1
                carry = acc
                continue
            v = b[r] - acc
            if direction == 1:
                v = v / val[an.diag_pos[r]]
            slot = int(rw[k, 1])
            ring[slot] = v
            owner[slot] = r
            assert np.isnan(pub[r]), "row emitted twice"
            pub[r] = v
            emit_step[r] = s
            assert rw[k, 2] == an.perm[r] and rw[k, 3] == an.diag_pos[r]
    # tail values fetched from the published buffer were computed at least Q steps
    # earlier (when the tail's levels are narrow, as here, always)
    assert far == fetched
    return pub, seen, T


@pytest.mark.parametrize("name,mk,k,M", [
    ("random_banded_4000", lambda: synth.random_banded(4000, rng=np.random.default_rng(3)), 0, 16),
    ("random_banded_4000_all", lambda: synth.random_banded(4000, rng=np.random.default_rng(4)), 0, 65536),
    ("laplace3d_16", lambda: synth.laplace3d(16), 0, 64),
    ("convdiff3d_10_ilu1", lambda: synth.convdiff3d(10), 1, 40),
    ("heavy_3000_long_rows", lambda: synth.heavy_rows(3000, heavy_len=(150, 700), heavy_frac=0.03,
                                                      rng=np.random.default_rng(5)), 0, 65536),
], ids=lambda v: v if isinstance(v, str) else "")
def test_tail_plan_replays_the_solve(jv, name, mk, k, M):
    A = mk()
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    f = O.factor(an, A.val, k=k)
    assert f.status == O.OK
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k, host_only=True, tail_min_rows=M)
    rng = np.random.default_rng(1)
    b = rng.uniform(-1, 1, A.n)
    for direction in (0, 1):
        T = ilu.tail(direction)
        lp = an.level_ptr if direction == 0 else an.ulevel_ptr
        sizes = np.diff(lp)
        if T["nsteps"] == 0:
            continue
        t = T["level0"]
        # the longest suffix of levels with fewer than M rows (at least 64 levels)
        assert (sizes[t:] < M).all() and (t == 0 or sizes[t - 1] >= M) and len(sizes) - t >= 64
        assert T["pos0"] == lp[t]
        want = serial(an, f.val, b, direction)
        order = np.arange(A.n) if direction == 0 else an.ulevel_rows
        upper = np.full(A.n, np.nan)
        upper[order[:T["pos0"]]] = want[order[:T["pos0"]]]
        got, seen, _ = replay(ilu, an, f.val, b, direction, upper)
        # every tail row once, with each of its dependencies once
        tail_rows = order[T["pos0"]:]
        assert not np.isnan(got[tail_rows]).any()
        for r in tail_rows:
            lo, hi = (an.lu_rp[r], an.diag_pos[r]) if direction == 0 else (an.diag_pos[r] + 1, an.lu_rp[r + 1])
            assert sorted(seen.get(int(r), [])) == list(range(lo, hi))
        assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


def test_tail_plan_off_and_too_short(jv):
    A = synth.laplace3d(12)                      # 34 levels: under the 64-level minimum
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, host_only=True, tail_min_rows=65536)
    assert ilu.tail(0)["nsteps"] == 0 and ilu.info()["tail_rows"] == 0
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, host_only=True)
    assert ilu.tail(0)["level0"] == -1
    B = synth.random_banded(3000, rng=np.random.default_rng(9))
    ilu = jv.Ilu(B.n, B.row_ptr, B.col_idx, host_only=True, tail_min_rows=65536)
    assert ilu.info()["tail_rows"] == B.n and ilu.tail(0)["pos0"] == 0


def test_tail_plan_with_an_upper_stage(jv):
    # a 150 x 150 grid: 299 levels, the last 64 of fewer than 65 rows form the tail,
    # the 235 before it stay in the upper stage
    A = synth.laplace2d(150)
    an = O.analyze(A.n, A.row_ptr, A.col_idx)
    f = O.factor(an, A.val)
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, host_only=True, tail_min_rows=65)
    b = np.random.default_rng(2).uniform(-1, 1, A.n)
    for direction in (0, 1):
        T = ilu.tail(direction)
        assert T["level0"] == 235 and T["pos0"] == A.n - 64 * 65 // 2
        want = serial(an, f.val, b, direction)
        order = np.arange(A.n) if direction == 0 else an.ulevel_rows
        upper = np.full(A.n, np.nan)
        upper[order[:T["pos0"]]] = want[order[:T["pos0"]]]
        got, _, _ = replay(ilu, an, f.val, b, direction, upper)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
