"""The factor's lower stage (host plan, CPU): what the streaming factor kernel is
told to do, replayed step by step in numpy as the kernel does it (the ring of
recent rows' U parts, U values of older rows and of rows before the tail read from
the factor buffer, lane groups), must give the serial up-looking factor bit for bit,
read only values that exist at that point (a value from the factor buffer at least
q steps old, a ring slot still holding its row), and cover every tail row once."""
import numpy as np
import pytest

import oracle as O
import synth


@pytest.fixture(scope="module")
def jv():
    import paper_1812_06160_amd as jv_mod
    jv_mod.load()
    return jv_mod


def replay(P, an, a, fval):
    """The kernel's arithmetic on plan P; rows before the tail from the serial factor."""
    n, pos0, q, W, umax = an.n, P["pos0"], P["q"], P["ring_rows"], P["umax"]
    lu_rp, lu_ci, diag, src = an.lu_rp, an.lu_ci, an.diag_pos, an.lu_src
    pub = np.full(len(lu_ci), np.nan)
    pub[:lu_rp[pos0]] = fval[:lu_rp[pos0]]
    done_step = np.full(n, -1)            # step that computed a tail row
    ring = np.full(W * umax, np.nan)
    owner = np.full(W * umax, -1)
    seen = np.zeros(n, int)
    hdr, rows, lsrc, match, lmap = P["hdr"], P["rows"], P["lsrc"], P["match"], P["lmap"]
    for s in range(P["nsteps"]):
        r0, nrows, kmax, _ = hdr[s]
        assert 1 <= nrows <= 64 and kmax <= 16
        lanes = lmap[s]
        used = 0
        for k in range(nrows):
            r, p0, packed, rbase, loff, moff = rows[r0 + k][:6]
            ln, K, g, lane0 = packed & 255, (packed >> 8) & 255, (packed >> 16) & 255, (packed >> 24) & 255
            assert ln <= 1 << g and lane0 % (1 << g) == 0 and lane0 + (1 << g) <= 64 and K <= kmax
            assert (lanes[lane0:lane0 + (1 << g)] == k).all()
            used += 1 << g
            assert p0 == lu_rp[r] and ln == lu_rp[r + 1] - lu_rp[r] and K == diag[r] - lu_rp[r]
            assert rbase == (r % W) * umax
            seen[r] += 1
            v = np.array([a[src[p0 + t]] if src[p0 + t] >= 0 else 0.0 for t in range(ln)])
            for e in range(K):
                c = lu_ci[p0 + e]
                sv = lsrc[loff + e]
                u = {}
                for t in range(ln):
                    j = match[moff + e * ln + t]
                    if t < e:
                        assert j == 255
                        continue
                    if j == 255:
                        continue
                    assert (t == e) == (j == 0)
                    if sv >= 0:
                        assert c >= pos0 and sv == (c % W) * umax
                        assert owner[sv + j] == c, "ring slot holds another row"
                        u[t] = ring[sv + j]
                    else:
                        ge = -sv - 1 + j
                        assert -sv - 1 == diag[c]
                        assert not np.isnan(pub[ge]), "read of a value not yet computed"
                        if c >= pos0:
                            assert done_step[c] <= s - q, "global read of a row fewer than q steps old"
                        u[t] = pub[ge]
                assert e in u
                v[e] = v[e] / u[e]
                for t, ut in u.items():
                    if t > e:
                        v[t] = v[t] - v[e] * ut
            pub[p0:p0 + ln] = v
            for t in range(K, ln):
                ring[rbase + t - K] = v[t]
                owner[rbase + t - K] = r
        assert (lanes[used:] == 255).all()
        for k in range(nrows):
            done_step[rows[r0 + k][0]] = s
    return pub, seen


@pytest.mark.parametrize("name,mk,k,M", [
    ("random_banded_4000_all", lambda: synth.random_banded(4000, rng=np.random.default_rng(4)), 0, 65536),
    ("random_banded_3000_ilu1", lambda: synth.random_banded(3000, band=2, rnd=2, rng=np.random.default_rng(6)), 1,
     65536),
    ("laplace2d_150_upper_and_tail", lambda: synth.laplace2d(150), 0, 65),
    ("tridiag_2000_chain", lambda: synth.tridiag(2000), 0, 65536),
    ("laplace2d_60_ilu1", lambda: synth.laplace2d(60), 1, 65536),
], ids=lambda v: v if isinstance(v, str) else "")
def test_factor_tail_plan_replays_the_factor(jv, name, mk, k, M):
    A = mk()
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k)
    f = O.factor(an, A.val, k=k)
    assert f.status == O.OK
    ilu = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k, host_only=True, tail_min_rows=M)
    P = ilu.factor_tail()
    T = ilu.tail(0)
    assert P["level0"] == T["level0"] >= 0 and P["pos0"] == T["pos0"]
    assert 2 <= P["q"] <= 6 and P["ring_rows"] * P["umax"] <= 8192
    pub, seen = replay(P, an, A.val, f.val)
    assert (seen[:P["pos0"]] == 0).all() and (seen[P["pos0"]:] == 1).all()
    assert np.array_equal(pub.view(np.uint64), f.val.view(np.uint64))


def test_factor_tail_plan_absent(jv):
    # no solve tail: no factor tail; rows with more than 16 L entries: none either
    A = synth.laplace3d(12)
    assert jv.Ilu(A.n, A.row_ptr, A.col_idx, host_only=True, tail_min_rows=65536).factor_tail()["level0"] == -1
    B = synth.random_banded(3000, band=4, rnd=4, rng=np.random.default_rng(6))   # ILU(1): L parts up to 35
    ilu = jv.Ilu(B.n, B.row_ptr, B.col_idx, k_max=1, host_only=True, tail_min_rows=65536)
    an = O.analyze(B.n, B.row_ptr, B.col_idx, k_max=1)
    assert ilu.tail(0)["nsteps"] > 0 and (an.diag_pos - an.lu_rp[:-1]).max() > 16
    assert ilu.factor_tail()["level0"] == -1
