"""CPU checks of the library's host side: exported symbols, host-only analysis
bit-exact against the oracle, and the error paths of the C ABI that need no GPU."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import synth
import paper_1812_06160_amd as jv
from paper_1812_06160_amd import _lib as L


def test_library_exports_every_declared_symbol():
    import os
    import re
    lib = jv.load()
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "javelin.h")).read()
    declared = set(re.findall(r"^\s*(?:ilu_status|const char \*)\s*(ilu_\w+)\s*\(", hdr, re.M))
    assert declared == set(L.SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.ilu_version().startswith(b"javelin")
    assert lib.ilu_status_str(5) == b"ILU_ERR_ZERO_PIVOT"


def host_ilu(A, k_max=0, sym=True, ordering="natural"):
    return jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k_max, pattern="sym" if sym else "a", host_only=True,
                  ordering=ordering)


def compare_schedule(A, k_max, sym, ordering="natural"):
    an = O.analyze(A.n, A.row_ptr, A.col_idx, k_max=k_max, sym=sym, rcm_order=ordering == "rcm")
    h = host_ilu(A, k_max, sym, ordering)
    s = h.schedule()
    assert h.info()["n_levels"] == an.n_levels
    assert h.info()["n_ulevels"] == an.n_ulevels
    np.testing.assert_array_equal(s["level_ptr"], an.level_ptr)
    np.testing.assert_array_equal(s["perm"], an.perm)
    np.testing.assert_array_equal(s["lu_row_ptr"], an.lu_rp)
    np.testing.assert_array_equal(s["lu_col_idx"], an.lu_ci)
    np.testing.assert_array_equal(s["diag_pos"], an.diag_pos)
    np.testing.assert_array_equal(s["fill_lev"], an.lu_lev)
    np.testing.assert_array_equal(s["lu_src"], an.lu_src)
    np.testing.assert_array_equal(s["ulevel_ptr"], an.ulevel_ptr)
    np.testing.assert_array_equal(s["ulevel_rows"], an.ulevel_rows)
    np.testing.assert_array_equal(s["b_row_ptr"], an.b_rp)
    np.testing.assert_array_equal(s["b_col_idx"], an.b_ci)
    return h, an


@pytest.mark.parametrize("seed", range(10))
def test_host_analysis_bit_exact_random(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(1, 200))
    A = synth.random_sparse(n, float(rng.uniform(0.005, 0.08)), rng,
                            symmetric_pattern=bool(seed % 3 == 0), drop_diag_frac=0.3 if seed % 4 == 1 else 0.0)
    compare_schedule(A, k_max=seed % 4, sym=bool(seed % 2))


@pytest.mark.parametrize("wid,k", [(1, 0), (2, 0), (3, 1), (4, 0)])
def test_host_analysis_bit_exact_workloads_small(wid, k):
    A, _ = synth.workload(wid, scale=0.1 if wid != 4 else 0.002)
    compare_schedule(A, k_max=k, sym=True)
    compare_schedule(A, k_max=k, sym=False)


@pytest.mark.parametrize("seed", range(8))
def test_host_analysis_rcm_bit_exact(seed):
    # the library's reverse Cuthill-McKee preorder and the composed analysis equal
    # the oracle's (several components, missing diagonals, both patterns, k <= 2)
    rng = np.random.default_rng(1300 + seed)
    n = int(rng.integers(2, 300))
    A = synth.random_sparse(n, float(rng.uniform(0.002, 0.05)), rng, symmetric_pattern=bool(seed % 3 == 0),
                            drop_diag_frac=0.2 if seed % 4 == 1 else 0.0)
    compare_schedule(A, k_max=seed % 3, sym=bool(seed % 2), ordering="rcm")


@pytest.mark.parametrize("wid,k", [(1, 0), (2, 0), (3, 1), (4, 0)])
def test_host_analysis_rcm_workloads_small(wid, k):
    A, _ = synth.workload(wid, scale=0.1 if wid != 4 else 0.002)
    compare_schedule(A, k_max=k, sym=True, ordering="rcm")


def test_rcm_option_errors():
    # an unknown ordering is an argument error; a batched handle refuses a preorder
    A = synth.laplace2d(5)
    assert _analyze_raw(A.n, A.row_ptr, A.col_idx, ordering=7) == L.ERR_ARG
    assert _analyze_raw(A.n, A.row_ptr, A.col_idx, ordering=L.ORDER_RCM) == L.OK
    lib = jv.load()
    rp = np.ascontiguousarray(A.row_ptr, np.int32)
    ci = np.ascontiguousarray(A.col_idx, np.int32)
    arr = (L.Csr * 1)(L.Csr(A.n, int(rp[-1]), rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p)))
    opts = L.AnalyzeOpts(0, 0, 1, 0, L.ORDER_RCM)
    h = C.c_void_p()
    assert lib.ilu_analyze_batched(1, arr, C.byref(opts), C.byref(h)) == L.ERR_UNSUPPORTED


def test_host_analysis_batched_is_block_diagonal():
    mats, _ = synth.workload(5, scale=0.06)
    mats = mats[:6]
    hb = jv.Ilu.batched(mats, host_only=True)
    ro, zo = hb.batch_offsets()
    assert ro.tolist() == np.concatenate([[0], np.cumsum([m.n for m in mats])]).tolist()
    assert zo.tolist() == np.concatenate([[0], np.cumsum([m.nnz for m in mats])]).tolist()
    # the merged levels equal the per-matrix levels, level by level
    s = hb.schedule()
    lv = np.repeat(np.arange(len(s["level_ptr"]) - 1), np.diff(s["level_ptr"]))
    level_of = np.empty(ro[-1], np.int64)
    level_of[s["perm"]] = lv
    for i, M in enumerate(mats):
        an = O.analyze(M.n, M.row_ptr, M.col_idx)
        np.testing.assert_array_equal(level_of[ro[i]:ro[i + 1]], an.level)
    assert hb.info()["n_levels"] == max(O.analyze(M.n, M.row_ptr, M.col_idx).n_levels for M in mats)


@pytest.mark.slow
def test_host_analysis_full_laplace3d():
    A, _ = synth.workload(2)
    h = host_ilu(A)
    I = h.info()
    assert (I["n_levels"], I["level_min"], I["level_max"], I["level_median"]) == (382, 1, 12288, 4656.0)
    assert I["nnz_lu"] == 14_581_760


def _analyze_raw(n, rp, ci, k_max=0, pattern=0, host_only=1, reserved=0, ordering=0):
    lib = jv.load()
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci, np.int32)
    csr = L.Csr(n, int(rp[-1]) if rp.size else 0, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p))
    opts = L.AnalyzeOpts(k_max, pattern, host_only, 0, ordering)
    opts.reserved[0] = reserved
    h = C.c_void_p()
    code = lib.ilu_analyze(C.byref(csr), C.byref(opts), C.byref(h))
    if code == 0:
        lib.ilu_destroy(h)
    return code


def test_analyze_error_paths():
    ok_rp, ok_ci = [0, 2, 4], [0, 1, 0, 1]
    assert _analyze_raw(2, ok_rp, ok_ci) == L.OK
    assert _analyze_raw(2, [0, 2, 4], [1, 0, 0, 1]) == L.ERR_CSR          # unsorted
    assert _analyze_raw(2, [0, 2, 4], [0, 0, 0, 1]) == L.ERR_CSR          # duplicate
    assert _analyze_raw(2, [0, 2, 4], [0, 2, 0, 1]) == L.ERR_CSR          # out of range
    assert _analyze_raw(2, [0, 3, 2], [0, 1, 0, 1]) == L.ERR_CSR          # decreasing row_ptr
    assert _analyze_raw(0, [0], []) == L.ERR_ARG                          # n = 0
    assert _analyze_raw(2, ok_rp, ok_ci, k_max=-1) == L.ERR_ARG
    assert _analyze_raw(2, ok_rp, ok_ci, pattern=7) == L.ERR_ARG
    assert _analyze_raw(2, ok_rp, ok_ci, reserved=1) == L.ERR_ARG
    assert _analyze_raw(2, ok_rp, ok_ci, host_only=2) == L.ERR_ARG
    assert _analyze_raw(2, ok_rp, ok_ci, pattern=L.PATTERN_UPPER_A) == L.ERR_ARG   # device level sets only


def test_device_analysis_argument_errors():
    # rejected before any device work, so these run without a GPU
    lib = jv.load()
    p = C.c_void_p(64)
    nl = C.c_int32(0)
    assert lib.ilu_levels_device(0, 0, p, p, 0, p, p, p, C.byref(nl), None) == L.ERR_ARG         # n = 0
    assert lib.ilu_levels_device(4, -1, p, p, 0, p, p, p, C.byref(nl), None) == L.ERR_ARG        # nnz < 0
    assert lib.ilu_levels_device(4, 4, p, None, 0, p, p, p, C.byref(nl), None) == L.ERR_ARG      # no columns
    assert lib.ilu_levels_device(4, 4, p, p, 3, p, p, p, C.byref(nl), None) == L.ERR_ARG         # pattern
    assert lib.ilu_levels_device(4, 4, p, p, 0, None, p, p, C.byref(nl), None) == L.ERR_ARG      # no level_ptr
    assert lib.ilu_levels_device(4, 4, p, p, 0, p, p, p, None, None) == L.ERR_ARG                # no n_levels
    assert lib.ilu_permute_device(4, 4, p, p, None, p, p, p, p, p, None) == L.ERR_ARG            # no perm
    assert lib.ilu_permute_device(4, 4, p, p, p, p, p, None, p, p, None) == L.ERR_ARG            # no out columns
    assert lib.ilu_permute_device(1 << 30, 4, p, p, p, p, p, p, p, p, None) == L.ERR_ARG         # n too large
    assert lib.ilu_transpose_device(4, 4, p, p, p, p, None, p, None) == L.ERR_ARG                 # no t_map
    assert lib.ilu_transpose_device(4, 1 << 31, p, p, p, p, p, p, None) == L.ERR_ARG              # nnz too large


def test_numeric_calls_on_host_only_handle_report_state():
    lib = jv.load()
    A = synth.laplace2d(4)
    h = host_ilu(A)
    fi = L.FactorInfo()
    assert lib.ilu_factor(h.h, None, 0, 0.0, 0, C.byref(fi), None) == L.ERR_STATE
    assert lib.ilu_apply(h.h, C.c_void_p(8), C.c_void_p(8), 1, 1, 0, 0, 0, None) == L.ERR_STATE
    assert lib.ilu_spmv(h.h, 1.0, C.c_void_p(8), 0.0, C.c_void_p(16), 1, 1, 0, None) == L.ERR_STATE
    si = L.SolveInfo()
    assert lib.ilu_solve_pcg(h.h, C.c_void_p(8), C.c_void_p(16), 1e-10, 10, 0, 0, C.byref(si), None) == L.ERR_STATE
    assert lib.ilu_tune(h.h, None, 1, None, 0, None, None) == L.ERR_STATE
    buf = C.create_string_buffer(256)
    lib.ilu_last_error(buf, 256)
    assert b"factor" in buf.value or b"state" in buf.value.lower() or buf.value
    assert lib.ilu_set_schedule(h.h, 1, 2, 0, 8) == L.OK
    assert lib.ilu_set_schedule(h.h, 5, 0, 0, 0) == L.ERR_ARG
    assert lib.ilu_set_schedule(h.h, 0, 0, 3, 0) == L.ERR_ARG


# ---------------------------------------------------------------------------------
# Tiles of the tiled triangular solves (host side)
# ---------------------------------------------------------------------------------

def _check_tiles(h, n):
    """Every row once per direction; tile order topological; no dependency inside a
    run of 16 positions; slot encoding of every off-diagonal entry."""
    sch = h.schedule()
    rp, ci, dg = sch["lu_row_ptr"], sch["lu_col_idx"], sch["diag_pos"]
    for d in (0, 1):
        ptr, row, sci = h.tiles(d)
        assert ptr[0] == 0 and np.all(np.diff(ptr) > 0) and np.all(np.diff(ptr) % 16 == 0)
        real = row[row >= 0]
        assert len(real) == n and len(np.unique(real)) == n
        tile_of = np.empty(n, np.int64)
        pos = np.empty(n, np.int64)
        slot = np.empty(n, np.int64)
        nrows = np.empty(len(ptr) - 1, np.int64)
        for t in range(len(ptr) - 1):
            seg = row[ptr[t]:ptr[t + 1]]
            m = seg >= 0
            tile_of[seg[m]] = t
            pos[seg[m]] = np.nonzero(m)[0]
            slot[seg[m]] = np.arange(m.sum())
            nrows[t] = m.sum()
        imports = {}
        for r in range(n):
            lo, hi = (rp[r], dg[r]) if d == 0 else (dg[r] + 1, rp[r + 1])
            t = tile_of[r]
            for p in range(lo, hi):
                c = ci[p]
                assert tile_of[c] <= t
                if tile_of[c] == t:
                    assert sci[p] == slot[c]
                    assert pos[c] // 16 < pos[r] // 16
                else:
                    assert sci[p] >= nrows[t]
                    assert imports.setdefault((t, c), sci[p]) == sci[p]
            assert sci[dg[r]] == -1
        per_tile = {}
        for (t, c), s in imports.items():
            per_tile.setdefault(t, []).append(s)
        for t, sl in per_tile.items():   # import slots of a tile are distinct and contiguous
            assert sorted(sl) == list(range(nrows[t], nrows[t] + len(sl)))


@pytest.mark.parametrize("name,mk,k,sym,tile_rows", [
    ("laplace3d_12", lambda: synth.laplace3d(12), 0, True, 256),
    ("laplace2d_30", lambda: synth.laplace2d(30), 0, True, 100),
    ("convdiff3d_8_ilu1", lambda: synth.convdiff3d(8), 1, True, 128),
    ("random_1500_lower_a", lambda: synth.random_banded(1500, rng=np.random.default_rng(21)), 0, False, 200),
    ("random_sparse_ilu2", lambda: synth.random_sparse(300, 0.015, np.random.default_rng(7)), 2, False, 64),
    ("tridiag_200", lambda: synth.tridiag(200), 0, True, 16),
    ("one_tile", lambda: synth.laplace2d(10), 0, True, 4096),
], ids=lambda v: v if isinstance(v, str) else "")
def test_tiles_invariants(name, mk, k, sym, tile_rows):
    A = mk()
    h = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k, pattern="sym" if sym else "a", host_only=True,
               tile_rows=tile_rows)
    info = h.info()
    assert info["tile_rows"] == tile_rows and info["max_tile"] <= tile_rows
    _check_tiles(h, A.n)


def test_tiles_are_cubes_on_grids():
    # greedy growth gives compact blocks without coordinates: 8^3 cubes at 512 rows
    # on a 3D 7-point grid, 16 x 16 squares at 256 rows on a 2D 5-point grid
    for A, m, t, side, dims in [(synth.laplace3d(16), 16, 512, 8, 3), (synth.laplace2d(64), 64, 256, 16, 2)]:
        h = jv.Ilu(A.n, A.row_ptr, A.col_idx, host_only=True, tile_rows=t)
        perm = h.schedule()["perm"]
        for d in (0, 1):
            ptr, row, _ = h.tiles(d)
            assert len(ptr) - 1 == A.n // t
            for q in range(len(ptr) - 1):
                o = perm[row[ptr[q]:ptr[q + 1]][row[ptr[q]:ptr[q + 1]] >= 0]]
                coords = [(o // m ** a) % m // side for a in range(dims)]
                assert len(o) == t and all(len(np.unique(c)) == 1 for c in coords)


@pytest.mark.parametrize("name,mk,k,ordering,on", [
    ("laplace3d_16", lambda: synth.laplace3d(16), 0, "natural", 1),
    ("convdiff3d_12_ilu1", lambda: synth.convdiff3d(12), 1, "natural", 1),
    ("laplace2d_30", lambda: synth.laplace2d(30), 0, "natural", 1),
    ("laplace3d_16x10x9", lambda: synth.laplace3d(16, 10, 9), 2, "natural", 1),
    ("laplace3d_6_too_small", lambda: synth.laplace3d(6), 0, "natural", 0),
    ("laplace3d_16_rcm", lambda: synth.laplace3d(16), 0, "rcm", 0),
    ("random_1500", lambda: synth.random_banded(1500, rng=np.random.default_rng(21)), 0, "natural", 0),
    ("tridiag_200", lambda: synth.tridiag(200), 0, "natural", 0),
], ids=lambda v: v if isinstance(v, str) else "")
def test_lattice_tiles_detection(name, mk, k, ordering, on):
    # box tiles only where the factor pattern is a grid stencil in natural order with
    # every extent above 7; everything else keeps the greedy growth
    A = mk()
    h = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=k, host_only=True, tile_rows=128, ordering=ordering)
    assert h.get_tuning("tile_lattice") == on
    _check_tiles(h, A.n)
    if on:
        h.set_tuning("tile_lattice", 0)
        assert h.get_tuning("tile_lattice") == 0
        _check_tiles(h, A.n)
        h.set_tuning("tile_lattice", 1)
        assert h.get_tuning("tile_lattice") == 1
    with pytest.raises(jv.IluError):
        h.set_tuning("tile_lattice", 2)


def _with_extra_pairs(A, pairs):
    # symmetric extra couplings (i, j) added to a CSR pattern
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    r = np.concatenate([rows] + [[i, j] for i, j in pairs])
    c = np.concatenate([A.col_idx] + [[j, i] for i, j in pairs])
    v = np.concatenate([A.val, np.full(2 * len(pairs), -0.01)])
    return synth.csr_from_coo(A.n, r, c, v)


def test_lattice_tiles_reject_non_grid_couplings():
    # one long-range coupling breaks the grid reading (a factor entry joins rows far
    # apart on an axis): the greedy growth takes over and the tiles stay valid; a
    # coupling within the stencil's reach (a diagonal neighbour) keeps the boxes
    m = 12
    A = synth.laplace3d(m)
    far = _with_extra_pairs(A, [(5 * m * m + 3, 5 * m * m + 3 + 6 * m + 7)])
    h = jv.Ilu(far.n, far.row_ptr, far.col_idx, host_only=True, tile_rows=128)
    assert h.get_tuning("tile_lattice") == 0
    _check_tiles(h, far.n)
    near = _with_extra_pairs(A, [(5 * m * m + 3 * m + 3, 5 * m * m + 4 * m + 4)])
    h = jv.Ilu(near.n, near.row_ptr, near.col_idx, host_only=True, tile_rows=128)
    assert h.get_tuning("tile_lattice") == 1
    _check_tiles(h, near.n)


def test_lattice_tiles_sheared_boxes_ilu1():
    # ILU(1) on a 7-point grid makes row (x, y, z) depend on (x+1, y-1, z),
    # (x+1, y, z-1) and (x, y+1, z-1) besides its three lower neighbours: no dependency
    # decreases z, y+z or x+y+z, and the tiles are 8 x 8 x 8 boxes of those three
    # functionals (clipped by the grid), taken in wavefront order
    m = 16
    A = synth.convdiff3d(m)
    h = jv.Ilu(A.n, A.row_ptr, A.col_idx, k_max=1, host_only=True, tile_rows=512)
    assert h.get_tuning("tile_lattice") == 1
    perm = h.schedule()["perm"]
    for d in (0, 1):
        ptr, row, _ = h.tiles(d)
        total = 0
        for t in range(len(ptr) - 1):
            o = perm[row[ptr[t]:ptr[t + 1]][row[ptr[t]:ptr[t + 1]] >= 0]]
            x, y, z = o % m, (o // m) % m, o // (m * m)
            total += len(o)
            for f in (z, y + z, x + y + z):
                assert np.ptp(f) < 8
        assert total == A.n
    # 3D 7-point ILU(0) at 512 rows: the boxes are the axis-aligned 8^3 cubes
    A = synth.laplace3d(m)
    h = jv.Ilu(A.n, A.row_ptr, A.col_idx, host_only=True, tile_rows=512)
    assert h.get_tuning("tile_lattice") == 1 and len(h.tiles(0)[0]) - 1 == 8


def test_factor_tile_rows_default_and_key():
    # the tiled factor's tiles shrink with the update work per row: 512 rows for
    # ILU(0) on a 7-point grid, 128 for ILU(1) (about four times the work per row)
    A = synth.laplace3d(16)
    h = jv.Ilu(A.n, A.row_ptr, A.col_idx, host_only=True)
    assert h.get_tuning("tile_rows") == 512 and h.get_tuning("factor_tile_rows") == 512
    C = synth.convdiff3d(24)
    hc = jv.Ilu(C.n, C.row_ptr, C.col_idx, k_max=1, host_only=True)
    assert hc.get_tuning("tile_rows") == 512 and hc.get_tuning("factor_tile_rows") == 128
    for fr, want in ((256, 256), (64, 64), (0, 128)):
        hc.set_tuning("factor_tile_rows", fr)
        assert hc.get_tuning("factor_tile_rows") == want and hc.get_tuning("factor_tiled") == 1
    # the solves' tiles do not move
    assert hc.get_tuning("tile_rows") == 512 and hc.info()["n_tiles"] == len(hc.tiles(0)[0]) - 1
    for bad in (8, 70000, -1):
        with pytest.raises(jv.IluError):
            hc.set_tuning("factor_tile_rows", bad)
    # a 3D grid of 256 or more 1024-row boxes: the solves take the doubled size
    # (two tiles still fit a CU's LDS), the factor keeps 512-row tiles of its own
    G = synth.laplace3d(64)
    hg = jv.Ilu(G.n, G.row_ptr, G.col_idx, host_only=True)
    assert hg.get_tuning("tile_rows") == 1024 and hg.get_tuning("factor_tile_rows") == 512
    _check_tiles(hg, G.n)


def test_tiles_default_fits_and_retile():
    A = synth.laplace3d(10)
    h = jv.Ilu(A.n, A.row_ptr, A.col_idx, host_only=True)
    assert h.info()["tile_rows"] == 512 and h.get_schedule()["solve"] == "tiled"
    h.set_tuning("tile_rows", 64)
    assert h.get_tuning("tile_rows") == 64 and h.info()["tile_rows"] == 64
    _check_tiles(h, A.n)
    with pytest.raises(jv.IluError):
        h.set_tuning("tile_rows", 8)
    # rows longer than any tiled launch handles: the default tiles are not used
    D = synth.dense_pattern(40, np.random.default_rng(3))
    hd = jv.Ilu(D.n, D.row_ptr, D.col_idx, host_only=True)
    assert hd.get_schedule()["solve"] == "syncfree"
