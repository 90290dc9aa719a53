"""Thin torch-facing wrapper of the C ABI.

torch supplies device memory and the current HIP stream; every step of the
method runs in libjavelin.so.  Methods take and return torch tensors on the GPU
(float64 unless stated); structure arrays are host numpy arrays.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


_PREC = {"f64": L.PREC_F64, "f32": L.PREC_F32, "bf16": L.PREC_BF16}
_SCHED = {"auto": L.SCHED_AUTO, "level": L.SCHED_LEVEL, "syncfree": L.SCHED_SYNCFREE, "tiled": L.SCHED_TILED}


def _rhs_shape(t):
    if t.dim() == 1:
        return 1, 1
    if t.dim() == 2:
        return t.shape[1], t.stride(0)
    raise ValueError("vectors must be [n] or [n][nrhs]")


def levels_device(row_ptr: torch.Tensor, col_idx: torch.Tensor, pattern: str = "sym"):
    """Level sets of a CSR pattern computed on the GPU (ilu_levels_device).

    row_ptr / col_idx: int32 device tensors; pattern "sym" (lower(S + S^T)),
    "lower" (lower(S)) or "upper" (the strictly upper part, levels from the last
    row: the backward schedule).  Returns (level_ptr, perm, iperm) as int32 device
    tensors, level_ptr trimmed to n_levels + 1 entries."""
    lib = L.load()
    n = row_ptr.numel() - 1
    dev = row_ptr.device
    lp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    iperm = torch.empty(n, dtype=torch.int32, device=dev)
    nl = C.c_int32(0)
    pat = {"sym": L.PATTERN_LOWER_SYM, "lower": L.PATTERN_LOWER_A, "upper": L.PATTERN_UPPER_A}[pattern]
    L.check(lib.ilu_levels_device(int(n), int(col_idx.numel()), _ptr(row_ptr), _ptr(col_idx), pat, _ptr(lp),
                                  _ptr(perm), _ptr(iperm), C.byref(nl), _stream()), "ilu_levels_device")
    return lp[:nl.value + 1], perm, iperm


def permute_device(row_ptr: torch.Tensor, col_idx: torch.Tensor, perm: torch.Tensor, iperm: torch.Tensor):
    """Permuted structure P S P^T on the GPU (ilu_permute_device): returns
    (row_ptr, col_idx, src, diag_pos) as int32 device tensors."""
    lib = L.load()
    n = row_ptr.numel() - 1
    nnz = col_idx.numel()
    dev = row_ptr.device
    orp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    oci = torch.empty(nnz, dtype=torch.int32, device=dev)
    src = torch.empty(nnz, dtype=torch.int32, device=dev)
    dp = torch.empty(n, dtype=torch.int32, device=dev)
    L.check(lib.ilu_permute_device(int(n), int(nnz), _ptr(row_ptr), _ptr(col_idx), _ptr(perm), _ptr(iperm), _ptr(orp),
                                   _ptr(oci), _ptr(src), _ptr(dp), _stream()), "ilu_permute_device")
    return orp, oci, src, dp


def transpose_device(row_ptr: torch.Tensor, col_idx: torch.Tensor):
    """Transposed structure on the GPU (ilu_transpose_device): returns
    (t_row_ptr, t_col_idx, t_map, t_diag) as int32 device tensors."""
    lib = L.load()
    n = row_ptr.numel() - 1
    nnz = col_idx.numel()
    dev = row_ptr.device
    trp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    tci = torch.empty(nnz, dtype=torch.int32, device=dev)
    tmap = torch.empty(nnz, dtype=torch.int32, device=dev)
    tdg = torch.empty(n, dtype=torch.int32, device=dev)
    L.check(lib.ilu_transpose_device(int(n), int(nnz), _ptr(row_ptr), _ptr(col_idx), _ptr(trp), _ptr(tci), _ptr(tmap),
                                     _ptr(tdg), _stream()), "ilu_transpose_device")
    return trp, tci, tmap, tdg


class Ilu:
    """Analysis handle: ILU(k_max) pattern, level schedule and permuted structure of A."""

    def __init__(self, n=None, row_ptr=None, col_idx=None, k_max=0, pattern="sym", host_only=False,
                 tile_rows=0, ordering="natural", tail_min_rows=0, _handle=None):
        self.lib = L.load()
        self.h = C.c_void_p()
        if _handle is not None:
            self.h = _handle
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            ci = np.ascontiguousarray(col_idx, dtype=np.int32)
            csr = L.Csr(int(n), int(rp[-1]), _np_ptr(rp), _np_ptr(ci))
            opts = L.AnalyzeOpts(int(k_max), L.PATTERN_LOWER_SYM if pattern == "sym" else L.PATTERN_LOWER_A,
                                 1 if host_only else 0, int(tile_rows),
                                 {"natural": L.ORDER_NATURAL, "rcm": L.ORDER_RCM}[ordering], int(tail_min_rows))
            L.check(self.lib.ilu_analyze(C.byref(csr), C.byref(opts), C.byref(self.h)), "ilu_analyze")
        self._info = L.Info()
        L.check(self.lib.ilu_get_info(self.h, C.byref(self._info)), "ilu_get_info")
        self.n = self._info.n
        self.nnz_lu = self._info.nnz_lu
        self.nnz_b = self._info.nnz_b
        self.nnz_a = self._info.nnz_a

    @classmethod
    def batched(cls, mats, k_max=0, pattern="sym", host_only=False):
        """Block-diagonal batch of CSR matrices (objects with n, row_ptr, col_idx)."""
        lib = L.load()
        keep = []
        arr = (L.Csr * len(mats))()
        for i, M in enumerate(mats):
            rp = np.ascontiguousarray(M.row_ptr, dtype=np.int32)
            ci = np.ascontiguousarray(M.col_idx, dtype=np.int32)
            keep += [rp, ci]
            arr[i] = L.Csr(int(M.n), int(rp[-1]), _np_ptr(rp), _np_ptr(ci))
        opts = L.AnalyzeOpts(int(k_max), L.PATTERN_LOWER_SYM if pattern == "sym" else L.PATTERN_LOWER_A,
                             1 if host_only else 0)
        h = C.c_void_p()
        L.check(lib.ilu_analyze_batched(len(mats), arr, C.byref(opts), C.byref(h)), "ilu_analyze_batched")
        obj = cls(_handle=h)
        obj.count = len(mats)
        return obj

    def __del__(self):
        try:
            if self.h:
                self.lib.ilu_destroy(self.h)
                self.h = C.c_void_p()
        except Exception:
            pass

    # ---------------------------------------------------------------- structure
    def info(self):
        I = self._info
        return dict(n=I.n, n_levels=I.n_levels, n_ulevels=I.n_ulevels, max_row_lu=I.max_row_lu,
                    nnz_a=I.nnz_a, nnz_lu=I.nnz_lu, nnz_b=I.nnz_b, level_min=I.level_min,
                    level_max=I.level_max, level_median=I.level_median, batch_count=I.batch_count,
                    n_tiles=I.n_tiles, n_utiles=I.n_utiles, tile_rows=I.tile_rows, max_tile=I.max_tile,
                    tail_rows=I.tail_rows, tail_urows=I.tail_urows)

    def schedule(self):
        I = self._info
        n = I.n
        out = dict(level_ptr=np.empty(I.n_levels + 1, np.int32), perm=np.empty(n, np.int32),
                   lu_row_ptr=np.empty(n + 1, np.int32), lu_col_idx=np.empty(I.nnz_lu, np.int32),
                   diag_pos=np.empty(n, np.int32), ulevel_ptr=np.empty(I.n_ulevels + 1, np.int32),
                   ulevel_rows=np.empty(n, np.int32), fill_lev=np.empty(I.nnz_lu, np.int8),
                   lu_src=np.empty(I.nnz_lu, np.int32), b_row_ptr=np.empty(n + 1, np.int32),
                   b_col_idx=np.empty(I.nnz_b, np.int32))
        keys = ["level_ptr", "perm", "lu_row_ptr", "lu_col_idx", "diag_pos", "ulevel_ptr", "ulevel_rows",
                "fill_lev", "lu_src", "b_row_ptr", "b_col_idx"]
        L.check(self.lib.ilu_copy_schedule(self.h, *[_np_ptr(out[k]) for k in keys]), "ilu_copy_schedule")
        return out

    def tiles(self, direction=0):
        """Tiles of the tiled solve of one direction (0: L, 1: U): (tile_ptr, tile_row, sci)."""
        I = self._info
        nt = I.n_tiles if direction == 0 else I.n_utiles
        ptr = np.empty(nt + 1, np.int32)
        L.check(self.lib.ilu_copy_tiles(self.h, int(direction), _np_ptr(ptr), None, None), "ilu_copy_tiles")
        row = np.empty(int(ptr[-1]), np.int32)
        sci = np.empty(I.nnz_lu, np.int32)
        L.check(self.lib.ilu_copy_tiles(self.h, int(direction), _np_ptr(ptr), _np_ptr(row), _np_ptr(sci)),
                "ilu_copy_tiles")
        return ptr, row, sci

    def tail(self, direction=0):
        """The lower stage of one solve direction: dict(level0, pos0, nsteps, hdr [nsteps+1][4], rec)."""
        sz = np.zeros(4, np.int32)
        L.check(self.lib.ilu_copy_tail(self.h, int(direction), _np_ptr(sz), None, None), "ilu_copy_tail")
        hdr = np.zeros((int(sz[2]) + 1) * 4 if sz[2] > 0 else 0, np.int32)
        rec = np.zeros(int(sz[3]), np.int32)
        L.check(self.lib.ilu_copy_tail(self.h, int(direction), None, _np_ptr(hdr), _np_ptr(rec)), "ilu_copy_tail")
        return dict(level0=int(sz[0]), pos0=int(sz[1]), nsteps=int(sz[2]), hdr=hdr.reshape(-1, 4), rec=rec)

    def factor_tail(self):
        """The factor's lower stage: dict(level0, pos0, nsteps, umax, ring_rows, q, hdr
        [nsteps+1][4], rows [records][8], lsrc, match, lmap [nsteps][64]); level0 -1 when
        the handle has no plan."""
        sz = np.zeros(10, np.int32)
        L.check(self.lib.ilu_copy_factor_tail(self.h, _np_ptr(sz), None, None, None, None, None),
                "ilu_copy_factor_tail")
        ns = int(sz[2])
        hdr = np.zeros((ns + 1) * 4 if ns > 0 else 0, np.int32)
        rows = np.zeros(int(sz[6]) * 8, np.int32)
        lsrc = np.zeros(int(sz[7]), np.int32)
        match = np.zeros(int(sz[8]), np.uint8)
        lmap = np.zeros(int(sz[9]), np.uint8)
        L.check(self.lib.ilu_copy_factor_tail(self.h, None, _np_ptr(hdr), _np_ptr(rows), _np_ptr(lsrc),
                                              _np_ptr(match), _np_ptr(lmap)), "ilu_copy_factor_tail")
        return dict(level0=int(sz[0]), pos0=int(sz[1]), nsteps=ns, umax=int(sz[3]), ring_rows=int(sz[4]),
                    q=int(sz[5]), hdr=hdr.reshape(-1, 4), rows=rows.reshape(-1, 8), lsrc=lsrc, match=match,
                    lmap=lmap.reshape(-1, 64))

    def batch_offsets(self):
        cnt = self._info.batch_count
        ro = np.empty(cnt + 1, np.int64)
        zo = np.empty(cnt + 1, np.int64)
        L.check(self.lib.ilu_batch_offsets(self.h, _np_ptr(ro), _np_ptr(zo)), "ilu_batch_offsets")
        return ro, zo

    def set_schedule(self, factor="auto", solve="auto", lanes_factor=0, lanes_solve=0):
        L.check(self.lib.ilu_set_schedule(self.h, _SCHED[factor], _SCHED[solve], int(lanes_factor),
                                          int(lanes_solve)), "ilu_set_schedule")

    def get_schedule(self):
        v = [C.c_int32() for _ in range(4)]
        L.check(self.lib.ilu_get_schedule(self.h, *[C.byref(x) for x in v]), "ilu_get_schedule")
        inv = {1: "level", 2: "syncfree", 3: "tiled"}
        return dict(factor=inv[v[0].value], solve=inv[v[1].value], lanes_factor=v[2].value,
                    lanes_solve=v[3].value)

    def set_tuning(self, key, value):
        L.check(self.lib.ilu_set_tuning(self.h, key.encode(), int(value)), "ilu_set_tuning")
        L.check(self.lib.ilu_get_info(self.h, C.byref(self._info)), "ilu_get_info")

    def get_tuning(self, key):
        v = C.c_int64()
        L.check(self.lib.ilu_get_tuning(self.h, key.encode(), C.byref(v)), "ilu_get_tuning")
        return v.value

    # ---------------------------------------------------------------- numerics
    def factor(self, a_val: torch.Tensor, k=None, tau=0.0, casts=("f32", "bf16"), milu=False):
        """ILU(k, tau) from device values in input order; milu: modified ILU (what a
        row loses goes to its diagonal).  Raises IluError on failure (the exception
        carries .code and the FactorInfo as .info)."""
        assert a_val.is_cuda and a_val.dtype == torch.float64 and a_val.is_contiguous()
        k = 0 if k is None else int(k)
        cbits = (L.CAST_F32 if "f32" in casts else 0) | (L.CAST_BF16 if "bf16" in casts else 0)
        if milu:
            cbits |= L.FACTOR_MODIFIED
        fi = L.FactorInfo()
        code = self.lib.ilu_factor(self.h, _ptr(a_val), k, float(tau), cbits, C.byref(fi), _stream())
        info = dict(bad_row=fi.bad_row, bad_row_original=fi.bad_row_original, bad_matrix=fi.bad_matrix,
                    n_dropped=fi.n_dropped, status=L.STATUS.get(code, code))
        if code != L.OK:
            err = L.IluError(code, "ilu_factor")
            err.info = info
            raise err
        return info

    def factor_values(self):
        """FP64 factor values and entry states (0 kept, 1 dropped, 2 absent) as host arrays."""
        v = np.empty(self.nnz_lu, np.float64)
        st = np.empty(self.nnz_lu, np.int8)
        L.check(self.lib.ilu_copy_factor(self.h, _np_ptr(v), _np_ptr(st)), "ilu_copy_factor")
        return v, st

    def factor_values_prec(self, prec):
        """The stored factor of one precision as a host array (float64, float32 or uint16 bits)."""
        dt = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}[prec]
        out = np.empty(self.nnz_lu, dt)
        L.check(self.lib.ilu_copy_factor_prec(self.h, _PREC[prec], _np_ptr(out)), "ilu_copy_factor_prec")
        return out

    def factor_tensor(self):
        """The FP64 factor values as a device tensor (a copy through the host)."""
        v, _ = self.factor_values()
        return torch.from_numpy(v).to("cuda")

    def apply(self, b: torch.Tensor, x: torch.Tensor | None = None, prec="f64", permuted=False):
        """x = M^{-1} b; b float64 or float32, [n] or [n][nrhs] (row-major)."""
        nrhs, ld = _rhs_shape(b)
        if x is None:
            x = torch.empty_like(b)
        vec = L.PREC_F64 if b.dtype == torch.float64 else L.PREC_F32
        L.check(self.lib.ilu_apply(self.h, _ptr(b), _ptr(x), nrhs, ld, _PREC[prec], vec,
                                   L.PERMUTED_SPACE if permuted else 0, _stream()), "ilu_apply")
        return x

    def status(self):
        """Synchronises the current stream; raises IluError (ILU_ERR_TIMEOUT) if an
        apply on this handle timed out since the last query."""
        L.check(self.lib.ilu_get_status(self.h, _stream()), "ilu_get_status")

    def apply_graph(self, b, x, prec="f64", permuted=False):
        """An ApplyGraph replaying x = M^{-1} b (fixed tensors b and x)."""
        return ApplyGraph(self, b, x, prec, permuted)

    def apply_ex(self, b, lu_val=None, want_y=True, permuted=False):
        nrhs, ld = _rhs_shape(b)
        x = torch.empty_like(b)
        y = torch.empty_like(b) if want_y else None
        L.check(self.lib.ilu_apply_ex(self.h, _ptr(lu_val), _ptr(b), _ptr(x), _ptr(y), nrhs, ld,
                                      L.PERMUTED_SPACE if permuted else 0, _stream()), "ilu_apply_ex")
        return x, y

    def adjoint(self, gx, x, y, lu_val=None, want_glu=True):
        nrhs, ld = _rhs_shape(gx)
        gb = torch.empty_like(gx)
        glu = torch.empty(self.nnz_lu, dtype=torch.float64, device=gx.device) if want_glu else None
        L.check(self.lib.ilu_apply_adjoint(self.h, _ptr(lu_val), _ptr(gx), _ptr(x), _ptr(y), _ptr(gb),
                                           _ptr(glu), nrhs, ld, _stream()), "ilu_apply_adjoint")
        return gb, glu

    def set_values(self, a_val):
        L.check(self.lib.ilu_set_values(self.h, _ptr(a_val), _stream()), "ilu_set_values")

    def spmv(self, x, y=None, alpha=1.0, beta=0.0, permuted=False):
        nrhs, ld = _rhs_shape(x)
        if y is None:
            y = torch.empty_like(x)
            beta = 0.0
        L.check(self.lib.ilu_spmv(self.h, float(alpha), _ptr(x), float(beta), _ptr(y), nrhs, ld,
                                  L.PERMUTED_SPACE if permuted else 0, _stream()), "ilu_spmv")
        return y

    def _solve_info(self, si, code):
        return dict(iters=si.iters, relres=si.relres, true_relres=si.true_relres,
                    status=L.STATUS.get(code, code))

    def pcg(self, b, rtol=1e-10, maxit=10000, prec="f64", permuted=False, raise_on_fail=True):
        x = torch.empty_like(b)
        si = L.SolveInfo()
        code = self.lib.ilu_solve_pcg(self.h, _ptr(b), _ptr(x), float(rtol), int(maxit), _PREC[prec],
                                      L.PERMUTED_SPACE if permuted else 0, C.byref(si), _stream())
        if code != L.OK and (raise_on_fail or code not in (L.ERR_NOCONV, L.ERR_BREAKDOWN)):
            raise L.IluError(code, "ilu_solve_pcg")
        return x, self._solve_info(si, code)

    def gmres(self, b, rtol=1e-10, restart=30, maxit=20000, prec="f64", permuted=False, raise_on_fail=True):
        x = torch.empty_like(b)
        si = L.SolveInfo()
        code = self.lib.ilu_solve_gmres(self.h, _ptr(b), _ptr(x), float(rtol), int(restart), int(maxit),
                                        _PREC[prec], L.PERMUTED_SPACE if permuted else 0, C.byref(si), _stream())
        if code != L.OK and (raise_on_fail or code not in (L.ERR_NOCONV, L.ERR_BREAKDOWN)):
            raise L.IluError(code, "ilu_solve_gmres")
        return x, self._solve_info(si, code)

    def profile(self, enable=True, capacity=8192):
        L.check(self.lib.ilu_profile_enable(self.h, 1 if enable else 0, int(capacity)), "ilu_profile_enable")

    def profile_read(self):
        """{stage: (milliseconds, launches)} accumulated since the last read."""
        ms = np.zeros(L.STAGE_COUNT, np.float64)
        cnt = np.zeros(L.STAGE_COUNT, np.int64)
        L.check(self.lib.ilu_profile_read(self.h, _np_ptr(ms), _np_ptr(cnt)), "ilu_profile_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(L.STAGES)}

    def tune(self, a_val=None, reps=3):
        res = np.zeros((128, 4), np.float64)
        nres = C.c_int32()
        L.check(self.lib.ilu_tune(self.h, _ptr(a_val), int(reps), _np_ptr(res), 128, C.byref(nres), _stream()),
                "ilu_tune")
        return res[:nres.value], self.get_schedule()


class ApplyGraph:
    """One captured ilu_apply (its launches in a HIP graph); launch() replays it on
    the current stream.  Keeps b, x and the handle alive."""

    def __init__(self, ilu, b, x, prec="f64", permuted=False):
        self.ilu, self.b, self.x = ilu, b, x
        nrhs, ld = _rhs_shape(b)
        vec = L.PREC_F64 if b.dtype == torch.float64 else L.PREC_F32
        self.g = C.c_void_p()
        torch.cuda.current_stream().synchronize()
        L.check(ilu.lib.ilu_apply_graph_create(ilu.h, _ptr(b), _ptr(x), nrhs, ld, _PREC[prec], vec,
                                               L.PERMUTED_SPACE if permuted else 0, C.byref(self.g)),
                "ilu_apply_graph_create")

    def launch(self):
        L.check(self.ilu.lib.ilu_graph_launch(self.g, _stream()), "ilu_graph_launch")
        return self.x

    def __del__(self):
        try:
            if self.g:
                self.ilu.lib.ilu_graph_destroy(self.g)
                self.g = C.c_void_p()
        except Exception:
            pass
