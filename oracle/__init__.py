"""Serial FP64 CPU oracle for the Javelin incomplete-LU hot path (arXiv:1812.06160).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the bench's
CPU-baseline leg may import this package.  It wraps ``liboracle.so`` (built from
``oracle.c`` by ``oracle/build.py``) with numpy glue; it shares no code with the
HIP library and never calls it.

The steps follow the paper's statement of the problem:

* ``canonical``  conventional CSR, diagonal made explicit (Sec. I-III)
* ``symbolic``   pattern S of ILU(K) by level of fill (Sec. III, Sec. IV "Incomplete levels")
* ``levels``     level sets of lower(S) or lower(S+S^T) (Sec. II, Sec. III)
* ``analyze``    all of the above plus the level-order permutation and permuted copy (Sec. III)
* ``factor``     up-looking fixed-pattern ILU(k, tau) (Sec. III, Fig. 1)
* ``apply``      M^{-1} b by forward and backward substitution (Sec. VI)
* ``spmv``, ``pcg``, ``fgmres``   the Krylov consumers (Sec. I-II)
* ``adjoint``    gradient of the apply with respect to b and the factor values
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, ERR_ARG, ERR_CSR, ERR_NOMEM, ERR_ZERO_PIVOT, ERR_NONFINITE, ERR_NOCONV, ERR_BREAKDOWN = 0, 1, 2, 3, 5, 6, 7, 8

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        vp = C.c_void_p
        L.orc_canonical.restype = C.c_long
        L.orc_canonical.argtypes = [C.c_int, _i32p, _i32p, vp, C.c_long, vp, vp, vp]
        L.orc_symbolic.restype = C.c_long
        L.orc_symbolic.argtypes = [C.c_int, _i32p, _i32p, C.c_int, C.c_long, vp, vp, vp]
        L.orc_levels.restype = C.c_int
        L.orc_levels.argtypes = [C.c_int, _i32p, _i32p, C.c_int, _i32p]
        L.orc_sort_by_key.restype = None
        L.orc_sort_by_key.argtypes = [C.c_int, _i32p, C.c_int, _i32p, _i32p, _i32p]
        L.orc_permute.restype = None
        L.orc_permute.argtypes = [C.c_int, _i32p, _i32p, _i32p, _i32p, _i32p, _i32p, _i64p, _i32p]
        L.orc_values_on_pattern.restype = None
        L.orc_values_on_pattern.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i64p]
        L.orc_upper_levels.restype = C.c_int
        L.orc_upper_levels.argtypes = [C.c_int, _i32p, _i32p, _i32p]
        L.orc_row_tau.restype = None
        L.orc_row_tau.argtypes = [C.c_int, _i32p, _f64p, _i32p, C.c_double, _f64p]
        L.orc_rcm.restype = C.c_int
        L.orc_rcm.argtypes = [C.c_int, _i32p, _i32p, _i32p]
        L.orc_factor.restype = C.c_int
        L.orc_factor.argtypes = [C.c_int, _i32p, _i32p, _i32p, _i32p, _f64p, C.c_int, _f64p, C.c_int,
                                 _i8p, C.POINTER(C.c_int)]
        L.orc_cast_f32.restype = None
        L.orc_cast_f32.argtypes = [C.c_long, _f64p, _f32p]
        L.orc_cast_bf16.restype = None
        L.orc_cast_bf16.argtypes = [C.c_long, _f64p, _u16p]
        L.orc_apply_f64.restype = None
        L.orc_apply_f64.argtypes = [C.c_int, _i32p, _i32p, _i32p, _f64p, vp, _f64p, _f64p, vp,
                                    C.c_int, C.c_long]
        L.orc_apply_lowp.restype = None
        L.orc_apply_lowp.argtypes = [C.c_int, _i32p, _i32p, _i32p, vp, C.c_int, vp, _f64p, _f64p,
                                     C.c_int, C.c_long]
        L.orc_spmv.restype = None
        L.orc_spmv.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, C.c_int, C.c_long]
        L.orc_pcg.restype = C.c_int
        L.orc_pcg.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _i32p, _f64p, vp, C.c_int,
                              _f64p, _f64p, C.c_double, C.c_int, _f64p]
        L.orc_fgmres.restype = C.c_int
        L.orc_fgmres.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _i32p, _f64p, vp,
                                 C.c_int, _f64p, _f64p, C.c_double, C.c_int, C.c_int, _f64p]
        L.orc_adjoint.restype = None
        L.orc_adjoint.argtypes = [C.c_int, _i32p, _i32p, _i32p, _f64p, _i32p, _f64p, _f64p, _f64p,
                                  _f64p, _f64p, C.c_int, C.c_long]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"oracle status {code} {msg}")
        self.code = code


# ------------------------------------------------------------------------------------
# Structure
# ------------------------------------------------------------------------------------

def canonical(n, row_ptr, col_idx, val=None):
    """Validated CSR with every diagonal stored (missing ones inserted as 0.0).

    Returns (row_ptr, col_idx, val, src) where src[e] is the input entry of canonical
    entry e (-1 for an inserted diagonal).
    """
    L = lib()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = None if val is None else np.ascontiguousarray(val, dtype=np.float64)
    need = L.orc_canonical(n, rp, ci, _ptr(v), 0, None, None, None)
    if need < 0:
        raise OracleError(-need, "invalid CSR")
    rp2 = np.empty(n + 1, np.int32)
    ci2 = np.empty(need, np.int32)
    v2 = np.empty(need, np.float64)
    L.orc_canonical(n, rp, ci, _ptr(v), need, _ptr(rp2), _ptr(ci2), _ptr(v2))
    # map canonical entries back to input entries (glue: key matching, no arithmetic of the method)
    rows_in = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    rows_c = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp2))
    key_in = rows_in * n + ci
    key_c = rows_c * n + ci2
    pos = np.searchsorted(key_in, key_c)
    pos = np.minimum(pos, max(0, key_in.size - 1))
    src = np.where((key_in.size > 0) & (key_in[pos] == key_c), pos, -1).astype(np.int64)
    return rp2, ci2, v2, src


def symbolic(n, rp, ci, K):
    """Pattern S of ILU(K) and the fill level of each entry: (srp, sci, slev)."""
    L = lib()
    need = L.orc_symbolic(n, rp, ci, K, 0, None, None, None)
    if need < 0:
        raise OracleError(-need)
    srp = np.empty(n + 1, np.int32)
    sci = np.empty(need, np.int32)
    slev = np.empty(need, np.int32)
    L.orc_symbolic(n, rp, ci, K, need, _ptr(srp), _ptr(sci), _ptr(slev))
    return srp, sci, slev


def levels(n, rp, ci, sym=True):
    level = np.empty(n, np.int32)
    nlev = lib().orc_levels(n, rp, ci, 1 if sym else 0, level)
    return level, nlev


def sort_by_key(key, nkey):
    n = key.size
    perm = np.empty(n, np.int32)
    iperm = np.empty(n, np.int32)
    ptr = np.empty(nkey + 1, np.int32)
    lib().orc_sort_by_key(n, np.ascontiguousarray(key, dtype=np.int32), nkey, perm, iperm, ptr)
    return perm, iperm, ptr


def permute(n, rp, ci, perm, iperm):
    prp = np.empty(n + 1, np.int32)
    pci = np.empty(int(rp[-1]), np.int32)
    src = np.empty(int(rp[-1]), np.int64)
    dpos = np.empty(n, np.int32)
    lib().orc_permute(n, rp, ci, perm, iperm, prp, pci, src, dpos)
    return prp, pci, src, dpos


def upper_levels(n, rp, ci):
    ulev = np.empty(n, np.int32)
    nul = lib().orc_upper_levels(n, rp, ci, ulev)
    return ulev, nul


@dataclass
class Analysis:
    n: int
    k_max: int
    sym: bool
    # canonical A (input ordering)
    a_rp: np.ndarray
    a_ci: np.ndarray
    a_src: np.ndarray        # canonical entry -> input entry (-1: inserted diagonal)
    # pattern S (input ordering)
    s_rp: np.ndarray
    s_ci: np.ndarray
    s_lev: np.ndarray
    # level schedule
    level: np.ndarray
    n_levels: int
    perm: np.ndarray         # new -> old
    iperm: np.ndarray        # old -> new
    level_ptr: np.ndarray
    # permuted factor structure P S P^T
    lu_rp: np.ndarray
    lu_ci: np.ndarray
    lu_lev: np.ndarray
    lu_src: np.ndarray       # factor entry -> input entry of A (-1: fill or inserted diagonal)
    diag_pos: np.ndarray
    # permuted copy of A for spmv
    b_rp: np.ndarray
    b_ci: np.ndarray
    b_src: np.ndarray        # entry -> input entry of A (-1: inserted diagonal)
    # backward-solve schedule
    ulev: np.ndarray
    n_ulevels: int
    ulevel_rows: np.ndarray
    ulevel_ptr: np.ndarray
    order: np.ndarray | None = None   # RCM preorder (new -> input), when one was applied
    extra: dict = field(default_factory=dict)

    @property
    def nnz_lu(self):
        return int(self.lu_rp[-1])

    def level_stats(self):
        sizes = np.diff(self.level_ptr)
        return dict(levels=int(self.n_levels), min=int(sizes.min()), max=int(sizes.max()),
                    median=float(np.median(sizes)))


def rcm(n, row_ptr, col_idx):
    """Reverse Cuthill-McKee order of the graph of A + A^T: order[i] is the input
    vertex that becomes vertex i (Sec. VII's RCM preordering)."""
    order = np.empty(n, np.int32)
    st = lib().orc_rcm(n, np.ascontiguousarray(row_ptr, dtype=np.int32),
                       np.ascontiguousarray(col_idx, dtype=np.int32), order)
    if st != OK:
        raise OracleError(st)
    return order


def analyze(n, row_ptr, col_idx, k_max=0, sym=True, rcm_order=False) -> Analysis:
    """Pattern, level schedule and permuted structure of ILU(k_max) (Sec. III).

    rcm_order: preorder A by reverse Cuthill-McKee first (Sec. VII); the pattern and
    levels then belong to Q A Q^T, and perm / the entry maps are composed so that
    they still refer to the input ordering and input entries."""
    if rcm_order:
        canonical(n, row_ptr, col_idx)          # validates A
        q = rcm(n, row_ptr, col_idx)
        iq = np.empty(n, np.int32)
        iq[q] = np.arange(n, dtype=np.int32)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        qrp, qci, qsrc, _ = permute(n, rp, ci, q, iq)
        an = analyze(n, qrp, qci, k_max, sym)
        # compose: Q A Q^T entries -> input entries, level rows -> input rows
        an.lu_src = np.where(an.lu_src >= 0, qsrc[np.maximum(an.lu_src, 0)], -1)
        an.b_src = np.where(an.b_src >= 0, qsrc[np.maximum(an.b_src, 0)], -1)
        an.perm = q[an.perm].astype(np.int32)
        an.iperm = np.empty(n, np.int32)
        an.iperm[an.perm] = np.arange(n, dtype=np.int32)
        # tau row norms are taken over the input rows, in input entry order
        an.a_rp, an.a_ci, _, an.a_src = canonical(n, row_ptr, col_idx)
        an.order = q
        return an
    a_rp, a_ci, _, a_src = canonical(n, row_ptr, col_idx, None)
    s_rp, s_ci, s_lev = symbolic(n, a_rp, a_ci, k_max)
    level, nlev = levels(n, s_rp, s_ci, sym)
    perm, iperm, level_ptr = sort_by_key(level, nlev)
    lu_rp, lu_ci, src, dpos = permute(n, s_rp, s_ci, perm, iperm)
    # S entry -> canonical A entry, then -> input entry
    dummy = np.zeros(a_ci.size, np.float64)
    sval = np.empty(s_ci.size, np.float64)
    amap = np.empty(s_ci.size, np.int64)
    lib().orc_values_on_pattern(n, a_rp, a_ci, dummy, s_rp, s_ci, sval, amap)
    s_to_in = np.where(amap >= 0, a_src[np.maximum(amap, 0)], -1)
    lu_src = s_to_in[src]
    lu_lev = s_lev[src].astype(np.int32)
    b_rp, b_ci, bsrc, _ = permute(n, a_rp, a_ci, perm, iperm)
    b_src = a_src[bsrc]
    ulev, nul = upper_levels(n, lu_rp, lu_ci)
    urows, _, uptr = sort_by_key(ulev, nul)
    return Analysis(n=n, k_max=k_max, sym=sym, a_rp=a_rp, a_ci=a_ci, a_src=a_src,
                    s_rp=s_rp, s_ci=s_ci, s_lev=s_lev, level=level, n_levels=nlev, perm=perm,
                    iperm=iperm, level_ptr=level_ptr, lu_rp=lu_rp, lu_ci=lu_ci, lu_lev=lu_lev,
                    lu_src=lu_src, diag_pos=dpos, b_rp=b_rp, b_ci=b_ci, b_src=b_src, ulev=ulev,
                    n_ulevels=nul, ulevel_rows=urows, ulevel_ptr=uptr)


def gather(src, values):
    """values[src] with 0.0 where src < 0."""
    out = np.zeros(src.size, np.float64)
    m = src >= 0
    out[m] = np.asarray(values, dtype=np.float64)[src[m]]
    return out


# ------------------------------------------------------------------------------------
# Numerics
# ------------------------------------------------------------------------------------

@dataclass
class Factor:
    val: np.ndarray          # L (strict lower) and U (with diagonal), factor order, FP64
    stat: np.ndarray         # 0 kept, 1 dropped by tau, 2 absent (fill level > k)
    status: int
    bad_row: int


def row_tau(an: Analysis, a_val_input, tau):
    a_val = gather(an.a_src, a_val_input)
    out = np.empty(an.n, np.float64)
    lib().orc_row_tau(an.n, an.a_rp, a_val, an.perm, float(tau), out)
    return out


def factor(an: Analysis, a_val_input, k=None, tau=0.0, milu=False) -> Factor:
    """Up-looking ILU(k, tau) on P S P^T (Sec. III, Fig. 1); milu: modified ILU
    (what a row loses goes to its diagonal; Sec. I, Sec. III)."""
    k = an.k_max if k is None else int(k)
    val = gather(an.lu_src, a_val_input)
    rt = row_tau(an, a_val_input, tau)
    stat = np.empty(an.nnz_lu, np.int8)
    bad = C.c_int(-1)
    st = lib().orc_factor(an.n, an.lu_rp, an.lu_ci, an.lu_lev, an.diag_pos, val, k, rt, 1 if milu else 0,
                          stat, C.byref(bad))
    return Factor(val=val, stat=stat, status=st, bad_row=bad.value)


def cast_f32(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(x.size, np.float32)
    lib().orc_cast_f32(x.size, x, y)
    return y


def cast_bf16(x):
    """BF16 bit patterns (uint16) of x rounded FP64 -> FP32 -> BF16."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(x.size, np.uint16)
    lib().orc_cast_bf16(x.size, x, y)
    return y


def _rhs2d(b):
    b = np.ascontiguousarray(b, dtype=np.float64)
    return b.reshape(b.shape[0], -1)


def apply(an: Analysis, lu_val, b, prec="f64", permuted=False, want_y=False):
    """x = M^{-1} b with M = P^T L U P (original ordering unless permuted=True).

    prec: "f64" (lu_val FP64), "f32" (lu_val float32) or "bf16" (lu_val uint16 bits).
    """
    b2 = _rhs2d(b)
    n, nrhs = b2.shape
    x = np.empty_like(b2)
    perm = None if permuted else an.perm
    L = lib()
    if prec == "f64":
        y = np.empty_like(b2) if want_y else None
        L.orc_apply_f64(n, an.lu_rp, an.lu_ci, an.diag_pos, np.ascontiguousarray(lu_val, np.float64),
                        _ptr(perm), b2, x, _ptr(y), nrhs, nrhs)
        xs = x.reshape(np.shape(b))
        return (xs, y.reshape(np.shape(b))) if want_y else xs
    code = {"f32": 1, "bf16": 2}[prec]
    v = np.ascontiguousarray(lu_val, dtype=np.float32 if code == 1 else np.uint16)
    L.orc_apply_lowp(n, an.lu_rp, an.lu_ci, an.diag_pos, _ptr(v), code, _ptr(perm), b2, x, nrhs, nrhs)
    return x.reshape(np.shape(b))


def spmv(n, rp, ci, val, x):
    x2 = _rhs2d(x)
    y = np.empty_like(x2)
    lib().orc_spmv(n, np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(ci, np.int32),
                   np.ascontiguousarray(val, np.float64), x2, y, x2.shape[1], x2.shape[1])
    return y.reshape(np.shape(x))


def _lowp(lu_val, prec):
    if prec == "f64":
        return 0, None
    if prec == "f32":
        return 1, np.ascontiguousarray(lu_val, np.float32)
    return 2, np.ascontiguousarray(lu_val, np.uint16)


def pcg(an: Analysis, b_val_perm, lu64, b, prec="f64", lu_low=None, tol=1e-10, maxit=10000):
    """PCG on the permuted system B x' = P b; returns (x original ordering, iters, relres, status)."""
    code, low = _lowp(lu_low, prec)
    bp = np.ascontiguousarray(np.asarray(b, np.float64)[an.perm])
    xp = np.empty_like(bp)
    out = np.zeros(2)
    st = lib().orc_pcg(an.n, an.b_rp, an.b_ci, np.ascontiguousarray(b_val_perm, np.float64),
                       an.lu_rp, an.lu_ci, an.diag_pos, np.ascontiguousarray(lu64, np.float64),
                       _ptr(low), code, bp, xp, tol, maxit, out)
    x = np.empty_like(xp)
    x[an.perm] = xp
    return x, int(out[0]), float(out[1]), st


def fgmres(an: Analysis, b_val_perm, lu64, b, prec="f64", lu_low=None, tol=1e-10, restart=30,
           maxcycles=1000):
    """Right-preconditioned FGMRES(restart) on the permuted system."""
    code, low = _lowp(lu_low, prec)
    bp = np.ascontiguousarray(np.asarray(b, np.float64)[an.perm])
    xp = np.empty_like(bp)
    out = np.zeros(2)
    st = lib().orc_fgmres(an.n, an.b_rp, an.b_ci, np.ascontiguousarray(b_val_perm, np.float64),
                          an.lu_rp, an.lu_ci, an.diag_pos, np.ascontiguousarray(lu64, np.float64),
                          _ptr(low), code, bp, xp, tol, restart, maxcycles, out)
    x = np.empty_like(xp)
    x[an.perm] = xp
    return x, int(out[0]), float(out[1]), st


def adjoint(an: Analysis, lu_val, gx, x, y):
    """Gradients of a loss through x = M^{-1} b: returns (gb, glu).

    gx, x: original ordering [n] or [n][nrhs]; y: the permuted forward intermediate.
    """
    gx2, x2, y2 = _rhs2d(gx), _rhs2d(x), _rhs2d(y)
    n, nrhs = gx2.shape
    gb = np.empty_like(gx2)
    glu = np.empty(an.nnz_lu, np.float64)
    lib().orc_adjoint(n, an.lu_rp, an.lu_ci, an.diag_pos, np.ascontiguousarray(lu_val, np.float64),
                      an.perm, gx2, x2, y2, gb, glu, nrhs, nrhs)
    return gb.reshape(np.shape(gx)), glu


def b_values(an: Analysis, a_val_input):
    """Values of the permuted copy of A (spmv operand), from the input values."""
    return gather(an.b_src, a_val_input)


def dense_factors(an: Analysis, lu_val):
    """Dense unit-lower L and upper U of the permuted factor (for small tests)."""
    n = an.n
    Lm = np.eye(n)
    Um = np.zeros((n, n))
    for r in range(n):
        for p in range(an.lu_rp[r], an.lu_rp[r + 1]):
            c = an.lu_ci[p]
            if c < r:
                Lm[r, c] = lu_val[p]
            else:
                Um[r, c] = lu_val[p]
    return Lm, Um
