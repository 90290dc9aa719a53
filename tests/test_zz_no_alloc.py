"""ilu_apply_noalloc (the apply whose intermediates live in the library's static
device workspace) against ilu_apply on the same handles: bit for bit, on two calls
in a row with the second one smaller, in FP64 and FP32; and the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def noalloc(jv, ilu, b, x, prec="f64", permuted=False):
    # straight through the C ABI (ctypes declarations of the binding)
    from paper_1812_06160_amd import _lib as L
    fn = L.load().ilu_apply_noalloc
    nrhs, ld = (1, 1) if b.dim() == 1 else (b.shape[1], b.stride(0))
    vec = L.PREC_F64 if b.dtype == torch.float64 else L.PREC_F32
    prec_c = {"f64": L.PREC_F64, "f32": L.PREC_F32, "bf16": L.PREC_BF16}[prec]
    return fn(ilu.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), nrhs, ld, prec_c, vec,
              L.PERMUTED_SPACE if permuted else 0, C.c_void_p(torch.cuda.current_stream().cuda_stream))


def same_bits(a, b):
    a = a.cpu().numpy()
    b = b.cpu().numpy()
    return np.array_equal(a.view(np.uint64 if a.dtype == np.float64 else np.uint32),
                          b.view(np.uint64 if b.dtype == np.float64 else np.uint32))


@pytest.mark.parametrize("sched", ["tiled", "syncfree", "level"])
def test_noalloc_matches_apply(jv, sched):
    rng = np.random.default_rng(41)
    big = synth.laplace3d(40)                        # n = 64000, 4 RHS
    small = synth.convdiff3d(12)                     # n = 1728, 1 RHS, ILU(1)
    hb = jv.Ilu(big.n, big.row_ptr, big.col_idx, tile_rows=256)
    hs = jv.Ilu(small.n, small.row_ptr, small.col_idx, k_max=1, tile_rows=64)
    for h in (hb, hs):
        h.set_schedule("syncfree", sched)
    hb.factor(dev(big.val), casts=("f32",))
    hs.factor(dev(small.val), k=1, tau=1e-3, casts=("f32",))
    for prec in ("f64", "f32"):
        Bb = dev(rng.uniform(-1, 1, (big.n, 4)))
        Bs = dev(rng.uniform(-1, 1, small.n))
        ref_b = hb.apply(Bb, prec=prec)
        ref_s = hs.apply(Bs, prec=prec)
        xb = torch.full_like(Bb, float("nan"))
        xs = torch.full_like(Bs, float("nan"))
        assert noalloc(jv, hb, Bb, xb, prec) == 0
        assert noalloc(jv, hs, Bs, xs, prec) == 0      # second call, smaller input
        torch.cuda.synchronize()
        assert same_bits(xb, ref_b) and same_bits(xs, ref_s)
        # in place and in the level ordering, repeated
        bp = Bs.clone()
        refp = hs.apply(Bs, prec=prec, permuted=True)
        for _ in range(2):
            xp = bp.clone()
            assert noalloc(jv, hs, xp, xp, prec, permuted=True) == 0
            torch.cuda.synchronize()
            assert same_bits(xp, refp)
        hb.status()
        hs.status()


def test_noalloc_size_limit(jv):
    # 2 * n * nrhs * 8 bytes above the 64 MiB workspace: refused, nothing launched
    A = synth.laplace2d(300)                         # n = 90000
    h = jv.Ilu(A.n, A.row_ptr, A.col_idx)
    h.factor(dev(A.val), casts=())
    B = dev(np.ones((A.n, 48)))                      # 4.32M elements > 4.19M
    X = torch.empty_like(B)
    assert noalloc(jv, h, B, X) == 1                 # ILU_ERR_ARG
    ok = dev(np.ones((A.n, 46)))                     # 4.14M elements: fits
    assert noalloc(jv, h, ok, torch.empty_like(ok)) == 0
    torch.cuda.synchronize()
