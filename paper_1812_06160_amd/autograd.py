"""torch.autograd.Function for the preconditioner apply x = M^{-1} b.

Forward calls ilu_apply_ex with the factor values as an explicit input and keeps
the permuted intermediate y = L^{-1} P b; backward calls ilu_apply_adjoint, whose
transposed solves and pattern-restricted outer products run in libjavelin.so.
"""
import torch


class IluApply(torch.autograd.Function):
    """x = IluApply.apply(ilu, b, lu_val): differentiable in b ([n] or [n][nrhs],
    float64) and in the factor values lu_val (float64 [nnz_lu], factor order)."""

    @staticmethod
    def forward(ctx, ilu, b, lu_val):
        b = b.contiguous()
        lu_val = lu_val.contiguous()
        x, y = ilu.apply_ex(b, lu_val=lu_val, want_y=True)
        ctx.ilu = ilu
        ctx.save_for_backward(lu_val, x, y)
        return x

    @staticmethod
    def backward(ctx, gx):
        lu_val, x, y = ctx.saved_tensors
        gx = gx.contiguous()
        want_glu = ctx.needs_input_grad[2]
        gb, glu = ctx.ilu.adjoint(gx, x, y, lu_val=lu_val, want_glu=want_glu)
        return None, (gb if ctx.needs_input_grad[1] else None), glu
