"""torch.autograd.Function around the type-II transform.

Forward: f = F2 c (nufft2_exec).  For a real loss L and g = dL/dRe f + i dL/dIm f
(torch's gradient convention for complex tensors):
  * dL/dc = F2^H g                       -- the adjoint kernel (nufft1_exec, sign +1)
  * dL/dx_j = Re(conj(g_j) (F2 (-2 pi i k c))_j)   -- one more type-II pass
    with the factor -2 pi i k folded into the scaling (nufft2_grad_x).
Both follow from differentiating f_j = sum_k c_k exp(-2 pi i x_j k) (Sec. 1, eq. (2)).
"""
import torch

from . import binding as B


class NufftTypeII(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, c, plan):
        # the plan must belong to x: the same number of samples, and when x is the very
        # tensor the plan was built from, no in-place write since then (a copy of the
        # planned samples, e.g. x.clone().requires_grad_(), is accepted as it is)
        key = getattr(plan, "x_key", None)
        if key is not None:
            ptr, version, m = key
            if x.numel() != m or (x.data_ptr() == ptr and x._version != version):
                raise ValueError("the plan was built from other samples (or x changed in place since): re-plan")
        ctx.plan = plan
        ctx.save_for_backward(c)
        return B.nufft2_exec(plan, c.resolve_conj().resolve_neg().contiguous())

    @staticmethod
    def backward(ctx, g):
        (c,) = ctx.saved_tensors
        need_x, need_c = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_x or need_c):
            return None, None, None
        # one call: g is put in the plan's sample order once for both passes
        # a conjugated view of g (e.g. from a loss over f.conj()) shares the unconjugated storage
        g = g.resolve_conj().resolve_neg().contiguous()
        gc, gx = B.nufft2_backward(ctx.plan, c.contiguous(), g, need_c=need_c, need_x=need_x)
        return gx, gc, None


class PlanCache:
    """Re-plans only when the samples change (data pointer or in-place version)."""

    def __init__(self, n_modes, eps, dtype=torch.complex64, flags=0):
        self.n_modes, self.eps, self.dtype, self.flags = n_modes, eps, dtype, flags
        self._key = None
        self._plan = None

    def __call__(self, x):
        key = (x.data_ptr(), x._version, x.numel())
        if key != self._key:
            self._plan = B.nufft2_plan(x.detach(), self.n_modes, self.eps, self.dtype, self.flags)
            self._key = key
        return self._plan


def nufft2(x, c, plan):
    """Differentiable f = F2(x) c using a plan built from x."""
    return NufftTypeII.apply(x, c, plan)
