"""torch.autograd front end of the long-range sums.

Both functions take a Plan and run every step on the GPU through the C ABI.

* ``energy(plan, pos, q[, rb=(P, seed, step)])`` returns E = 1/2 sum q_i phi_i
  (a 0-d float64 tensor).  Its gradients are outputs of the forward call
  itself: dE/dpos = -F and dE/dq = phi (Sec. 2.1 pair energy; App. E forces).
* ``potential(plan, pos, q[, rb])`` returns phi; its backward for an upstream
  gradient g runs the adjoint scans (q2d_long_range_vjp / q2d_rbm_step_vjp):
  dq = phi(g) and dpos = -(g f(q) + q f(g)), f being the field.

``rb`` selects the random-batch estimator with the modes of (seed, step)
(a deterministic function of pos and q for fixed modes); without it the
exact-k sum of the plan's k_c is used.
"""

import torch


def _forward(plan, pos, q, rb):
    if rb is None:
        phi, F, E = plan.long_range(pos, q)
    else:
        P, seed, step = rb
        phi, F, E, _ = plan.rbm_step(pos, q, P, seed, step)
    return phi, F, E


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, plan, rb):
        phi, F, E = _forward(plan, pos.detach(), q.detach(), rb)
        ctx.save_for_backward(phi, F)
        return E.reshape(())

    @staticmethod
    def backward(ctx, gE):
        phi, F = ctx.saved_tensors
        g = gE.to(F.dtype)
        dpos = -g * F if ctx.needs_input_grad[0] else None
        dq = g * phi if ctx.needs_input_grad[1] else None
        return dpos, dq, None, None


class _Potential(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, plan, rb):
        pos, q = pos.detach(), q.detach()
        phi, _, _ = _forward(plan, pos, q, rb)
        ctx.save_for_backward(pos, q)
        ctx.plan = plan
        ctx.rb = rb
        return phi

    @staticmethod
    def backward(ctx, g):
        pos, q = ctx.saved_tensors
        g = g.to(pos.dtype).contiguous()
        if ctx.rb is None:
            dq, dpos = ctx.plan.long_range_vjp(pos, q, g)
        else:
            P, seed, step = ctx.rb
            dq, dpos = ctx.plan.rbm_step_vjp(pos, q, g, P, seed, step)
        return (dpos if ctx.needs_input_grad[0] else None,
                dq if ctx.needs_input_grad[1] else None, None, None)


def energy(plan, pos, q, rb=None):
    """Long-range energy E(pos, q), differentiable in pos and q."""
    return _Energy.apply(pos, q, plan, rb)


def potential(plan, pos, q, rb=None):
    """Long-range potential phi(pos, q) (N,), differentiable through the adjoint scans."""
    return _Potential.apply(pos, q, plan, rb)
