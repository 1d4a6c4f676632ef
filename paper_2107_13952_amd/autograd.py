"""torch.autograd.Function for F(psi_1..psi_5, B) = contract(vertex_tensor(B), psi).

Forward: the vertex tensor (eq. (vertex-ampl)) followed by the boundary contraction.
Backward: the hand-written adjoint of the library (``eprl_contract_boundary_adjoint``): the
boundary-vector gradients from A, the booster gradients by recomputing every shell's {15j}
contribution; nothing per-shell is saved by the forward pass.

PyTorch's complex autograd convention: for an output F with incoming gradient g (the
conjugate Wirtinger derivative of the real loss with respect to F), a holomorphic input z
receives g * conj(dF/dz), and a real input b receives Re(g * conj(dF/db)) where dF/db is the
(complex) derivative of F with respect to the real b.  The library returns c * dF/d(.) for a
complex scalar c, so it is called with c = conj(g) and the results are conjugated.
"""
import torch


class VertexContract(torch.autograd.Function):
    @staticmethod
    def forward(ctx, boosters, psi1, psi2, psi3, psi4, psi5, two_j, dl, gamma):
        from . import vertex_tensor, contract_boundary
        A = vertex_tensor(two_j, dl, gamma, boosters.detach().contiguous())
        psis = [p.detach().contiguous() for p in (psi1, psi2, psi3, psi4, psi5)]
        F = contract_boundary(A, psis)
        ctx.save_for_backward(boosters, A, *psis)
        ctx.two_j, ctx.dl = list(two_j), int(dl)
        return F

    @staticmethod
    def backward(ctx, grad_F):
        from . import contract_boundary_adjoint
        boosters, A, *psis = ctx.saved_tensors
        g = complex(grad_F.detach().cpu().item())
        want_b = ctx.needs_input_grad[0]
        want_p = any(ctx.needs_input_grad[1:6])
        gpsi, gb = contract_boundary_adjoint(ctx.two_j, ctx.dl, boosters, A, psis, g.conjugate(),
                                             want_psi=want_p, want_boosters=want_b)
        out_b = gb.conj().real.contiguous() if want_b else None
        out_p = [t.conj() if (want_p and ctx.needs_input_grad[1 + a]) else None
                 for a, t in enumerate(gpsi if want_p else [None] * 5)]
        return (out_b, *out_p, None, None, None)


def vertex_contract(two_j, dl, gamma, boosters, psis):
    """Differentiable F = sum_i A(i) prod_a psi_a(i_a)."""
    return VertexContract.apply(boosters, *psis, list(two_j), int(dl), float(gamma))
