"""The pseudofermion action as a differentiable torch function.

S(U) = phi^dag (M_prec^dag M_prec)^-1 phi, phi on odd sites.  Its gradient with respect to the
links is the fermion force of Sec. 2 (e_a(S) with e_a(U) = T_a U), computed by the library's
adjoint outer-product kernel in the same call that solves for X = (M^dag M)^-1 phi.

PyTorch's convention for a real function of complex inputs is the gradient G with
dS = Re sum conj(G) dU (twice the conjugate Wirtinger derivative); the library returns exactly
that G (``out_kind = 1``), so ``backward`` only scales it by the incoming gradient.  The
generator components follow as e_a(S) = Re tr(G^dag T_a U).

With ``tau_fg > 0`` the Function is the force-gradient step of Sec. 2: the library forms
U' = exp(-tau^2/24 F^j T_j) U from the force at U, solves again at U' starting from the first
solution (forecasting), and returns S(U') with the gradient of S at U' (the gradient the middle
momentum update of the force-gradient integrator uses; U' is not differentiated through).
"""
import torch

from . import DWF_NOT_CONVERGED, FP64, KIND_ODD, DwfError, fermion_force


class PseudofermionAction(torch.autograd.Function):
    """S = PseudofermionAction.apply(U, phi, lattice, tol, tau_fg, maxit)

    U: complex128 natural gauge field [4][T][Z][Y][X][3][3] on the GPU (requires_grad allowed);
    phi: packed FP64 odd half field (from ``lattice.pack(phi, KIND_ODD)``) or a natural 5D
    complex128 field (its odd sites are used); lattice: a ``Lattice`` (operator parameters);
    tau_fg: 0 for S(U) and its gradient, > 0 for the force-gradient step's S(U') and gradient;
    maxit: iteration cap of the solves.
    The solve statistics of the last forward call are kept in ``PseudofermionAction.last_info``.
    Raises DwfError if a solve did not reach tol."""

    last_info = None

    @staticmethod
    def forward(ctx, U, phi, lattice, tol=1e-12, tau_fg=0.0, maxit=100000):
        if phi.dtype == torch.complex128:
            phi = lattice.pack(phi, KIND_ODD)
        Uc = U.detach().contiguous()
        G = torch.empty_like(Uc)
        info = fermion_force(lattice.ctx, lattice.params(FP64, FP64), Uc, phi, G, tau_fg=tau_fg, out_kind=1,
                             tol=tol, maxit=maxit)
        PseudofermionAction.last_info = info
        if not info["converged"]:
            raise DwfError(DWF_NOT_CONVERGED, f"force solve stopped at residual {info['true_rel_resid']:.3e}")
        ctx.save_for_backward(G)
        return torch.tensor(info["S"], dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, grad_S):
        (G,) = ctx.saved_tensors
        return grad_S.to(G.real.dtype) * G, None, None, None, None, None


def action(U, phi, lattice, tol=1e-12, tau_fg=0.0, maxit=100000):
    return PseudofermionAction.apply(U, phi, lattice, tol, tau_fg, maxit)
