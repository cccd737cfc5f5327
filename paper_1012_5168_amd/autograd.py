"""torch.autograd.Function for the loop estimator (differentiation in kappa and
in the gauge links).

Forward: the per-noise loop estimates L[n][g][t] = sum_d eta_d^+ P_t Gamma_g
M^-1 eta_d for fixed noise (:func:`dl_loops`).  Backward: with the cotangent
W = grad_output (dF = Re sum conj(W) dL),

* dF/dkappa = Re sum conj(W) dL/dkappa with dM^-1/dkappa = M^-1 D M^-1
  (a second solve u = M^-1 D s per right-hand side);
* dF/dU = the link gradient from the adjoint solve
  a = gamma5 M^-1 gamma5 (sum_g W Gamma_g^+ P_t eta) and dF = Re kappa a^+ dD s,

both from one :func:`dl_loops_link_grad` call (three solves per right-hand
side), which also contracts dL/dkappa with W.  Links are uploaded with all
three rows stored, so the gradient is exact for unconstrained 3x3 complex
links; gradients follow PyTorch's complex convention grad = dF/dRe + i dF/dIm.

Links on the GPU stay there: the gauge field is uploaded from the tensor's
device memory, the link gradient is written into a device tensor, and the
loops are returned on the links' device (they come back from the library as
a few host numbers per noise).  The gradient in kappa has kappa's device and
dtype.  Only the cotangent of the loops ([n_noise][n_gamma][T]) crosses to
the host.
"""
from __future__ import annotations

import numpy as np
import torch

from . import DL_F64, Gauge, Lattice, loops, loops_link_grad, solve_params


class DisconnectedLoops(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, links, dims, sources, gammas, params, t_antiperiodic=True):
        lat = Lattice(dims, t_antiperiodic)
        U = links.detach()
        if U.is_cuda:
            G = Gauge(lat, U.to(torch.complex128).contiguous(), precs=(DL_F64,), recon=18)
        else:
            G = Gauge(lat, U.to(torch.complex128).numpy(), precs=(DL_F64,), recon=18)
        k = float(kappa.detach())
        L, st = loops(G, k, sources, list(gammas), params)
        ctx.state = (lat, G, k, sources, list(gammas), params)
        ctx.links_meta = (links.device, links.dtype, tuple(links.shape))
        ctx.kappa_meta = (kappa.device, kappa.dtype)
        ctx.stats = st
        return torch.from_numpy(L).to(links.device)

    @staticmethod
    def backward(ctx, grad_out):
        lat, G, k, sources, gammas, params = ctx.state
        ldev, ldtype, lshape = ctx.links_meta
        W = grad_out.detach().to(torch.complex128).cpu().numpy()
        g_links = None
        if ldev.type == "cuda":
            g_links = torch.empty(lshape, dtype=torch.complex128, device=ldev)
            _, _, _, dfk, _ = loops_link_grad(G, k, sources, gammas, W, params, with_dkappa=True, grad_out=g_links)
        else:
            grad, _, _, dfk, _ = loops_link_grad(G, k, sources, gammas, W, params, with_dkappa=True)
            g_links = torch.from_numpy(np.ascontiguousarray(grad))
        kdev, kdtype = ctx.kappa_meta
        g_kappa = torch.tensor(dfk, dtype=kdtype, device=kdev)
        return g_kappa, g_links.to(ldtype), None, None, None, None, None


def disconnected_loops(kappa, links, dims, sources, gammas, params=None, t_antiperiodic=True):
    """Differentiable per-noise loop estimates [n_noise][n_gamma][T] (complex128).

    kappa: 0-d float64 tensor; links: complex128 tensor [4][V][3][3] (host or GPU).
    """
    params = params or solve_params(tol=1e-12, maxiter=2000)
    return DisconnectedLoops.apply(kappa, links, tuple(int(d) for d in dims), sources, tuple(gammas), params,
                                   t_antiperiodic)
