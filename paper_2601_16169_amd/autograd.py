"""Energy as a differentiable function of the integrals.

``SQDEnergy.apply(h, eri, space, **davidson_options)`` returns the lowest
eigenvalue of H restricted to the space (libsqd Davidson on the GPU).  Its
backward pass forms the spin-summed RDMs of the converged vector on the GPU
(libsqd's RDM kernels) and returns, by Hellmann-Feynman (the space does not
depend on the integrals),

    dE/dh_pq = rdm1_pq,    dE/d(pq|rs) = rdm2_pqrs / 2,

element by element.  The integrals enter the library as host copies; the
gradients are returned on the integrals' device and dtype.
"""
from __future__ import annotations

import torch

from . import sqd


class SQDEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, h, eri, space, ecore=0.0, tol=1e-10, max_iter=400, m_max=24, noise=None, guess=None):
        ctx = space.ctx
        ctx.set_hamiltonian(h.detach().cpu().double().numpy(), eri.detach().cpu().double().numpy(), float(ecore))
        E, x, rep = space.davidson(tol=tol, max_iter=max_iter, m_max=m_max, noise=noise, guess=guess)
        if not rep["converged"]:
            raise sqd.SQDError(1, f"Davidson did not converge: residual {rep['residual']:.3e}")
        fctx.space = space
        fctx.x = x
        fctx.h_meta = (h.dtype, h.device, eri.dtype, eri.device)
        fctx.report = rep
        return torch.tensor(E, dtype=h.dtype, device=h.device)

    @staticmethod
    def backward(fctx, gE):
        g1, g2 = fctx.space.rdm(fctx.x, two_body=fctx.needs_input_grad[1])
        hd, hdev, ed, edev = fctx.h_meta
        gh = (gE.to(hdev) * g1.to(device=hdev, dtype=hd)) if fctx.needs_input_grad[0] else None
        ge = (gE.to(edev) * 0.5 * g2.to(device=edev, dtype=ed)) if fctx.needs_input_grad[1] else None
        return gh, ge, None, None, None, None, None, None, None


def energy(h, eri, space, **kw):
    """Functional form of SQDEnergy.apply with keyword options."""
    return SQDEnergy.apply(h, eri, space, kw.get("ecore", 0.0), kw.get("tol", 1e-10), kw.get("max_iter", 400),
                           kw.get("m_max", 24), kw.get("noise"), kw.get("guess"))
