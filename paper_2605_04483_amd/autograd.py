"""torch.autograd glue for the RDM reverse pass (Sec. 3.4).

`fci_energy(h, eri, n_alpha, n_beta, ...)` is E(h, eri): forward creates a
context from the integrals it is given, runs coordinate descent to its
stopping rule (Alg. 1, or Alg. 2 with k > 1) and returns the variational
energy E = c^T H c / c^T c of the final, normalised wavefunction (its top_n
determinants by |c|); backward returns grad_E * gamma for h and
grad_E * Gamma / 2 for eri, the derivatives of that E with c held fixed
(eq. (subopt) at U = I), which is also the derivative of the ground energy
once c is converged (Hellmann-Feynman).

`support_energy(ctx, h, eri, top_n)` is the same quotient for an existing
context's wavefunction.  h and eri must equal the integrals the context was
created from (checked: anything else raises), since the value and the
gradients come from that context's Hamiltonian.

Both value and gradients come from cdfci_rdm_backward; nothing of the method
is computed here.
"""
import numpy as np
import torch

from . import api


def _same(a, b):
    if isinstance(a, torch.Tensor) or isinstance(b, torch.Tensor):
        ta = torch.as_tensor(a).detach().to("cpu", torch.float64)
        tb = torch.as_tensor(b).detach().to("cpu", torch.float64)
        return ta.shape == tb.shape and bool(torch.equal(ta, tb))
    return np.array_equal(np.asarray(a), np.asarray(b))


class _FCIEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, h, eri, n_alpha, n_beta, k, max_steps, top_n, opts):
        ctx = api.cdfci_init(h.detach(), eri.detach(), n_alpha, n_beta, **opts)
        try:
            api.cdfci_step(ctx, k, max_steps)
            energy, dh, deri, _ = api.cdfci_rdm_backward(ctx, 1.0, top_n, want_eri=True)
        finally:
            ctx.close()
        fctx.save_for_backward(torch.from_numpy(dh), torch.from_numpy(deri))
        fctx.like = (h.device, h.dtype, eri.device, eri.dtype)
        return torch.tensor(float(energy[0]), dtype=torch.float64, device=h.device)

    @staticmethod
    def backward(fctx, grad_out):
        gamma, half_Gamma = fctx.saved_tensors
        hdev, hdt, edev, edt = fctx.like
        g = grad_out.detach().to("cpu", torch.float64)
        gh = (g * gamma).to(device=hdev, dtype=hdt) if fctx.needs_input_grad[0] else None
        ge = (g * half_Gamma).to(device=edev, dtype=edt) if fctx.needs_input_grad[1] else None
        return gh, ge, None, None, None, None, None, None


def fci_energy(h, eri, n_alpha, n_beta, k=1, max_steps=10 ** 6, top_n=0, **opts):
    """Ground-state energy by coordinate descent from the given integrals.
    opts are cdfci_opts fields (table_slots, dx_threshold, z_threshold, ...);
    the run stops at dx_threshold or after max_steps iterations."""
    return _FCIEnergy.apply(h, eri, int(n_alpha), int(n_beta), int(k), int(max_steps), int(top_n), dict(opts))


class _SupportEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, h, eri, ctx, top_n):
        energy, _, _, _ = api.cdfci_rdm_backward(ctx, 1.0, top_n, want_eri=False)
        fctx.cd_ctx = ctx
        fctx.top_n = top_n
        fctx.like = (h, eri)
        return torch.tensor(float(energy[0]), dtype=torch.float64, device=h.device)

    @staticmethod
    def backward(fctx, grad_out):
        h, eri = fctx.like
        g = float(grad_out.detach().cpu())
        _, dh, deri, _ = api.cdfci_rdm_backward(fctx.cd_ctx, g, fctx.top_n, want_eri=eri.requires_grad)
        gh = torch.from_numpy(dh).to(device=h.device, dtype=h.dtype) if h.requires_grad else None
        ge = torch.from_numpy(deri).to(device=eri.device, dtype=eri.dtype) if deri is not None else None
        return gh, ge, None, None


def support_energy(ctx, h, eri, top_n=0):
    if ctx.integrals is None:
        raise ValueError("support_energy needs a context created by cdfci_init from integrals")
    h0, e0 = ctx.integrals
    if not (_same(h, h0) and _same(eri, e0)):
        raise ValueError("h and eri differ from the integrals the context was created from; "
                         "use fci_energy to solve for new integrals")
    return _SupportEnergy.apply(h, eri, ctx, int(top_n))
