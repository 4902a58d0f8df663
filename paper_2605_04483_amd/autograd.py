"""torch.autograd glue for the RDM reverse pass.

`support_energy(ctx, h, eri, top_n)` returns E = c^T H c / c^T c of the
context's truncated, normalised wavefunction (c held fixed) as a 0-d tensor
whose gradients in h and eri are gamma and Gamma / 2 per tensor element (Sec.
3.4, eq. (subopt) at U = I).  Both the value and the gradients come from
cdfci_rdm_backward; the h and eri given here must be the integrals the
context was created with (they serve as the autograd leaves).
"""
import torch

from . import api


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
    return _SupportEnergy.apply(h, eri, ctx, int(top_n))
