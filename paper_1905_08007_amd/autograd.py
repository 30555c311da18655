"""Variance-gradient of the Monte Carlo estimator with respect to one graph's
PDF exponents Deg(S), for pilot runs only (production stays nonadaptive).

For w = f/p with z ~ p_theta:  d E_p[w^2] / d theta = -E_p[w^2 d log p / d theta];
with log p = -ln W(full) - sum_l Deg(S_l) t_l - sum ln z (eq. (1) in log-ratio
coordinates) this is  E[w^2 sum_l t_l 1{S_l = S}] + E[w^2] d ln W(full) / d Deg(S).
The first term is scattered per sample by the library's backward kernel, the
second comes from the reverse pass of the W recursion on the host.
"""
import numpy as np


def variance_and_grad(gset, pdf, img, graph, seed, tag, first, count):
    """(E[w^2], d E[w^2]/d Deg) on `count` samples of the stream."""
    import torch
    from . import variance_grad
    grad, w2 = variance_grad(img, graph, seed, tag, first, count)
    torch.cuda.synchronize()
    g = grad.cpu().numpy() / count
    m2 = float(w2.item()) / count
    return m2, g + m2 * pdf.dlogw(graph)


class _Fn:
    pass


try:
    import torch

    class VarianceFn(torch.autograd.Function):
        """Second moment E_p[w^2] of one graph's weights as a function of its
        Deg table; backward runs the library's scatter kernel.

        forward(deg, ctx_data) with ctx_data = (gset, graph, seed, tag, first, count).
        The Deg tensor (float64, 2^M entries) defines a fresh pdf for this graph
        only; the other graphs keep their default tables."""

        @staticmethod
        def forward(ctx, deg, spec):
            from . import Pdf, upload
            gset, graph, seed, tag, first, count = spec
            tables = []
            for g in range(len(gset)):
                if g == graph:
                    tables.append(deg.detach().cpu().numpy())
                else:
                    base = Pdf(gset)
                    tables.append(base.tables(g)[0])
            pdf = Pdf(gset, tables)
            img = upload(gset, pdf, device=deg.device if deg.is_cuda else "cuda")
            m2, g = variance_and_grad(gset, pdf, img, graph, seed, tag, first, count)
            ctx.save_for_backward(torch.from_numpy(g).to(deg.device))
            return deg.new_tensor(m2)

        @staticmethod
        def backward(ctx, gout):
            (g,) = ctx.saved_tensors
            return gout * g, None
except ImportError:  # pragma: no cover
    VarianceFn = _Fn
