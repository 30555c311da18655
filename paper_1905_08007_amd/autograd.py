"""Variance gradient of the Monte Carlo estimator with respect to one graph's
PDF exponents Deg(S), for pilot runs only (production stays nonadaptive).

For w = f/p with z ~ p_theta:  d E_p[w^2] / d theta = -E_p[w^2 d log p / d theta];
with log p = -ln W(full) - sum_l Deg(S_l) t_l - sum ln z (eq. (1) in log-ratio
coordinates) this is  E[w^2 sum_l t_l 1{S_l = S}] + E[w^2] d ln W(full) / d Deg(S).
The library's backward kernel scatters the first term per sample and its
host side adds the second (qa_variance_gradient); this module only marshals.
"""


def variance_and_grad(gset, pdf, img, graph, seed, tag, first, count):
    """(E[w^2], d E[w^2]/d Deg) on `count` samples of the stream."""
    from . import variance_gradient
    return variance_gradient(pdf, img, graph, seed, tag, first, count)


class _Fn:
    pass


try:
    import torch

    class VarianceFn(torch.autograd.Function):
        """Second moment E_p[w^2] of one graph's weights as a function of its
        Deg table; backward returns the gradient the library's backward kernel
        assembled in the forward pass.

        forward(deg, spec) with spec = (base_pdf, graph, seed, tag, first, count):
        the Deg tensor (float64, 2^M entries) replaces the graph's table in a
        copy of base_pdf (the other graphs keep base_pdf's tables)."""

        @staticmethod
        def forward(ctx, deg, spec):
            from . import upload
            base, graph, seed, tag, first, count = spec
            pdf = base.with_graph(graph, deg.detach().cpu().numpy())
            img = upload(base.gset, pdf, device=deg.device if deg.is_cuda else "cuda")
            m2, g = variance_gradient_of(pdf, img, graph, seed, tag, first, count)
            ctx.save_for_backward(torch.from_numpy(g).to(deg.device))
            return deg.new_tensor(m2)

        @staticmethod
        def backward(ctx, gout):
            (g,) = ctx.saved_tensors
            return gout * g, None

    def variance_gradient_of(pdf, img, graph, seed, tag, first, count):
        from . import variance_gradient
        return variance_gradient(pdf, img, graph, seed, tag, first, count)
except ImportError:  # pragma: no cover
    VarianceFn = _Fn
