"""torch.autograd bindings over the fused derivative MatVec and the NLML
entry point.

* ``KMatVecFn.apply(X, V, l, f, s, kernel)`` = K̂·V; its backward returns
  K̂·G for V (K̂ is symmetric) and ⟨G, ∂K̂/∂θ·V⟩ for θ = l, f, s, from one fused
  derivative MatVec and the library's FP64 column dots.
* ``GPLossFn.apply(X, y, Z, l, f, s, kernel, opts)`` = the estimate of the
  negative log marginal likelihood; its backward is the hand-coded gradient
  (not autodiff through the solver), as in the paper ("Statement of Need",
  hand-coded gradients).
* ``GPRModel``: Θ registered as torch parameters, ``calc_loss_grad()`` fills
  their ``.grad`` (the shape of the paper's Listing 1).

Parameters l, f, s are 0-dim tensors; X carries no gradient.
"""
import torch

from . import api


def _scalar(t):
    return float(t.detach().item()) if isinstance(t, torch.Tensor) else float(t)


class KMatVecFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, V, l, f, s, kernel=0):
        lv, fv, sv = _scalar(l), _scalar(f), _scalar(s)
        ctx.save_for_backward(X, V)
        ctx.theta = (kernel, lv, fv, sv)
        return api.kmatvec(X, V.contiguous(), kernel, lv, fv, sv)

    @staticmethod
    def backward(ctx, G):
        X, V = ctx.saved_tensors
        kernel, lv, fv, sv = ctx.theta
        G = G.contiguous()
        gV = gl = gf = gs = None
        if ctx.needs_input_grad[1]:
            gV = api.kmatvec(X, G, kernel, lv, fv, sv)
        if any(ctx.needs_input_grad[2:5]):
            _, dl, df, _ = api.kmatvec_grad(X, V.contiguous(), kernel, lv, fv, sv,
                                            want=("dl", "df"))
            G2 = G if G.dim() == 2 else G.unsqueeze(1)
            V2 = V if V.dim() == 2 else V.unsqueeze(1)
            dl2 = dl if dl.dim() == 2 else dl.unsqueeze(1)
            df2 = df if df.dim() == 2 else df.unsqueeze(1)
            mk = lambda v: torch.tensor(float(v.sum()), dtype=torch.float64, device=G.device)
            gl = mk(api.coldot(G2, dl2)) if ctx.needs_input_grad[2] else None
            gf = mk(api.coldot(G2, df2)) if ctx.needs_input_grad[3] else None
            gs = mk(api.coldot(G2, V2.contiguous())) if ctx.needs_input_grad[4] else None
        return None, gV, gl, gf, gs, None


class GPLossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, y, Z, l, f, s, kernel=0, opts=None):
        opts = dict(opts or {})
        loss, grad, info = api.nlml(X, y, Z, kernel, _scalar(l), _scalar(f), _scalar(s), **opts)
        ctx.grad = grad
        ctx.info = info
        return torch.tensor(loss, dtype=torch.float64, device=X.device)

    @staticmethod
    def backward(ctx, g):
        gl, gf, gs = (g * float(v) for v in ctx.grad)
        return None, None, None, gl, gf, gs, None, None


class GPRModel(torch.nn.Module):
    """Θ = (l, f, s) as parameters over fixed data; ``calc_loss_grad()``
    returns the loss estimate and fills the parameters' gradients."""

    def __init__(self, X, y, Z, kernel=0, l=1.0, f=1.0, s=0.1, opts=None):
        super().__init__()
        self.X, self.y, self.Z, self.kernel = X, y, Z, kernel
        self.opts = dict(opts or {})
        self.l = torch.nn.Parameter(torch.tensor(float(l), dtype=torch.float64, device=X.device))
        self.f = torch.nn.Parameter(torch.tensor(float(f), dtype=torch.float64, device=X.device))
        self.s = torch.nn.Parameter(torch.tensor(float(s), dtype=torch.float64, device=X.device))

    def calc_loss_grad(self):
        for p in self.parameters():
            p.grad = None
        loss = GPLossFn.apply(self.X, self.y, self.Z, self.l, self.f, self.s, self.kernel, self.opts)
        loss.backward()
        return float(loss)

    def get_params(self):
        return dict(l=float(self.l), f=float(self.f), s=float(self.s))
