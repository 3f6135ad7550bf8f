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
  their ``.grad`` (the shape of the paper's Listing 1); ``train_gpr`` runs
  Adam on it.

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
    returns the loss estimate and fills the parameters' gradients.

    ``transform=None`` registers Θ itself.  ``transform="softplus"`` registers
    raw values ρ with Θ = log(1 + e^ρ), so that an optimizer cannot step a
    parameter out of its domain (l > 0, s ≥ 0); the gradient reaches ρ through
    torch's chain rule (∂L/∂ρ = ∂L/∂θ·σ(ρ))."""

    def __init__(self, X, y, Z, kernel=0, l=1.0, f=1.0, s=0.1, opts=None, transform=None):
        super().__init__()
        if transform not in (None, "softplus"):
            raise ValueError("transform must be None or 'softplus'")
        self.X, self.y, self.Z, self.kernel = X, y, Z, kernel
        self.opts = dict(opts or {})
        self.transform = transform

        def raw(v):
            v = float(v)
            if transform == "softplus":
                v = v + float(torch.log(-torch.expm1(torch.tensor(-v, dtype=torch.float64))))
            return torch.nn.Parameter(torch.tensor(v, dtype=torch.float64, device=X.device))

        self.l, self.f, self.s = raw(l), raw(f), raw(s)

    def theta(self):
        """(l, f, s) as 0-dim tensors (differentiable in the raw parameters)."""
        if self.transform == "softplus":
            sp = torch.nn.functional.softplus
            return sp(self.l), sp(self.f), sp(self.s)
        return self.l, self.f, self.s

    def calc_loss_grad(self):
        for p in self.parameters():
            p.grad = None
        l, f, s = self.theta()
        loss = GPLossFn.apply(self.X, self.y, self.Z, l, f, s, self.kernel, self.opts)
        loss.backward()
        return float(loss.detach())

    def get_params(self):
        with torch.no_grad():
            l, f, s = self.theta()
        return dict(l=float(l), f=float(f), s=float(s))


def train_gpr(model, steps=50, lr=0.01):
    """Adam on the model's parameters for `steps` steps (the paper's E2E
    training settings: 50 steps at learning rate 0.01, Listing 1's loop).
    Returns one record per step: the loss estimate and Θ before the step and
    the raw parameters' gradients."""
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    hist = []
    for i in range(steps):
        loss = model.calc_loss_grad()
        rec = dict(step=i, loss=loss, **model.get_params())
        rec["grad"] = [float(p.grad) for p in (model.l, model.f, model.s)]
        hist.append(rec)
        opt.step()
    return hist
