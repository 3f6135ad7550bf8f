"""Hyper-parameter training loop (oracle, FP64).

Test infrastructure only (see ``oracle/__init__``).

The paper trains Θ by a gradient-based optimizer over the hand-coded NLML
gradient (Listing 1's loop: compute loss and gradient, optimizer step); its
end-to-end runs use Adam, 50 steps, learning rate 0.01 ("Numerical
Experiments").  Adam is restated from Kingma & Ba (2015, Algorithm 1) with
β₁ = 0.9, β₂ = 0.999, ε = 1e-8 (the usual defaults):
    m ← β₁m + (1−β₁)g,  v ← β₂v + (1−β₂)g²,
    θ ← θ − lr·(m/(1−β₁ᵗ)) / (√(v/(1−β₂ᵗ)) + ε).
With the softplus transform the optimizer runs on ρ, Θ = log(1 + e^ρ), and
∂L/∂ρ = ∂L/∂θ·σ(ρ).
"""
import numpy as np

from .gp import nlml_grad_hutchinson


class Adam:
    def __init__(self, x0, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.x = np.array(x0, dtype=np.float64)
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = np.zeros_like(self.x)
        self.v = np.zeros_like(self.x)
        self.t = 0

    def step(self, g):
        g = np.asarray(g, dtype=np.float64)
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        self.x = self.x - self.lr * mhat / (np.sqrt(vhat) + self.eps)
        return self.x


def softplus(r):
    r = np.asarray(r, dtype=np.float64)
    return np.log1p(np.exp(-np.abs(r))) + np.maximum(r, 0.0)


def softplus_inv(t):
    t = np.asarray(t, dtype=np.float64)
    return t + np.log(-np.expm1(-t))


def sigmoid(r):
    return 1.0 / (1.0 + np.exp(-np.asarray(r, dtype=np.float64)))


def train_gpr(X, y, Z, kernel, theta0, steps=50, lr=0.01, transform=None):
    """Adam on Θ = (l, f, s) (or on ρ with Θ = softplus(ρ)) with the
    Hutchinson NLML gradient (Jacobi control variate, exact solves) over the
    fixed probes Z.  Returns the list of Θ before each step and the final Θ."""
    raw0 = softplus_inv(theta0) if transform == "softplus" else np.array(theta0, dtype=float)
    opt = Adam(raw0, lr)
    path = []
    for _ in range(steps):
        raw = opt.x
        theta = softplus(raw) if transform == "softplus" else raw
        path.append(theta.copy())
        g = nlml_grad_hutchinson(X, y, Z, kernel, *theta)
        if transform == "softplus":
            g = g * sigmoid(raw)
        opt.step(g)
    theta = softplus(opt.x) if transform == "softplus" else opt.x
    return path, theta
