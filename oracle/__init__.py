"""Plain FP64 CPU oracle for the HiGP on-the-fly kernel MatVec path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
link anything under ``oracle/``; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP path.

Every function forms the regularised kernel matrix densely (one row block at a
time), in float64, with direct coordinate differences, and then multiplies.  It
follows the paper's statement of the problem ("Gaussian Processes" section):

* ``K̂ = f²·k(X, X; l) + s·I`` with Θ = (s, f, l);
* the negative log marginal likelihood and its gradient;
* PCG for ``K̂⁻¹y`` with a preconditioner ``M ≈ K̂``;
* eq. (1) (log-determinant split) with stochastic Lanczos quadrature;
* eq. (1)'s quadrature with tridiagonals taken from PCG's coefficients;
* eq. (2) (trace split) with the Hutchinson and the Hutch++ estimators;
* prediction with the trained Θ (the textbook GP posterior);
* the training loop (Adam on Θ with that gradient);
* a low-rank (Nyström, farthest-point landmarks) preconditioner for PCG.

Parity status of each function is stated in its docstring.  Functions whose
result has no pin other than itself say "parity unpinned".
"""
from .kernels import (GAUSSIAN, MATERN32, sqdist, kernel_value, kernel_dl,
                      khat_dense, khat_block)
from .matvec import (kmatvec, kmatvec_grad, kmatvec_bf16_emulated, round_bf16,
                     split_bf16, kmatvec_bf16x3_emulated)
from .solvers import (pcg, lanczos, tridiag_eig, slq_logdet, slq_from_tridiag,
                      tridiag_from_cg, cg_logdet)
from .gp import (nlml_exact, nlml_grad_exact, nlml_grad_hutchinson,
                 logdet_exact, orth_range, hutchpp_trace, nlml_grad_hutchpp)
from .predict import kmatvec_cross, gpr_predict
from .train import Adam, softplus, softplus_inv, train_gpr
from .precond import fps_landmarks, nystrom_parts, nystrom_apply_inv, nystrom_dense

__all__ = [
    "GAUSSIAN", "MATERN32", "sqdist", "kernel_value", "kernel_dl", "khat_dense",
    "khat_block", "kmatvec", "kmatvec_grad", "kmatvec_bf16_emulated",
    "round_bf16", "split_bf16", "kmatvec_bf16x3_emulated", "pcg", "lanczos", "tridiag_eig", "slq_logdet",
    "slq_from_tridiag", "nlml_exact", "nlml_grad_exact",
    "nlml_grad_hutchinson", "logdet_exact", "kmatvec_cross", "gpr_predict", "Adam",
    "softplus", "softplus_inv", "train_gpr", "fps_landmarks", "nystrom_parts",
    "nystrom_apply_inv", "nystrom_dense", "tridiag_from_cg", "cg_logdet", "orth_range",
    "hutchpp_trace", "nlml_grad_hutchpp",
]
