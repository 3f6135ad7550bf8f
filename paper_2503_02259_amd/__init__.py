"""MI355X-native on-the-fly kernel MatVec engine for Gaussian processes.

The hot path of HiGP (arXiv 2503.02259): Y = K̂·V with
K̂ = f²·k(X, X; l) + s·I, its derivative MatVecs, and the PCG and SLQ drivers
that call it, as hand-written gfx950 HIP kernels behind a C ABI
(``include/higp.h``).  This package is the Python binding.
"""
from ._lib import GAUSSIAN, MATERN32, FP64, FP32, BF16, BF16X3, HigpError  # noqa: F401


def __getattr__(name):
    # Import the torch-facing API lazily so that `workloads` and the build
    # script can be used without importing torch.
    if name in ("kmatvec", "kmatvec_grad", "kmatvec_cross", "pcg", "slq_logdet", "tridiag_eig",
                "problem", "coldot", "nlml", "gpr_predict", "fps_landmarks", "debug_fail_allocs"):
        from . import api
        return getattr(api, name)
    if name in ("KMatVecFn", "GPLossFn", "GPRModel", "train_gpr"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
