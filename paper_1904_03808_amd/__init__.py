"""MI355X-native quasi-static projection solver (libqsmg) -- Python binding.

The compute path is the HIP library `libqsmg.so` built from `csrc/` for
gfx950; this package only marshals torch tensors into its C ABI
(include/qsmg.h).  Import of the binding fails loudly when the library has
not been built; there is no CPU fallback.
"""
from __future__ import annotations


def __getattr__(name):
    if name in ("MGSolver", "SolveInfo"):
        from . import qsmg
        return getattr(qsmg, name)
    if name in ("ProjectionRollout", "rollout_loss"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
