"""Sparsity-discovering exact Gaussian processes on AMD Instinct MI355X.

The compute path is libsdgp.so (HIP, gfx950) behind the C ABI in
include/sdgp.h; this package is its thin Python binding:

* ``Context``        -- a library context on a device / torch stream
* ``estimator``      -- estimator options (probes, Lanczos cap, CG tolerance)
* ``LMLFunction``    -- torch.autograd.Function over ``sdgp_lml_grad``
* ``workloads``      -- seeded synthetic inputs
"""
from . import workloads  # noqa: F401
from ._lib import (Context, SdgpError, estimator, exact_estimator, load,  # noqa: F401
                   CORE_KSTAT, CORE_WENDLAND_C2, COMBINE_PRODUCT, COMBINE_SUM,
                   PROBE_IDENTITY, PROBE_RADEMACHER, PRECOND_LOWRANK, PRECOND_NONE,
                   OPERATOR_ASSEMBLED, OPERATOR_FACTORED, OK, INVALID_ARG, OOM, NOT_SPD,
                   NOT_CONVERGED, HIP, CAPACITY, DE_LML, DE_AUGMENTED, DE_CONSTRAINED, de_trials,
                   de_select, tune_cache_get, tune_cache_put)


def __getattr__(name):
    if name in ("LMLFunction", "lml"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
