"""MI355X-native data-annealed SMC sampler for Bayesian neural-network posteriors.

The compute path is libsmc.so (hand-written HIP kernels for gfx950) behind the C
ABI in include/smc.h; this package is its thin Python binding.  Importing it
without the built library raises ImportError: there is no CPU fallback.
"""
from . import _lib
from ._lib import SMCError
from .sampler import ParticleMLPFn, SMCConfig, SMCSampler, n_params

__all__ = ["SMCConfig", "SMCSampler", "ParticleMLPFn", "SMCError", "n_params", "_lib"]
