"""MI355X (gfx950) bootstrap particle filter.

The hot path is the HIP library ``libpf_mi355x.so`` (sources in ``csrc/``,
C ABI in ``include/pf.h``); this package is its thin Python binding.
"""
from .binding import (PF_FP32_ACCURATE, PF_FP32_MIXED, PF_FP64, PF_LAYOUT_BATCHED, PF_LAYOUT_PLAIN,
                      PF_MODEL_L96, PF_MODEL_WK, PF_BATCHED_MAX_PARTICLES, PF_RESAMPLE_METROPOLIS,
                      PF_RESAMPLE_MULTINOMIAL, PF_RESAMPLE_REJECTION, PF_RESAMPLE_STRATIFIED, PF_RESAMPLE_SYSTEMATIC, Filter, PfError, load,
                      simulate, systematic)

__all__ = ["Filter", "PfError", "load", "simulate", "systematic", "PF_FP64", "PF_FP32_MIXED", "PF_FP32_ACCURATE",
           "PF_LAYOUT_PLAIN", "PF_LAYOUT_BATCHED", "PF_MODEL_WK", "PF_MODEL_L96",
           "PF_BATCHED_MAX_PARTICLES", "PF_RESAMPLE_SYSTEMATIC", "PF_RESAMPLE_STRATIFIED",
           "PF_RESAMPLE_METROPOLIS", "PF_RESAMPLE_MULTINOMIAL", "PF_RESAMPLE_REJECTION"]
