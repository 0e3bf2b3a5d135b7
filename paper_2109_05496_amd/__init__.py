"""MI355X-native complex constrained total-variation denoising (FGP) and its
phase-retrieval application (Gao & Cao, arXiv 2109.05496).

Every computation runs in the hand-written HIP kernels of ``libctv.so``
(C ABI in ``include/ctv.h``); this package only marshals arguments. PyTorch
supplies device memory and the current stream. There is no CPU fallback: if
the library is missing, the first call raises.
"""
from .api import (BatchedPlan, CTVDenoise, autotune, autotune_batched, batched_tuned, denoise, denoise_backward, fft2,
                  phase_retrieval, phase_retrieval_ip, pr_forward, pr_gradient, tiling, tune_cache_clear, tune_cache_load,
                  tune_cache_save, tune_cache_size, tuned, workspace_size)
from ._lib import CtvError, EXPORTS, LIB_PATH

__all__ = ["denoise", "denoise_backward", "workspace_size", "tiling", "BatchedPlan", "CTVDenoise",
           "phase_retrieval", "phase_retrieval_ip", "pr_forward", "pr_gradient", "fft2", "autotune", "autotune_batched", "batched_tuned",
           "tune_cache_save", "tune_cache_load", "tune_cache_clear", "tune_cache_size", "tuned", "CtvError", "EXPORTS",
           "LIB_PATH"]
