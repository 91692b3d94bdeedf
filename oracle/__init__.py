"""FP64 CPU oracle of the split-step Fourier propagation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or calls this package; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark do.  It
shares no code, tables or constants with the GPU path.
"""

from .ssfm_ref import (si_params, angular_frequency, linear_factor,
                       nl_step_length, linear_step, nl_step, ase_words,
                       uniform_from_words, ase_noise, edfa, propagate,
                       propagate_batch, nl_pullback, adjoint)

__all__ = ["si_params", "angular_frequency", "linear_factor",
           "nl_step_length", "linear_step", "nl_step", "ase_words",
           "uniform_from_words", "ase_noise", "edfa", "propagate",
           "propagate_batch", "nl_pullback", "adjoint"]

from .ldbp_ref import (fir, nl_rotate, ldbp_forward, matched_filter_samples,
                       mse_loss, mse_grad, ldbp_backward, init_params)

__all__ += ["fir", "nl_rotate", "ldbp_forward", "matched_filter_samples",
            "mse_loss", "mse_grad", "ldbp_backward", "init_params"]

from .dft_ref import dft_matrix, dft_direct, dft16_rounds, dft_bins

__all__ += ["dft_matrix", "dft_direct", "dft16_rounds", "dft_bins"]
