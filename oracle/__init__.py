"""FP64 CPU oracle of the augmented wavelet reconstructor -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it, shares
no code with it, and has no CPU fallback that routes through it.
"""
from .fewha_oracle import (db3_filters, dwt1, idwt1, dwt2, idwt2, OracleSystem,
                           AugmentedReconstructor, pcg, aug_pcg, exact_solution, warm_start_inputs,
                           warm_start_correction, warm_start_step)

from . import closed_loop  # noqa: F401  (pseudo-open-loop slopes, fitting, gain control)

__all__ = ["db3_filters", "dwt1", "idwt1", "dwt2", "idwt2", "OracleSystem",
           "AugmentedReconstructor", "pcg", "aug_pcg", "exact_solution", "warm_start_inputs",
           "warm_start_correction", "warm_start_step"]
