"""Seeded synthetic inputs for the augmented wavelet reconstructor.

This package is the only code shared by the FP64 oracle (``oracle/``) and the
GPU library's tests and benchmark.  It holds the *system description*
(telescope, guide stars, pupil masks, layer grids) and an atmosphere +
Shack-Hartmann *measurement simulator*.  It holds none of the reconstructor's
arithmetic: no wavelet transform, no discrete tomography operator, no prior,
no preconditioner and no solver.  The simulator measures continuous von Karman
phase screens sampled more finely than the reconstructor's grids (sub-sampled
subaperture-averaged gradients), i.e. it plays the role of the telescope, not
of the method.
"""
from .geometry import (ARCSEC, LayerSpec, WfsSpec, SystemSpec, subaperture_mask,
                       wfs_node_coords, fit_layer_grids, n_coeffs, n_slopes,
                       config_small, config_elt_mcao, config_elt_full, config_elt_lgs_noise, config_tiny, config_mixed, config_random_instance,
                       elt_mcao_dms, mcao_fit_directions)
from .atmosphere import FrozenFlowAtmosphere, SlopeSimulator, make_sequence

__all__ = [
    "ARCSEC", "LayerSpec", "WfsSpec", "SystemSpec", "subaperture_mask", "wfs_node_coords",
    "fit_layer_grids", "n_coeffs", "n_slopes", "config_small", "config_elt_mcao", "config_elt_full",
    "config_elt_lgs_noise",
    "config_tiny", "config_mixed", "config_random_instance", "elt_mcao_dms", "mcao_fit_directions",
    "FrozenFlowAtmosphere", "SlopeSimulator",
    "make_sequence",
]
