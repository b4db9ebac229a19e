"""MI355X-native augmented wavelet reconstructor (augmented FEWHA): HIP kernels behind the
C ABI of include/fewha.h, with a thin ctypes binding."""
from ._lib import (FewhaContext, FewhaError, LoopContext, UNetContext, LOOP_DM_SLOPES, LOOP_FIT, decode_info, fewha_workspace_size, load_library,
                   make_config, PIECE_A, PIECE_AT, PIECE_WINV, PIECE_WINVT, EXPORTS, LIB_PATH)

__all__ = ["FewhaContext", "FewhaError", "LoopContext", "UNetContext", "LOOP_DM_SLOPES", "LOOP_FIT", "decode_info", "fewha_workspace_size", "load_library", "make_config",
           "PIECE_A", "PIECE_AT", "PIECE_WINV", "PIECE_WINVT", "EXPORTS", "LIB_PATH"]
