"""MI355X (gfx950) line-by-line opacity: the hot path of HELIOS-K 2.0 (arXiv:2101.02005).

The computation lives in libhk.so (hand-written HIP, C ABI in include/hk.h); this package is
its Python binding. ``HkOpacityFn`` wraps the forward and backward calls for autograd."""
from ._lib import (CLASS_NAMES, CUT_DOPPLER, CUT_FIXED, CUT_LORENTZ, HK_EDEVICE, HK_EINVAL,  # noqa: F401
                   HK_ENOMEM, HK_EUNSUPPORTED, HK_OK, PROFILE_BINNED_GAUSS, PROFILE_DOPPLER, PROFILE_LORENTZ,
                   PROFILE_VOIGT, Grid, HkError, LineOverride, Lines, Options, Species, grid,
                   hk_debug_cut_bounds, hk_debug_grid_records, hk_debug_line_params, hk_debug_sorted,
                   hk_empty_cache, hk_get_timings, hk_noalloc_max_bytes, hk_opacity, hk_opacity_backward,
                   hk_opacity_batched, hk_opacity_hitran, hk_opacity_noalloc, hk_opacity_stream, hk_prepare_lines,
                   hk_prepare_lines_hitran, hk_release_lines,
                   hk_workspace_size, hk_workspace_size_ex, load, options, species)
from .autograd import HkOpacityFn, opacity  # noqa: F401,E402
