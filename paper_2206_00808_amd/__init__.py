"""MI355X-native hot path of fully relativistic (spinor) GW, Epsilon stage.

arXiv:2206.00808, Sec. II: spinor plane-wave matrix elements M_vc(q+G), the
polarizability chi0_GG'(q) on the imaginary axis (and on the real axis with
broadening) and eps^-1, as hand-written HIP
kernels for gfx950 behind the C ABI in include/gw.h.  This package is the thin
Python binding over that library; it raises ImportError when the library has
not been built.
"""
from .binding import (  # noqa: F401
    Context, GwError, QDesc,
    GW_OK, GW_EINVAL, GW_ENOMEM, GW_EDEVICE, GW_EALIAS, GW_ESINGULAR, GW_ENOTTRAINED,
    GW_EUNSUPPORTED, GW_EFALLBACK, GW_C128, GW_C64, GW_PREC_FP64, GW_PREC_SPLITBF16,
    GW_CLOSURE_INFER, GW_CLOSURE_TRAIN_STEP, GW_CLOSURE_FULL_FALLBACK,
    gw_mtxel_spinor, gw_chi0_accumulate, gw_epsinv, gw_chi0_accumulate_real, gw_epsinv_lu,
    gw_head_dipole, gw_screened_w, gw_sigma_sx, gw_unfold_spinor, gw_gpp_modes, gw_sigma_gpp, gw_chi0_symmetrize, gw_bse_kernel,
    gw_little_group, gw_kgrid_orbits, gw_epsinv_lowrank,
    gw_lowrank_basis, gw_mtxel_project, gw_epsinv_from_basis, gw_peak_probe,
    status_string, EXPORTED, LIB_PATH,
)
