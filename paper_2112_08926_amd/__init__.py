"""MI355X (gfx950) lattice Boltzmann hot path of Lehmann et al., arXiv
2112.08926: fused pull stream-collide with SRT/TRT collision, bounce-back,
Guo forcing, FP32 arithmetic over FP64/FP32/16-bit DDF storage, FP64
diagnostics and batched ensembles.

All computation runs in the HIP kernels of ``liblbm.so`` behind the C
interface of ``include/lbm.h``; this package only marshals arguments
(``_lib`` mirrors the C functions under the same names, ``Lattices`` is a
small convenience wrapper).  PyTorch provides the stream and, optionally, the
device allocator.  There is no CPU fallback: importing fails loudly when the
library is missing.
"""
from . import tuning  # noqa: F401
from ._lib import (  # noqa: F401
    ARITH, COLLISION, FLAG_EQ, FLAG_MOVING, FLAG_SOLID, LAUNCH_BATCHED, LAUNCH_PER_LATTICE,
    PROBE, STORAGE, LbmDiag, LbmError, LbmInfo, LbmLaunch, LbmParams, Lattices, lbm_autotune,
    lbm_copy_probe, lbm_create, lbm_decode, lbm_destroy, lbm_diagnostics, lbm_diagnostics_noalloc, lbm_encode,
    lbm_get_ddf, lbm_get_launch, lbm_get_rho_u, lbm_info_get, lbm_last_error, lbm_memory_probe, lbm_set_boundaries,
    lbm_step_diagnostics,
    lbm_set_ddf, lbm_set_launch, lbm_set_rho_u, lbm_step, lbm_synchronize, library, library_id, library_path,
    make_params,
)
