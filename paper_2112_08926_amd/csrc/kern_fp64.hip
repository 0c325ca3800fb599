// Kernels and host launchers of the fp64 storage format.
#define LBM_FMT lbm::S_FP64
#define LBM_NAME fp64
#define LBM_HAS_F32 0
#define LBM_HAS_F64 1
#include "kern_format.inc"
