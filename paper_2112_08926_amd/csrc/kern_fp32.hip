// Kernels and host launchers of the fp32 storage format.
#define LBM_FMT lbm::S_FP32
#define LBM_NAME fp32
#define LBM_HAS_F32 1
#define LBM_HAS_F64 1
#include "kern_format.inc"
