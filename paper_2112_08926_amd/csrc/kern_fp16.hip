// Kernels and host launchers of the fp16 storage format.
#define LBM_FMT lbm::S_FP16
#define LBM_NAME fp16
#define LBM_HAS_F32 1
#define LBM_HAS_F64 0
#include "kern_format.inc"
