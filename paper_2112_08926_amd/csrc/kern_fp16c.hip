// Kernels and host launchers of the fp16c storage format.
#define LBM_FMT lbm::S_FP16C
#define LBM_NAME fp16c
#define LBM_HAS_F32 1
#define LBM_HAS_F64 0
#include "kern_format.inc"
