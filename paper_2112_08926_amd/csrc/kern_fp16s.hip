// Kernels and host launchers of the fp16s storage format.
#define LBM_FMT lbm::S_FP16S
#define LBM_NAME fp16s
#define LBM_HAS_F32 1
#define LBM_HAS_F64 0
#include "kern_format.inc"
