// Kernels and host launchers of the p16_0s storage format.
#define LBM_FMT lbm::S_P16_0S
#define LBM_NAME p16_0s
#define LBM_HAS_F32 1
#define LBM_HAS_F64 0
#include "kern_format.inc"
