// Kernels and host launchers of the p16_1s storage format.
#define LBM_FMT lbm::S_P16_1S
#define LBM_NAME p16_1s
#define LBM_HAS_F32 1
#define LBM_HAS_F64 0
#include "kern_format.inc"
