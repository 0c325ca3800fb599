// Kernels and host launchers of the p16_2c storage format.
#define LBM_FMT lbm::S_P16_2C
#define LBM_NAME p16_2c
#define LBM_HAS_F32 1
#define LBM_HAS_F64 0
#include "kern_format.inc"
