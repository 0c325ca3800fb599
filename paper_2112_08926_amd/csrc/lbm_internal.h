// lbm_internal.h -- structures shared by the host runtime and the HIP kernels
// of liblbm.so (not part of the public C interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Cell flag bits.  SOLID/EQ/MOVING come from the caller; NEAR marks fluid
// cells with at least one SOLID neighbour and is computed by the library so
// that only those cells look at neighbour flags during streaming.
enum : uint8_t { F_SOLID = 1, F_EQ = 2, F_MOVING = 4, F_NEAR = 8 };

enum Storage : int { S_FP64 = 0, S_FP32 = 1, S_FP16 = 2, S_FP16S = 3, S_FP16C = 4,
                     S_P16_0S = 5, S_P16_1S = 6, S_P16_2C = 7 };

// Per-lattice descriptor, read by the kernels with scalar loads.
struct LatDev {
    void* f[2];              // DDF buffers: q planes of `plane` elements each
    const uint8_t* flags;    // one byte per cell
    const uint32_t* wall_mask; // per cell: bit i = source x - c_i is a wall, bit 31 = one of them moves
    const uint32_t* near_bits; // bit g: one of the cells 64g .. 64g+63 has a wall source (F_NEAR)
    uint32_t nx, ny, nz;
    uint32_t plane;          // elements between consecutive direction planes
    double omega;            // 1/tau (TRT: symmetric rate)
    double omega_m;          // TRT antisymmetric rate
    double force[3];         // Guo body force
    double wall_u[3];        // velocity of MOVING walls
    double eq_rho;           // state of EQ cells
    double eq_u[3];
    double shift;            // 1: DDFs stored as f_i - w_i; 0: f_i (ablation)
    const void* eq_codes;    // q stored codes of the EQ cells' equilibrium
    int32_t forced;          // any force component != 0
    float inv_nx, inv_ny;    // 1/nx, 1/ny rounded to float (cell-contiguous tiles)
    int32_t pad;
    unsigned long long* nonfinite; // cell updates with a non-finite density or velocity
                                   // before the clamp, since the last initialisation
};

// One workgroup's share of a batched step: cells x0 .. x0+T-1 of row (y, z)
// of lattice `lat`; for cell-contiguous tiles, the T cells that follow
// (x0, y, z) in index order, across rows and z-planes.
struct Tile {
    uint16_t lat, x0, y, z;
};

// Software encoder table of one posit format: for each sign and each of
// kEncWindow FP32 binades (exponent fields lo .. lo + kEncWindow - 1 of the
// format's window, the exponent clamped into it), code = base + min((bits(x)
// + bias) >> shift, cap), the sign in base and the sign and exponent bits
// cancelled by bias (see table_encode).
struct EncEntry {
    uint32_t base, cap, bias, shift;
};
constexpr int kEncWindow = 64;
constexpr int kEncEntries = 2 * kEncWindow;

struct StepLaunch {
    int q, storage, arith, collision;
    int block, cpl;
    int dense;               // batched over cell-contiguous tiles of `block` cells
    int parity;
    const LatDev* lats;      // batched: device array of descriptors
    const Tile* tiles;       // batched: device array of tiles
    uint32_t ntiles;
    uint32_t grid;           // batched: workgroups (persistent grid or ntiles)
    const EncEntry* enc;     // device table for FP16C and the posits, or null
    hipStream_t stream;
};

// Host entry points, dispatching on the storage format (lbm_runtime.hip).
hipError_t launch_step_single(const StepLaunch& s, const LatDev& lat);
hipError_t launch_step_batched(const StepLaunch& s);
hipError_t launch_init(int q, int storage, int arith, const LatDev& lat, const double* rho,
                       const double* u, const EncEntry* enc, hipStream_t st);
hipError_t launch_moments(int q, int storage, int arith, const LatDev& lat, int parity,
                          double* rho, double* u, hipStream_t st);
hipError_t launch_eq_codes(int q, int storage, int arith, const LatDev& lat, void* out,
                           const EncEntry* enc, hipStream_t st);

// Per-format launch hooks, defined in kern_<format>.hip.
#define LBM_DECLARE_FORMAT(NAME)                                                              \
    hipError_t step_single_##NAME(const StepLaunch& s, const LatDev& lat);                   \
    hipError_t step_batched_##NAME(const StepLaunch& s);                                     \
    hipError_t step_diag_##NAME(const StepLaunch& s, const LatDev& lat, const double* u_ref, \
                                double* partials, uint32_t segs);                            \
    hipError_t init_##NAME(int q, int arith, const LatDev& lat, const double* rho,           \
                           const double* u, const EncEntry* enc, hipStream_t st);            \
    hipError_t moments_##NAME(int q, int arith, const LatDev& lat, int parity, double* rho,  \
                              double* u, hipStream_t st);                                    \
    hipError_t eq_codes_##NAME(int q, int arith, const LatDev& lat, void* out,               \
                               const EncEntry* enc, hipStream_t st);                         \
    hipError_t diag_##NAME(int q, int arith, const LatDev& lat, int parity,                  \
                           const double* u_ref, double* partials, uint32_t segs, hipStream_t st);
LBM_DECLARE_FORMAT(fp64)
LBM_DECLARE_FORMAT(fp32)
LBM_DECLARE_FORMAT(fp16)
LBM_DECLARE_FORMAT(fp16s)
LBM_DECLARE_FORMAT(fp16c)
LBM_DECLARE_FORMAT(p16_0s)
LBM_DECLARE_FORMAT(p16_1s)
LBM_DECLARE_FORMAT(p16_2c)
#undef LBM_DECLARE_FORMAT

constexpr int kDiagThreads = 512;   // threads per workgroup of the first pass = cells per row tile
constexpr int kDiagFields = 12;     // mass, mom x3, ke, err2, ref2, force x3, nonfinite, max |u|^2
constexpr int kDiagReduceBlocks = 512;  // workgroups of the second pass (each a fixed range of tiles)

}  // namespace lbm
