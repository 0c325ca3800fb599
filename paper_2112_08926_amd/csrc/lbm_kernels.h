// lbm_kernels.h -- HIP kernels of the fused pull stream-collide step and its
// companions (initialisation, moments, FP64 diagnostics) for gfx950.
//
// Method (paper: appendix "LBM equations in a nutshell" with DDF shifting,
// Sec. 2.2, and the D3Q19 SRT kernel listing):
//   pull:     f_i(x) <- f_i^A(x - c_i); a wall source gives f_opp(i)^A(x)
//             (mid-grid bounce-back), plus 6 w_i c_i.u_w off a moving wall;
//   fields:   rho = f_0 + f_1 + ... + 1 (the 1 last), rho u = alternating
//             pair sums (+ F/2 with the Guo force), u clamped to +-c;
//   feq:      w_i rho (1/2 (B^2 + C) + B) + w_i (rho - 1), B = 3 c_i.u,
//             C = -3 u.u -- three FMAs per direction;
//   collide:  SRT f' = (1 - w) f + w feq (+ (1 - w/2) S_i), or TRT on the
//             symmetric/antisymmetric parts of each opposite pair;
//   store:    f'_i -> B at x, encoded in the storage format.
//
// Work decomposition (one lattice, or one tile of an ensemble): a workgroup
// owns `block` consecutive cells of one x-row (y, z).  The nine source rows
// (y +- 1, z +- 1) and their periodic wrap are workgroup-uniform, so every
// direction's source address is a scalar base (plane + source row) plus a
// per-lane x offset from {x-1, x, x+1}: no integer division per cell, and
// each direction is one contiguous, coalesced segment of a source row.  A
// row's x-shifted loads stay inside that row (periodic wrap), so a row's
// cache lines are fetched by one workgroup only.  No neighbour flag is read
// per direction: a per-cell mask of wall sources, precomputed with the
// flags, is read only by wavefronts that a bitmap of 64-cell groups marks as
// holding a cell next to a wall (F_NEAR).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "lbm_codecs.h"
#include "lbm_internal.h"

namespace lbm {

// ------------------------------------------------------------ velocity sets
// D3Q19: 0 rest, then opposite pairs in the order of the paper's listing
// (+00 -00, 0+0 0-0, 00+ 00-, ++0 --0, +0+ -0-, 0++ 0--, +-0 -+0, +0- -0+,
// 0+- 0-+); weights 1/3, 1/18, 1/36.  D3Q27 appends the corner pairs
// (+++ ---, ++- --+, +-+ -+-, -++ +--); weights 8/27, 2/27, 1/54, 1/216.
// D2Q9 (Table 1; the paper's Taylor-Green runs): rest, +x -x, +y -y,
// ++ --, +- -+; weights 4/9, 1/9, 1/36.  D3Q15 (Table 1): rest, the six
// faces as in D3Q19, the corner pairs as in D3Q27; weights 2/9, 1/9, 1/72.
// Every set: direction 0 at rest, directions 2k-1 and 2k opposite.
template <int Q> struct VelSet;

struct VelSetTables {
    static constexpr int c[27][3] = {
        { 0, 0, 0},
        { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0}, { 0, 0, 1}, { 0, 0,-1},
        { 1, 1, 0}, {-1,-1, 0}, { 1, 0, 1}, {-1, 0,-1}, { 0, 1, 1}, { 0,-1,-1},
        { 1,-1, 0}, {-1, 1, 0}, { 1, 0,-1}, {-1, 0, 1}, { 0, 1,-1}, { 0,-1, 1},
        { 1, 1, 1}, {-1,-1,-1}, { 1, 1,-1}, {-1,-1, 1}, { 1,-1, 1}, {-1, 1,-1},
        {-1, 1, 1}, { 1,-1,-1}};
};

template <> struct VelSet<19> : VelSetTables {
    static constexpr int Q = 19;
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
};
template <> struct VelSet<27> : VelSetTables {
    static constexpr int Q = 27;
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 8.0 / 27.0 : (i < 7 ? 2.0 / 27.0 : (i < 19 ? 1.0 / 54.0 : 1.0 / 216.0));
    }
};
template <> struct VelSet<9> {
    static constexpr int Q = 9;
    static constexpr int c[9][3] = {
        { 0, 0, 0}, { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0},
        { 1, 1, 0}, {-1,-1, 0}, { 1,-1, 0}, {-1, 1, 0}};
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
};
template <> struct VelSet<15> {
    static constexpr int Q = 15;
    static constexpr int c[15][3] = {
        { 0, 0, 0},
        { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0}, { 0, 0, 1}, { 0, 0,-1},
        { 1, 1, 1}, {-1,-1,-1}, { 1, 1,-1}, {-1,-1, 1}, { 1,-1, 1}, {-1, 1,-1},
        {-1, 1, 1}, { 1,-1,-1}};
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 2.0 / 9.0 : (i < 7 ? 1.0 / 9.0 : 1.0 / 72.0);
    }
};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// The listing's velocity limit, OpenCL's clamp(v, -c, c) with c = 1/sqrt(3),
// which that language defines as fmin(fmax(v, -c), c).  fmax and fmin return
// the other operand when one is NaN, so a NaN component becomes -c (a cell of
// zero density would otherwise turn its whole equilibrium into NaN).
template <class A> __device__ __forceinline__ A clamp_c(A v) {
    const A cs = (A)0.57735026918962576451;   // lattice speed of sound 1/sqrt(3)
    if constexpr (sizeof(A) == 4) return __builtin_fminf(__builtin_fmaxf(v, -cs), cs);
    else return __builtin_fmin(__builtin_fmax(v, -cs), cs);
}

// c . v for a lattice direction with components in {-1, 0, 1}, written with
// additions only (a multiply by a zero component is not foldable in IEEE
// arithmetic); the components are compile-time constants after unrolling.
template <class A>
__device__ __forceinline__ A cdot(int cx, int cy, int cz, A x, A y, A z) {
    A s = cx > 0 ? x : (cx < 0 ? -x : (A)0);
    bool any = cx != 0;
    if (cy != 0) { s = any ? (cy > 0 ? s + y : s - y) : (cy > 0 ? y : -y); any = true; }
    if (cz != 0) { s = any ? (cz > 0 ? s + z : s - z) : (cz > 0 ? z : -z); any = true; }
    return s;
}
template <int Q, class A>
__device__ __forceinline__ A cdot_i(int i, A x, A y, A z) {
    return cdot<A>(VelSet<Q>::c[i][0], VelSet<Q>::c[i][1], VelSet<Q>::c[i][2], x, y, z);
}

// ------------------------------------------------------------ geometry of a row
struct RowCtx {
    uint32_t rows[9];   // cell index of x = 0 of row (y+dy, z+dz), index (dy+1) + 3 (dz+1)
};

__device__ __forceinline__ uint32_t wrap_add(uint32_t a, int d, uint32_t n) {
    return d < 0 ? (a == 0 ? n - 1 : a - 1) : (d > 0 ? (a + 1 == n ? 0 : a + 1) : a);
}

__device__ __forceinline__ void make_rows(const LatDev& L, uint32_t y, uint32_t z, RowCtx& rc) {
#pragma unroll
    for (int dz = -1; dz <= 1; dz++)
#pragma unroll
        for (int dy = -1; dy <= 1; dy++) {
            const uint32_t yy = wrap_add(y, dy, L.ny), zz = wrap_add(z, dz, L.nz);
            rc.rows[(dy + 1) + 3 * (dz + 1)] = (yy + zz * L.ny) * L.nx;
        }
}

// Source row and x of direction i for a cell at (x, row (y, z)): x - c_i.
template <int Q>
__device__ __forceinline__ uint32_t src_row(const RowCtx& rc, int i) {
    return rc.rows[(1 - VelSet<Q>::c[i][1]) + 3 * (1 - VelSet<Q>::c[i][2])];
}
template <int Q>
__device__ __forceinline__ uint32_t src_x(int i, uint32_t x, uint32_t xm, uint32_t xp) {
    return VelSet<Q>::c[i][0] > 0 ? xm : (VelSet<Q>::c[i][0] < 0 ? xp : x);
}

// ------------------------------------------------------------ pull with bounce-back
// Element `idx` of a row/plane at a wavefront-uniform base: the byte offset
// is formed in 32 bits so that the load/store can use a scalar 64-bit base
// plus a 32-bit per-lane offset (no 64-bit address arithmetic per lane).
// Every offset passed here is below 2^32 bytes: DDF planes (N * bytes per
// DDF < 2^32) and byte-per-cell arrays (N < 2^31); the 4-byte-per-cell wall
// mask goes through ld_mask.
// The pointers are in the global address space: every buffer of the library
// is device memory.  Saying so matters where a pointer comes from a
// descriptor table in memory rather than a kernel argument; the compiler
// would otherwise emit flat instructions.
#define LBM_GLOBAL __attribute__((address_space(1)))
// Clang vector types for wide accesses (HIP's uint2/uint4 are classes whose
// copy constructor takes a generic reference, which loses the address space).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ T ld_off(const T* base, uint32_t idx) {
    return *(const LBM_GLOBAL T*)((const LBM_GLOBAL char*)base + (uint32_t)(idx * (uint32_t)sizeof(T)));
}
// The wall mask of cell n.  It holds 4 bytes per cell, so its byte offset can
// pass 2^32 in lattices of 2^30 cells or more (allowed with 16-bit storage):
// the address is formed in 64 bits.
__device__ __forceinline__ uint32_t ld_mask(const uint32_t* mask, uint32_t n) {
    return *(const LBM_GLOBAL uint32_t*)(mask + (size_t)n);
}
// New DDFs are streamed out: nontemporal stores (each element is written
// once per step and read back only by the next step).
template <class T>
__device__ __forceinline__ void st_off(T* base, uint32_t idx, T v) {
    __builtin_nontemporal_store(v, (LBM_GLOBAL T*)((LBM_GLOBAL char*)base + (uint32_t)(idx * (uint32_t)sizeof(T))));
}

// 2^e for e >= 0, exactly, at compile time.
constexpr double exp2i(int e) {
    double r = 1.0;
    for (int k = 0; k < e; k++) r *= 2.0;
    return r;
}

// RAW: values in the storage's raw units (2^-kRawExp), as the step uses them;
// otherwise physical values (moments and diagnostics).
template <int Q, int F, class A, bool RAW>
__device__ __forceinline__ A load_ddf(typename Codec<F>::T v) {
    if constexpr (RAW) return Codec<F>::template load_raw<A>(v);
    else return Codec<F>::template load<A>(v);
}
template <int F, bool RAW>
constexpr double kRawScale = RAW ? exp2i(Codec<F>::kRawExp) : 1.0;   // a constant: evaluated at compile time

// Whether a wavefront whose cells lie in n_first .. n_first + 63 holds a cell
// with a wall source: bits g and g + 1 (g = n_first / 64) of the lattice's
// group bitmap, read with one scalar load before any DDF load is issued.
// A lattice without walls has no bitmap (null) and skips the read.
__device__ __forceinline__ bool wave_has_walls(const LatDev& L, uint32_t n_first) {
    if (L.near_bits == nullptr) return false;
    typedef const __attribute__((address_space(4))) uint32_t* ConstPtr;
    const uint32_t g = (uint32_t)__builtin_amdgcn_readfirstlane((int)(n_first >> 6));
    const ConstPtr b = (ConstPtr)(const void*)L.near_bits + (g >> 5);
    const uint64_t v = (uint64_t)b[0] | ((uint64_t)b[1] << 32);
    return ((v >> (g & 31)) & 3u) != 0;
}

// LANE_ROWS: the row bases differ between lanes (cell-contiguous tiles), so
// the whole in-plane index is the per-lane offset; otherwise the row base
// is wavefront-uniform and folded into the scalar base address.
// walls (wavefront-uniform): some cell of the wavefront may have a wall
// source.  A wall source hands back what this cell sent towards it last
// step, its own opposite DDF: such a direction takes that address in the
// same load instruction (chosen per lane from the cell's wall mask), so a
// wavefront next to a wall issues one extra load (the mask), not one per
// bounced direction.
// Decodes the Q pulled codes; for the sign-magnitude posits, with the
// cheaper decoder when no code of the wavefront has a run of ones as regime
// (a wavefront-uniform choice: values below 2^-7 everywhere, as in most of a
// flow's cells), else with the full one.
template <int Q, int F, class A, bool RAW>
__device__ __forceinline__ void decode_pulled(const typename Codec<F>::T (&c)[Q], A (&f)[Q]) {
    if constexpr (ZerosRun<F>::value) {
        uint32_t any = 0;
#pragma unroll
        for (int i = 0; i < Q; i++) any |= (uint32_t)c[i];
        if (__any((any & 0x4000u) != 0)) {
#pragma unroll
            for (int i = 0; i < Q; i++) f[i] = load_ddf<Q, F, A, RAW>(c[i]);
        } else {
#pragma unroll
            for (int i = 0; i < Q; i++) f[i] = ZerosRun<F>::template load<A>(c[i]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; i++) f[i] = load_ddf<Q, F, A, RAW>(c[i]);
    }
}

template <int Q, int F, class A, bool RAW, bool LANE_ROWS = false>
__device__ __forceinline__ void pull(const LatDev& L, const typename Codec<F>::T* __restrict__ src,
                                     const RowCtx& rc, uint32_t x, uint32_t xm, uint32_t xp,
                                     uint32_t n, bool walls, A (&f)[Q]) {
    using T = typename Codec<F>::T;
    const size_t plane = L.plane;
    T c[Q];
    if (!walls) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            if constexpr (LANE_ROWS) {
                c[i] = ld_off(src + (size_t)i * plane, src_row<Q>(rc, i) + src_x<Q>(i, x, xm, xp));
            } else {
                const T* p = src + ((size_t)i * plane + src_row<Q>(rc, i));
                c[i] = ld_off(p, src_x<Q>(i, x, xm, xp));
            }
        }
        decode_pulled<Q, F, A, RAW>(c, f);
        return;
    }
    const uint32_t m = ld_mask(L.wall_mask, n);
    // All Q loads first, addresses chosen by selects (no branch between the
    // loads, so they are all in flight at once) ...
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const T* p;
        uint32_t idx;
        if constexpr (LANE_ROWS) {
            p = src + (size_t)i * plane;
            idx = src_row<Q>(rc, i) + src_x<Q>(i, x, xm, xp);
        } else {
            p = src + ((size_t)i * plane + src_row<Q>(rc, i));
            idx = src_x<Q>(i, x, xm, xp);
        }
        if (i > 0) {
            const bool wall = (m >> i) & 1u;
            p = wall ? src + (size_t)opp(i) * plane : p;
            idx = wall ? n : idx;
        }
        c[i] = ld_off(p, idx);
    }
    decode_pulled<Q, F, A, RAW>(c, f);
    // ... then the moving walls' momentum, only in wavefronts next to one.
    if (__any((m & 0x80000000u) != 0)) {
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (((m >> i) & 1u) && (m & 0x80000000u)) {
                const uint8_t fs = ld_off(L.flags, src_row<Q>(rc, i) + src_x<Q>(i, x, xm, xp));
                if (fs & F_MOVING) {
                    const A cu = (A)(VelSet<Q>::c[i][0] * L.wall_u[0] + VelSet<Q>::c[i][1] * L.wall_u[1] +
                                     VelSet<Q>::c[i][2] * L.wall_u[2]);
                    f[i] += (A)(6.0 * VelSet<Q>::w(i) * kRawScale<F, RAW>) * cu;
                }
            }
        }
    }
}

// The pull's parts for the diagnostics kernels, which also need the wall
// mask and the bounced directions' values before the moving walls' term
// (those are this cell's own opposite DDFs, which the momentum exchange
// reads).  The same loads, decode (decode_pulled) and wall terms as pull,
// which keeps them in one body for the step kernels.
// pull_codes: the Q loads; m = the cell's wall mask in a wavefront with
// walls (a wall source hands back this cell's own opposite DDF, taken by the
// same load instruction with a per-lane address), else 0.
template <int Q, int F>
__device__ __forceinline__ void pull_codes(const LatDev& L, const typename Codec<F>::T* __restrict__ src,
                                           const RowCtx& rc, uint32_t x, uint32_t xm, uint32_t xp, uint32_t n,
                                           bool walls, typename Codec<F>::T (&c)[Q], uint32_t& m) {
    using T = typename Codec<F>::T;
    const size_t plane = L.plane;
    if (!walls) {
        m = 0;
#pragma unroll
        for (int i = 0; i < Q; i++) c[i] = ld_off(src + ((size_t)i * plane + src_row<Q>(rc, i)), src_x<Q>(i, x, xm, xp));
        return;
    }
    m = ld_mask(L.wall_mask, n);
    constexpr uint32_t b = sizeof(T);
    if ((uint64_t)plane * (2 * b) < (1ull << 32)) {
        // where two planes fit in 32-bit byte offsets, each load takes one
        // scalar base, the lower plane of the direction's opposite pair
        // (directions 2k-1 and 2k are opposite) at the lower of the source
        // row and this cell's row (n = own + x), plus a per-lane offset
        // picked by one select: the source cell's or, from a wall, this
        // cell's in the opposite plane (fewer instructions than two 64-bit
        // addresses per lane; both offsets stay below two planes)
        const LBM_GLOBAL char* base0 = (const LBM_GLOBAL char*)src;
        const uint32_t pb = (uint32_t)plane * b;
        const uint32_t own = rc.rows[4];
        const uint32_t xb = x * b, xmb = xm * b, xpb = xp * b;
        c[0] = ld_off(src + own, x);
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const int lo = (i & 1) ? i : i - 1;
            const int cx = VelSet<Q>::c[i][0];
            const uint32_t ri = src_row<Q>(rc, i);
            const uint32_t r0 = ri < own ? ri : own;
            const uint32_t sxb = cx > 0 ? xmb : (cx < 0 ? xpb : xb);
            const uint32_t normal = ((i & 1) ? 0u : pb) + (ri - r0) * b + sxb;
            const uint32_t bounce = ((i & 1) ? pb : 0u) + (own - r0) * b + xb;
            c[i] = *(const LBM_GLOBAL T*)(base0 + ((size_t)lo * plane + r0) * b + (((m >> i) & 1u) ? bounce : normal));
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const T* p = src + ((size_t)i * plane + src_row<Q>(rc, i));
        uint32_t idx = src_x<Q>(i, x, xm, xp);
        if (i > 0) {
            const bool wall = (m >> i) & 1u;
            p = wall ? src + (size_t)opp(i) * plane : p;
            idx = wall ? n : idx;
        }
        c[i] = ld_off(p, idx);
    }
}
// add_moving_walls: to the decoded values (RAW: the step's raw units), the
// moving walls' momentum, only in wavefronts next to one.
template <int Q, int F, class A, bool RAW>
__device__ __forceinline__ void add_moving_walls(const LatDev& L, const RowCtx& rc, uint32_t x, uint32_t xm,
                                                 uint32_t xp, uint32_t m, A (&f)[Q]) {
    if (__any((m & 0x80000000u) != 0)) {
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (((m >> i) & 1u) && (m & 0x80000000u)) {
                const uint8_t fs = ld_off(L.flags, src_row<Q>(rc, i) + src_x<Q>(i, x, xm, xp));
                if (fs & F_MOVING) {
                    const A cu = (A)(VelSet<Q>::c[i][0] * L.wall_u[0] + VelSet<Q>::c[i][1] * L.wall_u[1] +
                                     VelSet<Q>::c[i][2] * L.wall_u[2]);
                    f[i] += (A)(6.0 * VelSet<Q>::w(i) * kRawScale<F, RAW>) * cu;
                }
            }
        }
    }
}

// ------------------------------------------------------------ fields
// Momentum by alternating pair sums (Sec. 2.2), in index order.
template <int Q, class A>
__device__ __forceinline__ void fields_j(const A (&f)[Q], A (&j)[3]) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        A s = (A)0;
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const int c = VelSet<Q>::c[i][a];
            if (c > 0) { s += f[i]; s -= f[i + 1]; }
            else if (c < 0) { s += f[i + 1]; s -= f[i]; }
        }
        j[a] = s;
    }
}

// Sum of the DDFs, f_0 first then in index order.
template <int Q, class A>
__device__ __forceinline__ A fields_sum(const A (&f)[Q]) {
    A r = f[0];
#pragma unroll
    for (int i = 1; i < Q; i++) r += f[i];
    return r;
}

template <int Q, class A>
__device__ __forceinline__ void fields(const A (&f)[Q], A shift, A& rho, A (&j)[3]) {
    A r = f[0];
#pragma unroll
    for (int i = 1; i < Q; i++) r += f[i];
    rho = r + shift;                                         // the 1 of the shift last
    fields_j<Q, A>(f, j);
}

// ------------------------------------------------------------ collision
// Fused multiply-add in the arithmetic precision (__builtin_fma alone would
// promote float operands to double).
template <class A> __device__ __forceinline__ A fmaa(A a, A b, A c) {
    if constexpr (sizeof(A) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

// ------------------------------------------------------------ MRT (D3Q19)
// Moment basis of d'Humieres et al. (2002), each row a polynomial in c_i
// (c2 = |c_i|^2): rho 1; e 19 c2 - 30; eps (21 c2^2 - 53 c2 + 24)/2; j_a c_a
// and q_a (5 c2 - 9) c_a interleaved for x, y, z; 3p_xx 3 cx^2 - c2;
// 3pi_xx (3 c2 - 5)(3 cx^2 - c2); p_ww cy^2 - cz^2; pi_ww (3 c2 - 5)(cy^2 - cz^2);
// p_xy, p_yz, p_xz; m_x (cy^2 - cz^2) cx, m_y (cz^2 - cx^2) cy,
// m_z (cx^2 - cy^2) cz.  The rows are orthogonal: M^-1 = M^T diag(1/|row|^2).
__host__ __device__ constexpr int mrt_m(int k, int i) {
    const int cx = VelSet<19>::c[i][0], cy = VelSet<19>::c[i][1], cz = VelSet<19>::c[i][2];
    const int c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return cx;
    case 4: return (5 * c2 - 9) * cx;
    case 5: return cy;
    case 6: return (5 * c2 - 9) * cy;
    case 7: return cz;
    case 8: return (5 * c2 - 9) * cz;
    case 9: return 3 * cx * cx - c2;
    case 10: return (3 * c2 - 5) * (3 * cx * cx - c2);
    case 11: return cy * cy - cz * cz;
    case 12: return (3 * c2 - 5) * (cy * cy - cz * cz);
    case 13: return cx * cy;
    case 14: return cy * cz;
    case 15: return cx * cz;
    case 16: return (cy * cy - cz * cz) * cx;
    case 17: return (cz * cz - cx * cx) * cy;
    default: return (cx * cx - cy * cy) * cz;
    }
}
__host__ __device__ constexpr int mrt_norm2(int k) {
    int n = 0;
    for (int i = 0; i < 19; i++) n += mrt_m(k, i) * mrt_m(k, i);
    return n;
}
// Relaxation rate of moment k: 0 for the conserved rho and j, omega = 1/tau
// for the shear moments (3p_xx, p_ww, p_xy, p_yz, p_xz), and the fixed rates
// of d'Humieres et al. for the others.
__host__ __device__ constexpr double mrt_rate_fixed(int k) {
    switch (k) {
    case 1: return 1.19;
    case 2: case 10: case 12: return 1.4;
    case 4: case 6: case 8: return 1.2;
    case 16: case 17: case 18: return 1.98;
    default: return 0.0;
    }
}
__host__ __device__ constexpr bool mrt_shear(int k) { return k == 9 || k == 11 || k == 13 || k == 14 || k == 15; }
__host__ __device__ constexpr bool mrt_conserved(int k) { return k == 0 || k == 3 || k == 5 || k == 7; }

// Every row is even or odd in c (rho, e, eps and the stress moments even; j,
// q and m odd), so a direction and its opposite carry the same coefficient
// up to the sign: the products are taken over the 9 opposite pairs, even
// rows on the pair sums and odd rows on the pair differences, as fold
// expressions over compile-time indices so that each coefficient is a
// constant and the zero ones vanish.
__host__ __device__ constexpr bool mrt_odd(int k) { return (k >= 3 && k <= 8) || k >= 16; }
// Row K of M applied to v, given v0 = v[0], s[p] = v[2p+1] + v[2p+2] and
// a[p] = v[2p+1] - v[2p+2].
template <class A, int K, int... P>
__device__ __forceinline__ A mrt_row(A v0, const A (&s)[9], const A (&a)[9], std::integer_sequence<int, P...>) {
    A acc = (A)0;
    if constexpr (!mrt_odd(K) && mrt_m(K, 0) != 0) acc = (A)mrt_m(K, 0) * v0;
    ((acc = mrt_m(K, 2 * P + 1) != 0 ? fmaa((A)mrt_m(K, 2 * P + 1), mrt_odd(K) ? a[P] : s[P], acc) : acc), ...);
    return acc;
}
// Column entries of M^T r for direction I over the rows K of one parity.
template <class A, int I, bool ODD, int... K>
__device__ __forceinline__ A mrt_col(const A (&r)[19], std::integer_sequence<int, K...>) {
    A acc = (A)0;
    ((acc = (mrt_odd(K) == ODD && mrt_m(K, I) != 0) ? fmaa((A)mrt_m(K, I), r[K], acc) : acc), ...);
    return acc;
}
// Relaxed moment K divided by |row K|^2: S_K (M d)_K, minus (1 - S_K/2)
// (M src)_K with a body force (FORCED).
template <class A, int K, bool FORCED>
__device__ __forceinline__ A mrt_relax_one(A w, A d0, const A (&ds)[9], const A (&da)[9], A f0,
                                           const A (&fs)[9], const A (&fa)[9]) {
    constexpr auto pairs = std::make_integer_sequence<int, 9>{};
    const A sk = mrt_shear(K) ? w : (A)mrt_rate_fixed(K);
    A rk = (A)0;
    if constexpr (!mrt_conserved(K)) rk = sk * mrt_row<A, K>(d0, ds, da, pairs);
    if constexpr (FORCED) rk = fmaa(-((A)1 - (A)0.5 * sk), mrt_row<A, K>(f0, fs, fa, pairs), rk);
    return rk * (A)(1.0 / mrt_norm2(K));
}
template <class A, bool FORCED, int... K>
__device__ __forceinline__ void mrt_relax(A w, const A (&d)[19], const A (&src)[19], A (&r)[19],
                                          std::integer_sequence<int, K...>) {
    A ds[9], da[9], fs[9], fa[9];
#pragma unroll
    for (int p = 0; p < 9; p++) {
        ds[p] = d[2 * p + 1] + d[2 * p + 2];
        da[p] = d[2 * p + 1] - d[2 * p + 2];
        fs[p] = FORCED ? src[2 * p + 1] + src[2 * p + 2] : (A)0;
        fa[p] = FORCED ? src[2 * p + 1] - src[2 * p + 2] : (A)0;
    }
    ((r[K] = mrt_relax_one<A, K, FORCED>(w, d[0], ds, da, src[0], fs, fa)), ...);
}
// fo = f - M^T r: per pair, the even rows' sum E and the odd rows' sum O give
// f_i - (E + O) and f_opp - (E - O).
template <class A, int... P>
__device__ __forceinline__ void mrt_back(const A (&f)[19], const A (&r)[19], A (&fo)[19],
                                         std::integer_sequence<int, P...>) {
    constexpr auto rows = std::make_integer_sequence<int, 19>{};
    fo[0] = f[0] - mrt_col<A, 0, false>(r, rows);
    ((fo[2 * P + 1] = f[2 * P + 1] - (mrt_col<A, 2 * P + 1, false>(r, rows) + mrt_col<A, 2 * P + 1, true>(r, rows))), ...);
    ((fo[2 * P + 2] = f[2 * P + 2] - (mrt_col<A, 2 * P + 1, false>(r, rows) - mrt_col<A, 2 * P + 1, true>(r, rows))), ...);
}

// f' = f - M^-1 [S M (f - f^eq) - (I - S/2) M S^F] with the Guo source S^F;
// values in units of 2^-E like the rest of the collision.
template <class A, int E>
__device__ __forceinline__ void collide_mrt(A w, A rho, A rhom1, A C, A u3x, A u3y, A u3z, A ux, A uy, A uz,
                                            A Fx, A Fy, A Fz, A uF, bool forced, const A (&f)[19], A feq0,
                                            A (&fo)[19]) {
    constexpr double kSc = exp2i(E);
    const A sc = (A)kSc;
    A d[19];
    d[0] = f[0] - feq0;
#pragma unroll
    for (int i = 1; i < 19; i += 2) {
        const A wi = (A)(VelSet<19>::w(i) * kSc);
        const A B = cdot_i<19, A>(i, u3x, u3y, u3z);
        const A t = fmaa(B, B, C);
        d[i] = f[i] - fmaa(wi * rho, fmaa((A)0.5, t, B), wi * rhom1);
        d[i + 1] = f[i + 1] - fmaa(wi * rho, fmaa((A)0.5, t, -B), wi * rhom1);
    }
    A r[19];                                     // relaxed moments, divided by |row|^2
    if (forced) {                                // wavefront-uniform
        A src[19];
        src[0] = sc * ((A)VelSet<19>::w(0) * ((A)(-3) * uF));
#pragma unroll
        for (int i = 1; i < 19; i += 2) {
            const A wp = (A)VelSet<19>::w(i);
            const A cF = cdot_i<19, A>(i, Fx, Fy, Fz);
            const A cu = cdot_i<19, A>(i, ux, uy, uz);
            const A sym = wp * ((A)9 * cu * cF - (A)3 * uF);
            const A anti = wp * (A)3 * cF;
            src[i] = sc * (sym + anti);
            src[i + 1] = sc * (sym - anti);
        }
        mrt_relax<A, true>(w, d, src, r, std::make_integer_sequence<int, 19>{});
    } else {
        const A none[19] = {};
        mrt_relax<A, false>(w, d, none, r, std::make_integer_sequence<int, 19>{});
    }
    mrt_back<A>(f, r, fo, std::make_integer_sequence<int, 9>{});
}

// Computes the post-collision DDFs fo[] of one cell from the pulled f[].
// f and fo are in units of 2^-E (E = the storage's raw exponent, see
// Codec::load_raw): density is sum(f) 2^-E + 1 and every term that enters
// fo is multiplied by 2^E; being powers of two these scalings are exact.
// Opposite directions i, i+1 share B (with opposite sign) and B^2 + C.
// SRT evaluates each f^eq in the paper's three-FMA order and collides with
// one FMA.  TRT needs only the pair sums and differences of f^eq, which
// have the closed forms  feq_i + feq_j = w rho (B^2 + C) + 2 w (rho - 1)
// and  feq_i - feq_j = 2 w rho B.
// EXACT_DIV: u = j / rho as the paper's listing divides (FP32/FP64 storage,
// where the division's rounding is visible); otherwise j * (1/rho) with the
// hardware reciprocal, whose error (~1e-7 relative) is far below a 16-bit
// storage step.
// bad: the density or a velocity component before the clamp is not finite
// (a blow-up that the clamp and the saturating 16-bit encoders would hide).
template <int Q, int COLL, class A, bool EXACT_DIV, int E>
__device__ __forceinline__ void collide(const LatDev& L, const A (&f)[Q], A (&fo)[Q], bool& bad) {
    static_assert(!EXACT_DIV || E == 0, "scaled units only with the reciprocal path");
    constexpr double kSc = exp2i(E);
    const A sc = (A)kSc;
    A j[3];
    const A r = fields_sum<Q, A>(f);                         // raw units
    fields_j<Q, A>(f, j);
    const A shift = (A)L.shift;                              // 1, or 0 without DDF shifting
    A rho;                                                   // the 1 of the shift added last
    if constexpr (E == 0) rho = r + shift;
    else rho = fmaa(r, (A)(1.0 / kSc), shift);
    const bool forced = L.forced != 0;
    const A Fx = (A)L.force[0], Fy = (A)L.force[1], Fz = (A)L.force[2];
    if (forced) {
        j[0] += (A)(0.5 * kSc) * Fx;
        j[1] += (A)(0.5 * kSc) * Fy;
        j[2] += (A)(0.5 * kSc) * Fz;
    }
    A vx, vy, vz;                                            // velocity before the clamp
    if constexpr (EXACT_DIV) {
        vx = j[0] / rho;
        vy = j[1] / rho;
        vz = j[2] / rho;
    } else {
        A inv;
        if constexpr (sizeof(A) == 4) inv = (A)(1.0 / kSc) * __builtin_amdgcn_rcpf(rho);
        else inv = (A)(1.0 / kSc) / rho;
        vx = j[0] * inv;
        vy = j[1] * inv;
        vz = j[2] * inv;
    }
    bad = !(__builtin_isfinite(rho) && __builtin_isfinite(vx) && __builtin_isfinite(vy) && __builtin_isfinite(vz));
    const A ux = clamp_c(vx), uy = clamp_c(vy), uz = clamp_c(vz);
    const A C = (A)(-3) * fmaa(ux, ux, fmaa(uy, uy, uz * uz));
    const A rhom1 = rho - shift;                             // rho - 1 (shifted) or rho
    const A u3x = (A)3 * ux, u3y = (A)3 * uy, u3z = (A)3 * uz;
    const A w = (A)L.omega, wm = (A)L.omega_m;
    const A uF = fmaa(ux, Fx, fmaa(uy, Fy, uz * Fz));
    const A w0 = (A)(VelSet<Q>::w(0) * kSc);
    const A feq0 = fmaa(w0 * rho, (A)0.5 * C, w0 * rhom1);

    if constexpr (COLL == 2) {
        collide_mrt<A, E>(w, rho, rhom1, C, u3x, u3y, u3z, ux, uy, uz, Fx, Fy, Fz, uF, forced, f, feq0, fo);
    } else if constexpr (COLL == 0) {
        const A omw = (A)1 - w;
        const A pre = ((A)1 - (A)0.5 * w) * sc;
        fo[0] = fmaa(omw, f[0], w * feq0);
        if (forced) fo[0] += pre * ((A)VelSet<Q>::w(0) * ((A)(-3) * uF));
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const A wi = (A)(VelSet<Q>::w(i) * kSc);
            const A B = cdot_i<Q, A>(i, u3x, u3y, u3z);
            const A t = fmaa(B, B, C);
            const A ei = fmaa(wi * rho, fmaa((A)0.5, t, B), wi * rhom1);
            const A ej = fmaa(wi * rho, fmaa((A)0.5, t, -B), wi * rhom1);
            fo[i] = fmaa(omw, f[i], w * ei);
            fo[i + 1] = fmaa(omw, f[i + 1], w * ej);
            if (forced) {
                const A wp = (A)VelSet<Q>::w(i);
                const A cF = cdot_i<Q, A>(i, Fx, Fy, Fz);
                const A cu = cdot_i<Q, A>(i, ux, uy, uz);
                const A sym = wp * ((A)9 * cu * cF - (A)3 * uF);
                const A anti = wp * (A)3 * cF;
                fo[i] += pre * (sym + anti);
                fo[i + 1] += pre * (sym - anti);
            }
        }
    } else {
        static_assert(COLL == 1, "collision operator");
        const A hw = (A)0.5 * w, hwm = (A)0.5 * wm;
        const A prep = ((A)1 - hw) * sc, prem = ((A)1 - hwm) * sc;
        fo[0] = fmaa(-w, f[0] - feq0, f[0]);
        if (forced) fo[0] += prep * ((A)VelSet<Q>::w(0) * ((A)(-3) * uF));
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const A wi = (A)(VelSet<Q>::w(i) * kSc);
            const A B = cdot_i<Q, A>(i, u3x, u3y, u3z);
            const A wr = wi * rho;
            const A esum = fmaa(wr, fmaa(B, B, C), (A)2 * wi * rhom1);
            const A edif = (A)2 * wr * B;
            const A s = (f[i] + f[i + 1]) - esum;
            const A d = (f[i] - f[i + 1]) - edif;
            fo[i] = fmaa(-hw, s, fmaa(-hwm, d, f[i]));
            fo[i + 1] = fmaa(-hw, s, fmaa(hwm, d, f[i + 1]));
            if (forced) {
                const A wp = (A)VelSet<Q>::w(i);
                const A cF = cdot_i<Q, A>(i, Fx, Fy, Fz);
                const A cu = cdot_i<Q, A>(i, ux, uy, uz);
                const A sym = wp * ((A)9 * cu * cF - (A)3 * uF);
                const A anti = wp * (A)3 * cF;
                fo[i] += prep * sym + prem * anti;
                fo[i + 1] += prep * sym - prem * anti;
            }
        }
    }
}

// What a wall or EQ cell keeps: zero DDFs, or the lattice's equilibrium
// codes.  The step writes them back unchanged, so that every wavefront
// writes whole rows: a store that leaves holes in a cache line makes the
// memory side read the line to merge it, which at a wall in every row cost
// ~15 % of the 512^3 cavity's step.
// The lattice's stored equilibrium code of direction i, the same for every
// lane: read with scalar loads (16-bit codes two to a word), so that a
// wavefront's Q codes arrive together instead of as Q dependent vector loads.
template <int F>
__device__ __forceinline__ typename Codec<F>::T eq_code(const LatDev& L, int i) {
    using T = typename Codec<F>::T;
    if constexpr (sizeof(T) == 2) {
        typedef const __attribute__((address_space(4))) uint32_t* ConstWords;
        const uint32_t w = ((ConstWords)(const void*)L.eq_codes)[i >> 1];
        return (T)((i & 1) ? (w >> 16) : (w & 0xFFFFu));
    } else {
        typedef const __attribute__((address_space(4))) T* ConstCodes;
        return ((ConstCodes)(const void*)L.eq_codes)[i];
    }
}
// The Q equilibrium codes, read only if the wavefront holds an EQ cell
// (any_eq, wavefront-uniform); zero otherwise.
template <int Q, int F>
__device__ __forceinline__ void eq_codes_if(const LatDev& L, bool any_eq, typename Codec<F>::T (&e)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; i++) e[i] = 0;
    if (any_eq) {
#pragma unroll
        for (int i = 0; i < Q; i++) e[i] = eq_code<F>(L, i);
    }
}
// The Q codes a cell (flags fl) stores: the collision's (c, encoded from
// fo), or what a wall (zero) or EQ cell (the lattice's equilibrium codes)
// keeps.  The replacement runs only in wavefronts that hold a wall or EQ
// cell (wavefront-uniform branch), so the others store the encoded values
// without per-direction selects.
template <int Q, int F, class A>
__device__ __forceinline__ void out_codes(const LatDev& L, uint32_t fl, const A (&fo)[Q], const EncEntry* tab,
                                          typename Codec<F>::T (&c)[Q]) {
    using T = typename Codec<F>::T;
    if constexpr (FixedRange<F>::value && std::is_same_v<A, float>) {
        // the arithmetic encoder where every value of the wavefront is in its
        // range (wall and EQ lanes are replaced below, whatever they hold);
        // a NaN fails the comparison and goes to the table
        bool fixed = (fl & (F_SOLID | F_EQ)) != 0;
        if (!fixed) {
            fixed = true;
#pragma unroll
            for (int i = 0; i < Q; i++) fixed = fixed && (__builtin_fabsf(fo[i]) < FixedRange<F>::kBound);
        }
        if (__all(fixed)) {
#pragma unroll
            for (int i = 0; i < Q; i++) c[i] = FixedRange<F>::store(fo[i]);
        } else {
#pragma unroll
            for (int i = 0; i < Q; i++) c[i] = Codec<F>::template store_raw<A>(fo[i], tab);
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; i++) c[i] = Codec<F>::template store_raw<A>(fo[i], tab);
    }
    if (__any((fl & (F_SOLID | F_EQ)) != 0)) {
        const bool solid = (fl & F_SOLID) != 0, eqc = (fl & F_EQ) != 0;
        T eq[Q];
        eq_codes_if<Q, F>(L, __any(eqc), eq);
#pragma unroll
        for (int i = 0; i < Q; i++) c[i] = solid ? (T)0 : (eqc ? eq[i] : c[i]);
    }
}

// Adds the wavefront's cells whose update had a non-finite density or
// velocity (`bad`) to the lattice's counter: one ballot, and, only in a
// wavefront that holds such a cell, one vector atomic by a single lane.
__device__ __forceinline__ void count_nonfinite(const LatDev& L, bool bad) {
    const uint64_t b = __ballot(bad);
    if (b != 0 && (int)__lane_id() == __builtin_ctzll(b))
        __hip_atomic_fetch_add((LBM_GLOBAL unsigned long long*)L.nonfinite, (unsigned long long)__popcll(b),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ one tile of the step
// WAVE_TABLE: `tab` is this wavefront's own LDS copy of the encoder table,
// written by direct loads the kernel issued before calling this; the
// wavefront waits for them (vmcnt) after its DDF loads, before the first
// encode.  Lanes past the row's end then do not leave early (the wavefront's
// loads must be waited for): they step the row's last cell (loads in
// bounds) and store nothing.
template <int Q, int F, class A, int COLL, bool WAVE_TABLE = false>
__device__ __forceinline__ void step_tile(const LatDev& L, uint32_t x0, uint32_t y, uint32_t z,
                                          int parity, const EncEntry* tab) {
    using T = typename Codec<F>::T;
    const bool active = x0 + threadIdx.x < L.nx;
    if constexpr (!WAVE_TABLE) {
        if (!active) return;
    }
    const uint32_t x = active ? x0 + threadIdx.x : L.nx - 1;
    RowCtx rc;
    make_rows(L, y, z, rc);
    const uint32_t n = rc.rows[4] + x;
    const uint8_t fl = ld_off(L.flags, n);
    const uint32_t xm = x == 0 ? L.nx - 1 : x - 1;
    const uint32_t xp = x + 1 == L.nx ? 0 : x + 1;
    const T* __restrict__ src = (const T*)L.f[parity];
    T* __restrict__ dst = (T*)L.f[parity ^ 1];

    // The DDF loads go out together with the flag load (every address is in
    // the lattice whatever the flag), so a wavefront waits for memory once;
    // wall and EQ cells load, decode and collide too (on the finite values
    // their sources hold) and then store what they keep instead.
    A f[Q], fo[Q];
    const bool special = (fl & (F_SOLID | F_EQ)) != 0;
    pull<Q, F, A, true>(L, src, rc, x, xm, xp, n, wave_has_walls(L, n), f);
    if constexpr (WAVE_TABLE) __builtin_amdgcn_s_waitcnt(0);   // the table's direct loads have landed
    bool bad;
    collide<Q, COLL, A, (sizeof(T) >= 4), Codec<F>::kRawExp>(L, f, fo, bad);
    count_nonfinite(L, bad && !special && active);
    T c[Q];
    out_codes<Q, F, A>(L, fl, fo, tab, c);
    const size_t plane = L.plane;
    if (active) {
#pragma unroll
        for (int i = 0; i < Q; i++) st_off(dst + ((size_t)i * plane + rc.rows[4]), x, c[i]);
    }
}

// ------------------------------------------------------------ cell-contiguous tiles
// q = a / d for a < 2^17, d <= 65535: the float quotient with the rounded
// reciprocal is within one of q (its relative error is ~2^-23, and
// a / d < 2^17), and one remainder test on each side makes it exact.
__device__ __forceinline__ uint32_t div_small(uint32_t a, uint32_t d, float inv_d) {
    uint32_t q = (uint32_t)((float)a * inv_d);
    int r = (int)a - (int)(q * d);
    if (r < 0) { q -= 1; r += (int)d; }
    if (r >= (int)d) q += 1;
    return q;
}

// One cell per lane; the workgroup's cells follow (x0, y0, z0) in index
// order, so short rows pack without idle lanes.  Lanes find their own
// (x, y, z) and neighbour rows; the rest is the row tile's step.
template <int Q, int F, class A, int COLL>
__device__ __forceinline__ void step_tile_dense(const LatDev& L, uint32_t x0, uint32_t y0, uint32_t z0,
                                                int parity, const EncEntry* tab) {
    using T = typename Codec<F>::T;
    uint32_t x = x0 + threadIdx.x;                           // < nx + 512
    const uint32_t dy = div_small(x, L.nx, L.inv_nx);
    x -= dy * L.nx;
    uint32_t y = y0 + dy;                                    // < ny + 512
    const uint32_t dz = div_small(y, L.ny, L.inv_ny);
    y -= dz * L.ny;
    const uint32_t z = z0 + dz;
    if (z >= L.nz) return;                                   // past the lattice's last cell
    RowCtx rc;
    make_rows(L, y, z, rc);
    const uint32_t n = rc.rows[4] + x;
    const uint8_t fl = ld_off(L.flags, n);
    const uint32_t xm = x == 0 ? L.nx - 1 : x - 1;
    const uint32_t xp = x + 1 == L.nx ? 0 : x + 1;
    const T* __restrict__ src = (const T*)L.f[parity];
    T* __restrict__ dst = (T*)L.f[parity ^ 1];

    A f[Q], fo[Q];
    pull<Q, F, A, true, true>(L, src, rc, x, xm, xp, n, wave_has_walls(L, n), f);   // loads with the flag's
    const bool special = (fl & (F_SOLID | F_EQ)) != 0;
    bool bad;
    collide<Q, COLL, A, (sizeof(T) >= 4), Codec<F>::kRawExp>(L, f, fo, bad);   // all lanes: fo always defined
    count_nonfinite(L, bad && !special);
    T c[Q];
    out_codes<Q, F, A>(L, fl, fo, tab, c);
    const size_t plane = L.plane;
#pragma unroll
    for (int i = 0; i < Q; i++) st_off(dst + (size_t)i * plane, n, c[i]);
}

// ------------------------------------------------------------ several cells per lane
// A lane owns CPL consecutive cells x .. x+CPL-1 of a row (x a multiple of
// CPL, nx a multiple of CPL), so each direction is one aligned vector load
// of CPL stored DDFs and each result one aligned vector store.  Directions
// with c_x = +1 need the elements x-1 .. x+CPL-2: the lane's own vector
// shifted by one element, with the missing element taken from the previous
// lane's vector (cross-lane shift); the first lane of a wavefront loads it
// directly (periodic wrap at x = 0).  c_x = -1 mirrors this with the next
// lane.  Row vectors are kept as 32-bit words.
template <class T, int CPL>
struct RowVec {
    static constexpr int W = CPL * (int)sizeof(T) / 4;   // 32-bit words
    uint32_t w[W];
};

template <class T, int CPL>
__device__ __forceinline__ RowVec<T, CPL> vload(const T* p) {
    RowVec<T, CPL> r;
    constexpr int W = RowVec<T, CPL>::W;
    if constexpr (W == 1) {
        r.w[0] = *(const LBM_GLOBAL uint32_t*)p;
    } else if constexpr (W == 2) {
        const u32x2 v = *(const LBM_GLOBAL u32x2*)p;
        r.w[0] = v.x; r.w[1] = v.y;
    } else {
        static_assert(W % 4 == 0, "row vector width");
#pragma unroll
        for (int k = 0; k < W / 4; k++) {
            const u32x4 v = ((const LBM_GLOBAL u32x4*)p)[k];
            r.w[4 * k] = v.x; r.w[4 * k + 1] = v.y; r.w[4 * k + 2] = v.z; r.w[4 * k + 3] = v.w;
        }
    }
    return r;
}

template <class T, int CPL>
__device__ __forceinline__ void vstore(T* p, const RowVec<T, CPL>& r) {
    constexpr int W = RowVec<T, CPL>::W;
    if constexpr (W == 1) {
        *(LBM_GLOBAL uint32_t*)p = r.w[0];
    } else if constexpr (W == 2) {
        *(LBM_GLOBAL u32x2*)p = u32x2{r.w[0], r.w[1]};
    } else {
#pragma unroll
        for (int k = 0; k < W / 4; k++)
            ((LBM_GLOBAL u32x4*)p)[k] = u32x4{r.w[4 * k], r.w[4 * k + 1], r.w[4 * k + 2], r.w[4 * k + 3]};
    }
}

template <class T>
__device__ __forceinline__ T from_bits64(uint64_t b) {
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, b);
    else if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, (uint32_t)b);
    else return (T)b;
}
template <class T>
__device__ __forceinline__ uint64_t to_bits64(T v) {
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(uint64_t, v);
    else if constexpr (sizeof(T) == 4) return __builtin_bit_cast(uint32_t, v);
    else return (uint16_t)v;
}

template <class T, int CPL>
__device__ __forceinline__ T velem(const RowVec<T, CPL>& r, int k) {
    if constexpr (sizeof(T) == 2) return (T)(r.w[k >> 1] >> (16 * (k & 1)));
    else if constexpr (sizeof(T) == 4) return from_bits64<T>(r.w[k]);
    else return from_bits64<T>((uint64_t)r.w[2 * k] | ((uint64_t)r.w[2 * k + 1] << 32));
}

template <class T, int CPL>
__device__ __forceinline__ void vset(RowVec<T, CPL>& r, int k, T v) {
    const uint64_t b = to_bits64<T>(v);
    if constexpr (sizeof(T) == 2) {
        if (k & 1) r.w[k >> 1] = (r.w[k >> 1] & 0xFFFFu) | ((uint32_t)b << 16);
        else r.w[k >> 1] = (uint32_t)b;    // even element is set first
    } else if constexpr (sizeof(T) == 4) {
        r.w[k] = (uint32_t)b;
    } else {
        r.w[2 * k] = (uint32_t)b;
        r.w[2 * k + 1] = (uint32_t)(b >> 32);
    }
}

// Replaces element k, keeping the others (vset may clear the odd neighbour
// of an even 16-bit element).
template <class T, int CPL>
__device__ __forceinline__ void vreplace(RowVec<T, CPL>& r, int k, T v) {
    if constexpr (sizeof(T) == 2) {
        const uint32_t b = (uint32_t)(uint16_t)v;
        if (k & 1) r.w[k >> 1] = (r.w[k >> 1] & 0xFFFFu) | (b << 16);
        else r.w[k >> 1] = (r.w[k >> 1] & 0xFFFF0000u) | b;
    } else {
        vset<T, CPL>(r, k, v);
    }
}

// Elements (prev, in[0], ..., in[CPL-2]): `prev` is the element before the
// vector, `in` shifted up by one element.
template <class T, int CPL>
__device__ __forceinline__ RowVec<T, CPL> shift_up(const RowVec<T, CPL>& in, T prev) {
    RowVec<T, CPL> o;
    constexpr int W = RowVec<T, CPL>::W;
    if constexpr (sizeof(T) == 2) {
        o.w[0] = __builtin_amdgcn_alignbit(in.w[0], (uint32_t)(uint16_t)prev << 16, 16);
#pragma unroll
        for (int j = 1; j < W; j++) o.w[j] = __builtin_amdgcn_alignbit(in.w[j], in.w[j - 1], 16);
    } else {
        constexpr int E = (int)sizeof(T) / 4;              // words per element
        const uint64_t b = to_bits64<T>(prev);
        o.w[0] = (uint32_t)b;
        if constexpr (E == 2) o.w[1] = (uint32_t)(b >> 32);
#pragma unroll
        for (int j = E; j < W; j++) o.w[j] = in.w[j - E];
    }
    return o;
}

// Elements (in[1], ..., in[CPL-1], next).
template <class T, int CPL>
__device__ __forceinline__ RowVec<T, CPL> shift_down(const RowVec<T, CPL>& in, T next) {
    RowVec<T, CPL> o;
    constexpr int W = RowVec<T, CPL>::W;
    if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int j = 0; j < W - 1; j++) o.w[j] = __builtin_amdgcn_alignbit(in.w[j + 1], in.w[j], 16);
        o.w[W - 1] = __builtin_amdgcn_alignbit((uint32_t)(uint16_t)next, in.w[W - 1], 16);
    } else {
        constexpr int E = (int)sizeof(T) / 4;
#pragma unroll
        for (int j = 0; j < W - E; j++) o.w[j] = in.w[j + E];
        const uint64_t b = to_bits64<T>(next);
        o.w[W - E] = (uint32_t)b;
        if constexpr (E == 2) o.w[W - 1] = (uint32_t)(b >> 32);
    }
    return o;
}

template <class T>
__device__ __forceinline__ T shfl_elem_up(T v) {
    const uint64_t b = to_bits64<T>(v);
    uint64_t r = (uint32_t)__shfl_up((int)(uint32_t)b, 1u, 64);
    if constexpr (sizeof(T) == 8) r |= (uint64_t)(uint32_t)__shfl_up((int)(uint32_t)(b >> 32), 1u, 64) << 32;
    return from_bits64<T>(r);
}
template <class T>
__device__ __forceinline__ T shfl_elem_down(T v) {
    const uint64_t b = to_bits64<T>(v);
    uint64_t r = (uint32_t)__shfl_down((int)(uint32_t)b, 1u, 64);
    if constexpr (sizeof(T) == 8) r |= (uint64_t)(uint32_t)__shfl_down((int)(uint32_t)(b >> 32), 1u, 64) << 32;
    return from_bits64<T>(r);
}

template <int CPL>
__device__ __forceinline__ uint32_t load_flags(const uint8_t* p) {
    if constexpr (CPL == 1) return *(const LBM_GLOBAL uint8_t*)p;
    else if constexpr (CPL == 2) return *(const LBM_GLOBAL uint16_t*)p;
    else return *(const LBM_GLOBAL uint32_t*)p;
}

template <int Q, int F, class A, int COLL, int CPL>
__device__ __forceinline__ void step_tile_v(const LatDev& L, uint32_t x0, uint32_t y, uint32_t z,
                                            int parity, const EncEntry* tab) {
    using T = typename Codec<F>::T;
    using RV = RowVec<T, CPL>;
    const uint32_t nx = L.nx;
    const uint32_t x = x0 + threadIdx.x * CPL;
    if (x >= nx) return;
    RowCtx rc;
    make_rows(L, y, z, rc);
    const uint32_t row = rc.rows[4];
    const uint32_t fl4 = load_flags<CPL>(L.flags + row + x);
    bool near[CPL], special[CPL];
    bool any_special = false;
#pragma unroll
    for (int k = 0; k < CPL; k++) {
        const uint32_t fk = (fl4 >> (8 * k)) & 0xFF;
        near[k] = (fk & F_NEAR) != 0;
        special[k] = (fk & (F_SOLID | F_EQ)) != 0;
        any_special |= special[k];
    }
    const T* __restrict__ src = (const T*)L.f[parity];
    T* __restrict__ dst = (T*)L.f[parity ^ 1];
    const size_t plane = L.plane;
    // The elements just outside this wavefront's span of the row: before its
    // first lane and after its last active lane (periodic wrap).  Both indices
    // are wavefront-uniform, so every lane loads the same address (no
    // divergent branch) and only the edge lane keeps the value.
    const uint32_t xw0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
    const uint32_t xw_end = min(xw0 + 64u * CPL, nx);
    const uint32_t xm = xw0 == 0 ? nx - 1 : xw0 - 1;
    const uint32_t xn = xw_end == nx ? 0 : xw_end;
    const bool first_lane = x == xw0;
    const bool last_lane = x + CPL == xw_end;

    RV raw[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const T* p = src + ((size_t)i * plane + src_row<Q>(rc, i));
        const RV v = vload<T, CPL>(p + x);
        if (VelSet<Q>::c[i][0] > 0) {
            const T edge = ld_off(p, xm);
            const T prev = shfl_elem_up<T>(velem<T, CPL>(v, CPL - 1));
            raw[i] = shift_up<T, CPL>(v, first_lane ? edge : prev);
        } else if (VelSet<Q>::c[i][0] < 0) {
            const T edge = ld_off(p, xn);
            const T next = shfl_elem_down<T>(velem<T, CPL>(v, 0));
            raw[i] = shift_down<T, CPL>(v, last_lane ? edge : next);
        } else {
            raw[i] = v;
        }
    }

    RV out[Q];
#pragma unroll
    for (int k = 0; k < CPL; k++) {
        A f[Q], fo[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) f[i] = load_ddf<Q, F, A, true>(velem<T, CPL>(raw[i], k));
        if (__any(near[k])) {
            const uint32_t xk = x + k;
            const uint32_t xkm = xk == 0 ? nx - 1 : xk - 1;
            const uint32_t xkp = xk + 1 == nx ? 0 : xk + 1;
            const uint32_t m = near[k] ? ld_mask(L.wall_mask, row + xk) : 0u;
#pragma unroll
            for (int i = 1; i < Q; i++) {
                if (m & (1u << i)) {
                    A v = load_ddf<Q, F, A, true>(ld_off(src + (size_t)opp(i) * plane, row + xk));
                    if (m & 0x80000000u) {
                        const uint8_t fs = ld_off(L.flags, src_row<Q>(rc, i) + src_x<Q>(i, xk, xkm, xkp));
                        if (fs & F_MOVING) {
                            const A cu = (A)(VelSet<Q>::c[i][0] * L.wall_u[0] + VelSet<Q>::c[i][1] * L.wall_u[1] +
                                             VelSet<Q>::c[i][2] * L.wall_u[2]);
                            v += (A)(6.0 * VelSet<Q>::w(i) * kRawScale<F, true>) * cu;
                        }
                    }
                    f[i] = v;
                }
            }
        }
        bool bad;
        collide<Q, COLL, A, (sizeof(T) >= 4), Codec<F>::kRawExp>(L, f, fo, bad);
        count_nonfinite(L, bad && !special[k]);
#pragma unroll
        for (int i = 0; i < Q; i++) vset<T, CPL>(out[i], k, Codec<F>::template store_raw<A>(fo[i], tab));
    }
    if (__any(any_special)) {
        // wall and equilibrium cells write back what they keep (whole rows)
        bool any_eq_cell = false;
#pragma unroll
        for (int k = 0; k < CPL; k++) any_eq_cell |= ((fl4 >> (8 * k)) & F_EQ) != 0;
        T eq[Q];
        eq_codes_if<Q, F>(L, __any(any_eq_cell), eq);
#pragma unroll
        for (int k = 0; k < CPL; k++) {
            const uint32_t fk = (fl4 >> (8 * k)) & 0xFF;
#pragma unroll
            for (int i = 0; i < Q; i++)
                if (special[k]) vreplace<T, CPL>(out[i], k, (fk & F_EQ) ? eq[i] : (T)0);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; i++) vstore<T, CPL>(dst + ((size_t)i * plane + row + x), out[i]);
}

// One wavefront's copy of the encoder table, from global memory to LDS by
// direct loads (16 bytes per lane, no registers; one instruction per 64
// entries); the wavefront waits for them (vmcnt) before reading the table.
static_assert(sizeof(EncEntry) == 16, "one 16-byte direct load per table entry");
static_assert(kEncEntries % 64 == 0, "whole wavefront loads");
__device__ __forceinline__ void fetch_wave_table(const EncEntry* g, EncEntry (&s)[kEncEntries]) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (uint32_t k = 0; k < (uint32_t)kEncEntries; k += 64u)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(g + k + lane),
                                         (__attribute__((address_space(3))) void*)(&s[k]), 16, 0, 0);
}

template <int F>
__device__ __forceinline__ const EncEntry* stage_table(const EncEntry* g, EncEntry* s) {
    if constexpr (Codec<F>::kTable) {
        for (int k = threadIdx.x; k < kEncEntries; k += blockDim.x) s[k] = g[k];
        __syncthreads();
        return s;
    } else {
        return nullptr;
    }
}

template <int Q, int F, class A, int COLL, int CPL>
__device__ __forceinline__ void run_tile(const LatDev& L, uint32_t x0, uint32_t y, uint32_t z, int parity,
                                         const EncEntry* tab) {
    if constexpr (CPL == 1) step_tile<Q, F, A, COLL>(L, x0, y, z, parity, tab);
    else step_tile_v<Q, F, A, COLL, CPL>(L, x0, y, z, parity, tab);
}

template <int Q, int F, class A, int COLL, int CPL>
__global__ void __launch_bounds__(512) k_step_single(LatDev L, int parity, uint32_t segs,
                                                     const EncEntry* __restrict__ enc) {
    // grid (ny, segments, nz): no index division, and the segments of one row
    // are ny workgroups apart, which for ny a multiple of 8 puts them on the
    // same XCD (workgroups go round-robin to the 8 XCDs), so the cache lines
    // their +-x neighbours share are fetched into one L2 only
    if constexpr (Codec<F>::kTable && CPL == 1) {
        // every wavefront fetches its own copy of the (2 KB) table, which
        // arrives while its DDF loads are in flight: no workgroup barrier.
        // The copies are dynamic LDS, 2 KB per wavefront of the launch.
        extern __shared__ __attribute__((aligned(16))) EncEntry s_wave_tabs[];
        EncEntry(&mine)[kEncEntries] = reinterpret_cast<EncEntry(*)[kEncEntries]>(s_wave_tabs)[threadIdx.x >> 6];
        fetch_wave_table(enc, mine);
        step_tile<Q, F, A, COLL, true>(L, blockIdx.y * blockDim.x, blockIdx.x, blockIdx.z, parity, mine);
    } else {
        __shared__ EncEntry s_tab[Codec<F>::kTable ? kEncEntries : 1];
        const EncEntry* tab = stage_table<F>(enc, s_tab);
        run_tile<Q, F, A, COLL, CPL>(L, blockIdx.y * blockDim.x * CPL, blockIdx.x, blockIdx.z, parity, tab);
    }
}

// Ensemble: workgroups walk the tile table (one tile each, or a persistent
// grid-stride walk when the grid is smaller than the table).
template <int Q, int F, class A, int COLL, int CPL>
__global__ void __launch_bounds__(512) k_step_batched(const LatDev* __restrict__ lats,
                                                      const Tile* __restrict__ tiles, uint32_t ntiles,
                                                      int parity, const EncEntry* __restrict__ enc) {
    __shared__ EncEntry s_tab[Codec<F>::kTable ? kEncEntries : 1];
    const EncEntry* tab = stage_table<F>(enc, s_tab);
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        run_tile<Q, F, A, COLL, CPL>(lats[tl.lat], tl.x0, tl.y, tl.z, parity, tab);
    }
}

template <int Q, int F, class A, int COLL>
__global__ void __launch_bounds__(512) k_step_dense(const LatDev* __restrict__ lats,
                                                    const Tile* __restrict__ tiles, uint32_t ntiles,
                                                    int parity, const EncEntry* __restrict__ enc) {
    __shared__ EncEntry s_tab[Codec<F>::kTable ? kEncEntries : 1];
    const EncEntry* tab = stage_table<F>(enc, s_tab);
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        step_tile_dense<Q, F, A, COLL>(lats[tl.lat], tl.x0, tl.y, tl.z, parity, tab);
    }
}

// ------------------------------------------------------------ initialisation
// Stored code of direction i of the (shifted) equilibrium of rho, u.
template <int Q, int F, class A>
__device__ __forceinline__ typename Codec<F>::T eq_code(int i, A rho, A ux, A uy, A uz, A shift,
                                                       const EncEntry* tab) {
    const A C = (A)(-3) * (ux * ux + uy * uy + uz * uz);
    const A rhom1 = rho - shift;
    const A wi = (A)VelSet<Q>::w(i);
    const A B = (A)3 * cdot_i<Q, A>(i, ux, uy, uz);
    return Codec<F>::template store<A>(fmaa(wi * rho, fmaa((A)0.5, fmaa(B, B, C), B), wi * rhom1), tab);
}

// The q codes of the lattice's EQ cells (eq_rho, eq_u), computed once; the
// initialisation and the step write EQ cells from this table, so both agree
// bit for bit.
template <int Q, int F, class A>
__global__ void __launch_bounds__(64) k_eq_codes(LatDev L, typename Codec<F>::T* __restrict__ out,
                                                 const EncEntry* __restrict__ enc) {
    __shared__ EncEntry s_tab[Codec<F>::kTable ? kEncEntries : 1];
    const EncEntry* tab = stage_table<F>(enc, s_tab);
    const int i = threadIdx.x;
    if (i < Q) out[i] = eq_code<Q, F, A>(i, (A)L.eq_rho, (A)L.eq_u[0], (A)L.eq_u[1], (A)L.eq_u[2], (A)L.shift, tab);
}

// DDFs of the (shifted) equilibrium of rho, u (the paper's initialize kernel)
// written to both buffers; wall cells get zeros, EQ cells the lattice's
// equilibrium codes.
template <int Q, int F, class A>
__global__ void __launch_bounds__(256) k_init(LatDev L, const double* __restrict__ rho_in,
                                              const double* __restrict__ u_in,
                                              const EncEntry* __restrict__ enc) {
    using T = typename Codec<F>::T;
    __shared__ EncEntry s_tab[Codec<F>::kTable ? kEncEntries : 1];
    const EncEntry* tab = stage_table<F>(enc, s_tab);
    const size_t N = (size_t)L.nx * L.ny * L.nz;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint8_t fl = L.flags[n];
    A rho = (A)1, ux = (A)0, uy = (A)0, uz = (A)0;
    if (rho_in) rho = (A)rho_in[n];
    if (u_in) { ux = (A)u_in[n]; uy = (A)u_in[N + n]; uz = (A)u_in[2 * N + n]; }
    const T* eqc = (const T*)L.eq_codes;
    T* d0 = (T*)L.f[0];
    T* d1 = (T*)L.f[1];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        T code = eq_code<Q, F, A>(i, rho, ux, uy, uz, (A)L.shift, tab);
        if (fl & F_EQ) code = eqc[i];
        if (fl & F_SOLID) code = Codec<F>::template store<A>((A)0, tab);
        d0[(size_t)i * L.plane + n] = code;
        d1[(size_t)i * L.plane + n] = code;
    }
}

// ------------------------------------------------------------ per-cell moments
// rho, u the next step sees (velocity with F/2, not clamped); walls: rho 1 and
// wall velocity; EQ cells: moments of their own DDFs.
template <int Q, int F, class A>
__device__ __forceinline__ void cell_moments(const LatDev& L, int parity, uint32_t n, uint32_t& fl_out,
                                             A& rho, A (&u)[3], A (&f)[Q]) {
    using T = typename Codec<F>::T;
    const T* __restrict__ src = (const T*)L.f[parity];
    const uint32_t x = n % L.nx, yz = n / L.nx, y = yz % L.ny, z = yz / L.ny;
    const uint8_t fl = L.flags[n];
    fl_out = fl;
    if (fl & F_SOLID) {
        rho = (A)1;
        const bool mv = fl & F_MOVING;
        for (int a = 0; a < 3; a++) u[a] = mv ? (A)L.wall_u[a] : (A)0;
        return;
    }
    A j[3];
    if (fl & F_EQ) {
#pragma unroll
        for (int i = 0; i < Q; i++) f[i] = Codec<F>::template load<A>(src[(size_t)i * L.plane + n]);
        fields<Q, A>(f, (A)L.shift, rho, j);
    } else {
        RowCtx rc;
        make_rows(L, y, z, rc);
        const uint32_t xm = x == 0 ? L.nx - 1 : x - 1;
        const uint32_t xp = x + 1 == L.nx ? 0 : x + 1;
        pull<Q, F, A, false>(L, src, rc, x, xm, xp, n, __any((fl & F_NEAR) != 0), f);
        fields<Q, A>(f, (A)L.shift, rho, j);
        if (L.forced) {
            for (int a = 0; a < 3; a++) j[a] += (A)0.5 * (A)L.force[a];
        }
    }
    for (int a = 0; a < 3; a++) u[a] = j[a] / rho;
}

template <int Q, int F, class A>
__global__ void __launch_bounds__(256) k_moments(LatDev L, int parity, double* __restrict__ rho_out,
                                                 double* __restrict__ u_out) {
    const size_t N = (size_t)L.nx * L.ny * L.nz;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    uint32_t fl;
    A rho, u[3], f[Q];
    cell_moments<Q, F, A>(L, parity, (uint32_t)n, fl, rho, u, f);
    if (rho_out) rho_out[n] = (double)rho;
    if (u_out) {
        u_out[n] = (double)u[0];
        u_out[N + n] = (double)u[1];
        u_out[2 * N + n] = (double)u[2];
    }
}

// ------------------------------------------------------------ FP64 diagnostics
// Sum (or max) of a double over each row of 16 lanes with DPP moves (no LDS):
// xor 1 and xor 2 inside quads, then the mirrored half rows and rows; every
// lane of a row ends with the row's result, combined in a fixed order.
// dpp_f64: a permutation inside each row (every lane is written, from a lane
// that exists), so the destination needs no initial value.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64_rows(double v) {      // rows outside ROWS read 0
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF, false);
    return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}
// Sum (or max, of non-negative values) of a double over the wavefront, in a
// fixed order: rows of 16 lanes first (xor 1, xor 2, mirrored half rows,
// mirrored rows), then lane 15 of rows 0 and 2 into rows 1 and 3, then lane
// 31 into rows 2 and 3; lane 63 ends with the result.
template <bool MAX>
__device__ __forceinline__ double wave_reduce(double v) {
    constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140, kBcast15 = 0x142,
                  kBcast31 = 0x143;
    v = MAX ? fmax(v, dpp_f64<kXor1>(v)) : v + dpp_f64<kXor1>(v);
    v = MAX ? fmax(v, dpp_f64<kXor2>(v)) : v + dpp_f64<kXor2>(v);
    v = MAX ? fmax(v, dpp_f64<kHalfMirror>(v)) : v + dpp_f64<kHalfMirror>(v);
    v = MAX ? fmax(v, dpp_f64<kMirror>(v)) : v + dpp_f64<kMirror>(v);
    v = MAX ? fmax(v, dpp_f64_rows<kBcast15, 0xA>(v)) : v + dpp_f64_rows<kBcast15, 0xA>(v);
    v = MAX ? fmax(v, dpp_f64_rows<kBcast31, 0xC>(v)) : v + dpp_f64_rows<kBcast31, 0xC>(v);
    return v;
}

// Pairwise sums across the wavefront's halves (lanes i and i + 32) of two
// fields at once: lanes 0-31 get a's, lanes 32-63 b's (one v_permlane32_swap
// per 32-bit half of the doubles, one add).
__device__ __forceinline__ double comb32(double a, double b) {
    const uint64_t ab = __builtin_bit_cast(uint64_t, a), bb = __builtin_bit_cast(uint64_t, b);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)ab, (uint32_t)bb, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(ab >> 32), (uint32_t)(bb >> 32), false, false);
    const double a2 = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
    const double b2 = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
    return a2 + b2;
}
// The same across neighbouring rows of 16 lanes: rows 0 and 2 keep a's sums
// of rows (0,1) and (2,3), rows 1 and 3 get b's.
__device__ __forceinline__ double comb16(double a, double b) {
    const uint64_t ab = __builtin_bit_cast(uint64_t, a), bb = __builtin_bit_cast(uint64_t, b);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)ab, (uint32_t)bb, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(ab >> 32), (uint32_t)(bb >> 32), false, false);
    const double a2 = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
    const double b2 = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
    return a2 + b2;
}
// Four fields summed over the wavefront, one per row of 16 lanes: row 0
// f0, row 1 f2, row 2 f1, row 3 f3 (every lane of a row holds its total).
__device__ __forceinline__ double reduce4(double f0, double f1, double f2, double f3) {
    constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;
    double v = comb16(comb32(f0, f1), comb32(f2, f3));
    v += dpp_f64<kXor1>(v);
    v += dpp_f64<kXor2>(v);
    v += dpp_f64<kHalfMirror>(v);
    v += dpp_f64<kMirror>(v);
    return v;
}

// Block-wide reduction of kDiagFields values (the last one by max, of
// non-negative values) in a fixed order, without a barrier at the end: each
// wavefront reduces its values -- the sums four fields at a time, one field
// per row of 16 lanes after two cross-lane swaps (reduce4), the max with DPP
// -- and puts them in its LDS slots (the wall force only in wavefronts next
// to a wall, bit 7 of the wavefront-uniform `skip`; 0 otherwise), then counts
// itself in; the wavefront that counts last sums the slots in wavefront
// order and writes out[k].  The others leave as soon as they have counted,
// instead of waiting for the slowest.  `count` must be zero at entry for the
// whole workgroup (set before a barrier at the start of the kernel).
// Slots: reduce4 leaves its fields in the rows in the order f0, f2, f1, f3,
// so each group is passed in the order that puts field g_r in row r, and row
// r of group g writes slot 4 g + r: fields 0-3, then 4, 5, 6, 10, then 7, 8,
// 9, and the max in slot 11.  Which argument a field is passed as does not
// change its sum: every field goes through the same tree of additions.
__device__ __forceinline__ void block_reduce_store(double (&acc)[kDiagFields], uint32_t skip, double* out,
                                                   uint32_t* count) {
    constexpr int kMaxWaves = 1024 / 64;
    __shared__ double s[kDiagFields][kMaxWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = (blockDim.x + 63) >> 6;
    const int row = lane >> 4;
    const bool last_of_row = (lane & 15) == 15;
    const double g1 = reduce4(acc[0], acc[2], acc[1], acc[3]);
    const double g2 = reduce4(acc[4], acc[6], acc[5], acc[10]);
    if (last_of_row) {
        s[row][wave] = g1;
        s[4 + row][wave] = g2;
    }
    double g3 = 0.0;
    if (!((skip >> 7) & 1u)) g3 = reduce4(acc[7], acc[9], acc[8], 0.0);
    if (last_of_row && row != 3) s[8 + row][wave] = g3;
    const double mx = wave_reduce<true>(acc[kDiagFields - 1]);
    if (lane == 63) s[kDiagFields - 1][wave] = mx;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    uint32_t before = 0;
    if (lane == 0) before = __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    before = (uint32_t)__builtin_amdgcn_readfirstlane((int)before);
    if (before == (uint32_t)nwaves - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (lane < kDiagFields) {
            double v = s[lane][0];
            for (int w = 1; w < nwaves; w++) v = (lane == kDiagFields - 1) ? fmax(v, s[lane][w]) : v + s[lane][w];
            const int field = lane == 7 ? 10 : (lane >= 8 && lane <= 10 ? lane - 1 : lane);
            out[field] = v;
        }
    }
}

// The FP64 contributions of one fluid cell (flags fl) whose pulled DDFs are
// f, added to v: mass, momentum, kinetic energy, the error norms against
// u_ref, the non-finite count and the largest |u|^2 (the momentum exchange
// into walls is diag_exchange's, taken from f before the moving walls' term).  The moments are those the next step sees after streaming
// (velocity with F/2, not clamped), in the step's arithmetic.  RAWE: f in
// units of 2^-RAWE (the step's raw units); the sums are taken in those units
// and scaled back, a power of two, so rho and j are bit-identical to sums of
// the unscaled values.
template <int Q, int F, class A, int RAWE = 0>
__device__ __forceinline__ void diag_cell(const LatDev& L, uint32_t fl, uint32_t n, const A (&f)[Q],
                                          const double* __restrict__ u_ref, double (&v)[kDiagFields]) {
    if (fl & (F_SOLID | F_EQ)) return;
    A rho, j[3];
    fields<Q, A>(f, (A)(L.shift * exp2i(RAWE)), rho, j);
    if constexpr (RAWE != 0) {
        constexpr A kUnraw = (A)(1.0 / exp2i(RAWE));
        rho *= kUnraw;
#pragma unroll
        for (int a = 0; a < 3; a++) j[a] *= kUnraw;
    }
    if (L.forced) {
#pragma unroll
        for (int a = 0; a < 3; a++) j[a] += (A)0.5 * (A)L.force[a];
    }
    const A inv = (A)1 / rho;                                    // one division, three products
    const double r = (double)rho, ux = (double)(j[0] * inv), uy = (double)(j[1] * inv), uz = (double)(j[2] * inv);
    if (!(isfinite(r) && isfinite(ux) && isfinite(uy) && isfinite(uz))) {
        v[10] += 1.0;
        v[7] = v[8] = v[9] = 0.0;                                // no wall force from such a cell
        return;
    }
    v[0] += r;
    v[1] += r * ux;
    v[2] += r * uy;
    v[3] += r * uz;
    const double u2 = ux * ux + uy * uy + uz * uz;
    v[4] += 0.5 * r * u2;
    v[11] = fmax(v[11], u2);
    if (u_ref) {
        const size_t N = (size_t)L.nx * L.ny * L.nz;
        const double rx = u_ref[n], ry = u_ref[N + n], rz = u_ref[2 * N + n];
        v[5] += (ux - rx) * (ux - rx) + (uy - ry) * (uy - ry) + (uz - rz) * (uz - rz);
        v[6] += rx * rx + ry * ry + rz * rz;
    }
}

// The momentum exchange of one fluid cell next to a wall (wall mask m) into
// v[7..9], which hold 0 for this cell on entry: every link to a wall source
// x - c_i carries c_opp (2 (f*_opp + w_opp) + 6 w_i c_i.u_w) into the wall,
// f*_opp being what this cell sent towards the wall in the last step, which
// the pull took for direction i (this cell's own opposite DDF): f[i] before
// the moving walls' term, in units of 2^-RAWE (scaled back exactly), so no
// load waits here.  A branch per direction, skipped by wavefronts in which
// no lane has that wall source; only a moving wall source needs a load (its
// flag).  diag_cell clears v[7..9] again for a cell whose moments are not
// finite.
template <int Q, int F, class A, int RAWE = 0>
__device__ __forceinline__ void diag_exchange(const LatDev& L, uint32_t x, uint32_t y, uint32_t z, uint32_t m,
                                              const A (&f)[Q], double (&v)[kDiagFields]) {
    constexpr A kUnraw = (A)(1.0 / exp2i(RAWE));
    const uint32_t xm = x == 0 ? L.nx - 1 : x - 1;
    const uint32_t xp = x + 1 == L.nx ? 0 : x + 1;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        if ((m >> i) & 1u) {
            const int o = opp(i);
            const int cx = VelSet<Q>::c[i][0], cy = VelSet<Q>::c[i][1], cz = VelSet<Q>::c[i][2];
            const double fo = (double)(f[i] * kUnraw) + VelSet<Q>::w(o) * L.shift;
            double mv = 0.0;
            if (m & 0x80000000u) {
                const uint32_t sx = cx > 0 ? xm : (cx < 0 ? xp : x);
                const uint32_t sy = wrap_add(y, -cy, L.ny), sz = wrap_add(z, -cz, L.nz);
                const uint8_t fs = ld_off(L.flags, sx + (sy + sz * L.ny) * L.nx);
                if (fs & F_MOVING) mv = 6.0 * VelSet<Q>::w(i) * (cx * L.wall_u[0] + cy * L.wall_u[1] + cz * L.wall_u[2]);
            }
            const double t = 2.0 * fo + mv;                             // c_opp = -c_i
            // a component 0 adds nothing: the sums start at +0, and t is
            // finite unless the DDF is (then so are the moments, and diag_cell
            // clears the force) or above 2^1022 in magnitude (FP64 storage
            // only, far outside any flow)
            if (cx) v[7] -= cx * t;
            if (cy) v[8] -= cy * t;
            if (cz) v[9] -= cz * t;
        }
    }
}

// First pass: the step's decomposition, one workgroup per row tile of
// kDiagThreads cells (grid (ny, segs, nz): the row's y and z are the block
// indices, neighbour rows and wrap workgroup-uniform, the wall mask read only
// by wavefronts next to a wall), one cell per lane.  The workgroup's FP64
// sums, in a fixed order, go to partials[tile] (tile = (z ny + y) segs +
// segment), which the fixed-order passes of k_diag_reduce sum, so repeated
// calls give identical results.  The largest |u|^2 is reduced by max; its
// square root is taken once, at the end.  Nothing is carried from one cell to
// the next and the workgroup's wavefronts leave without waiting for each
// other, which keeps the kernel's occupancy and its wavefronts' lifetimes
// close to the step's.  (Two rows per workgroup, with both cells' loads in
// flight, was slower: the extra registers cost more wavefronts than the
// second cell gained.)
template <int Q, int F, class A>
__global__ void __launch_bounds__(kDiagThreads) k_diag(LatDev L, int parity, const double* __restrict__ u_ref,
                                                       double* __restrict__ partials, uint32_t segs) {
    using T = typename Codec<F>::T;
    __shared__ uint32_t waves_done;
    if (threadIdx.x == 0) waves_done = 0;
    __syncthreads();
    const uint32_t y = blockIdx.x, seg = blockIdx.y, z = blockIdx.z;
    const uint32_t x = seg * kDiagThreads + threadIdx.x;
    double v[kDiagFields];
#pragma unroll
    for (int k = 0; k < kDiagFields; k++) v[k] = 0.0;
    if (x < L.nx) {
        const T* __restrict__ src = (const T*)L.f[parity];
        RowCtx rc;
        make_rows(L, y, z, rc);
        const uint32_t n = rc.rows[4] + x;
        const uint8_t fl = ld_off(L.flags, n);
        const uint32_t xm = x == 0 ? L.nx - 1 : x - 1;
        const uint32_t xp = x + 1 == L.nx ? 0 : x + 1;
        T c[Q];
        uint32_t m;
        A f[Q];
        pull_codes<Q, F>(L, src, rc, x, xm, xp, n, wave_has_walls(L, n), c, m);
        decode_pulled<Q, F, A, true>(c, f);                                  // the step's raw units
        if ((fl & (F_SOLID | F_EQ | F_NEAR)) == F_NEAR) diag_exchange<Q, F, A, Codec<F>::kRawExp>(L, x, y, z, m, f, v);
        add_moving_walls<Q, F, A, true>(L, rc, x, xm, xp, m, f);
        diag_cell<Q, F, A, Codec<F>::kRawExp>(L, fl, n, f, u_ref, v);
    }
    // the wall force is reduced only by wavefronts next to a wall
    const uint32_t skip = __any(v[7] != 0.0 || v[8] != 0.0 || v[9] != 0.0) ? 0u : (1u << 7);
    block_reduce_store(v, skip, partials + ((size_t)(z * L.ny + y) * segs + seg) * kDiagFields, &waves_done);
}

// One time step fused with the diagnostics of the state it reads: the row
// tiles of k_diag (kDiagThreads cells of one row per workgroup, grid (ny,
// segs, nz)), each lane pulling its cell once for both.  The pulled DDFs,
// scaled from the step's raw units (a power of two, exact), give diag_cell
// exactly the sums k_diag's own pull gives, and the workgroup reduces them
// in k_diag's order into the same partial slot, so the diagnostics are
// bit-identical to k_diag on the same state; the DDFs written are the
// step's.  Lanes past the row's end step the row's last cell, store nothing
// and add nothing (every lane takes part in the cross-lane reduction).
template <int Q, int F, class A, int COLL>
__global__ void __launch_bounds__(kDiagThreads) k_step_diag(LatDev L, int parity, uint32_t segs,
                                                            const EncEntry* __restrict__ enc,
                                                            const double* __restrict__ u_ref,
                                                            double* __restrict__ partials) {
    using T = typename Codec<F>::T;
    __shared__ uint32_t waves_done;
    __shared__ EncEntry s_tab[Codec<F>::kTable ? kEncEntries : 1];
    if (threadIdx.x == 0) waves_done = 0;
    const EncEntry* tab = nullptr;
    if constexpr (Codec<F>::kTable) tab = stage_table<F>(enc, s_tab);     // its barrier also publishes waves_done
    else __syncthreads();
    const uint32_t y = blockIdx.x, seg = blockIdx.y, z = blockIdx.z;
    const bool active = seg * kDiagThreads + threadIdx.x < L.nx;
    const uint32_t x = active ? seg * kDiagThreads + threadIdx.x : L.nx - 1;
    RowCtx rc;
    make_rows(L, y, z, rc);
    const uint32_t n = rc.rows[4] + x;
    const uint8_t fl = ld_off(L.flags, n);
    const uint32_t xm = x == 0 ? L.nx - 1 : x - 1;
    const uint32_t xp = x + 1 == L.nx ? 0 : x + 1;
    const T* __restrict__ src = (const T*)L.f[parity];
    T* __restrict__ dst = (T*)L.f[parity ^ 1];

    A f[Q], fo[Q];
    const bool special = (fl & (F_SOLID | F_EQ)) != 0;
    {
        // the diagnostics first, so that their registers are free for the collision
        double v[kDiagFields];
#pragma unroll
        for (int k = 0; k < kDiagFields; k++) v[k] = 0.0;
        T cin[Q];
        uint32_t m;
        pull_codes<Q, F>(L, src, rc, x, xm, xp, n, wave_has_walls(L, n), cin, m);
        decode_pulled<Q, F, A, true>(cin, f);
        if (active && (fl & (F_SOLID | F_EQ | F_NEAR)) == F_NEAR)
            diag_exchange<Q, F, A, Codec<F>::kRawExp>(L, x, y, z, m, f, v);
        add_moving_walls<Q, F, A, true>(L, rc, x, xm, xp, m, f);
        if (active) diag_cell<Q, F, A, Codec<F>::kRawExp>(L, fl, n, f, u_ref, v);
        const uint32_t skip = __any(v[7] != 0.0 || v[8] != 0.0 || v[9] != 0.0) ? 0u : (1u << 7);
        block_reduce_store(v, skip, partials + ((size_t)(z * L.ny + y) * segs + seg) * kDiagFields, &waves_done);
    }
    bool bad;
    collide<Q, COLL, A, (sizeof(T) >= 4), Codec<F>::kRawExp>(L, f, fo, bad);
    count_nonfinite(L, bad && !special && active);
    T c[Q];
    out_codes<Q, F, A>(L, fl, fo, tab, c);
    const size_t plane = L.plane;
    if (active) {
#pragma unroll
        for (int i = 0; i < Q; i++) st_off(dst + ((size_t)i * plane + rc.rows[4]), x, c[i]);
    }
}

// ------------------------------------------------------------ host launchers
// Instantiated once per storage format in kern_<format>.hip.
template <int F>
struct FormatLaunchers {
    // cells per lane built: up to 4 for 16-bit DDFs, 2 for FP32, 1 for FP64
    // (two FP64 cells per lane exceed the register file for D3Q27)
    static constexpr int kMaxCpl = sizeof(typename Codec<F>::T) == 2 ? 4 : (sizeof(typename Codec<F>::T) == 4 ? 2 : 1);

    template <int Q, class A, int COLL, int CPL>
    static hipError_t single_cpl(const StepLaunch& s, const LatDev& L) {
        const uint32_t per_wg = (uint32_t)s.block * CPL;
        const uint32_t segs = (L.nx + per_wg - 1) / per_wg;
        const size_t lds = (Codec<F>::kTable && CPL == 1) ? (size_t)(s.block / 64) * sizeof(EncEntry) * kEncEntries : 0;
        hipLaunchKernelGGL((k_step_single<Q, F, A, COLL, CPL>), dim3(L.ny, segs, L.nz), dim3(s.block), lds, s.stream,
                           L, s.parity, segs, s.enc);
        return hipGetLastError();
    }
    template <int Q, class A, int COLL, int CPL>
    static hipError_t batched_cpl(const StepLaunch& s) {
        hipLaunchKernelGGL((k_step_batched<Q, F, A, COLL, CPL>), dim3(s.grid), dim3(s.block), 0, s.stream,
                           s.lats, s.tiles, s.ntiles, s.parity, s.enc);
        return hipGetLastError();
    }
    template <int Q, class A, int COLL>
    static hipError_t dense_k(const StepLaunch& s) {
        hipLaunchKernelGGL((k_step_dense<Q, F, A, COLL>), dim3(s.grid), dim3(s.block), 0, s.stream, s.lats, s.tiles,
                           s.ntiles, s.parity, s.enc);
        return hipGetLastError();
    }
    // several cells per lane are built for D3Q19 and D3Q27 with SRT and
    // TRT; the other sets and MRT run one cell per lane
    static constexpr bool kWide(int Q) { return Q == 19 || Q == 27; }

    template <int Q, class A, int COLL>
    static hipError_t single_qac(const StepLaunch& s, const LatDev& L) {
        if (s.cpl == 1) return single_cpl<Q, A, COLL, 1>(s, L);
        if constexpr (kWide(Q) && COLL != 2) {
            if constexpr (kMaxCpl >= 2)
                if (s.cpl == 2) return single_cpl<Q, A, COLL, 2>(s, L);
            if constexpr (kMaxCpl >= 4)
                if (s.cpl == 4) return single_cpl<Q, A, COLL, 4>(s, L);
        }
        return hipErrorInvalidValue;
    }
    template <int Q, class A, int COLL>
    static hipError_t step_diag_qac(const StepLaunch& s, const LatDev& L, const double* u_ref, double* partials,
                                    uint32_t segs) {
        hipLaunchKernelGGL((k_step_diag<Q, F, A, COLL>), dim3(L.ny, segs, L.nz), dim3(kDiagThreads), 0, s.stream, L,
                           s.parity, segs, s.enc, u_ref, partials);
        return hipGetLastError();
    }
    template <int Q, class A, int COLL>
    static hipError_t batched_qac(const StepLaunch& s) {
        if (s.dense) return s.cpl == 1 ? dense_k<Q, A, COLL>(s) : hipErrorInvalidValue;
        if (s.cpl == 1) return batched_cpl<Q, A, COLL, 1>(s);
        if constexpr (kWide(Q) && COLL != 2) {
            if constexpr (kMaxCpl >= 2)
                if (s.cpl == 2) return batched_cpl<Q, A, COLL, 2>(s);
            if constexpr (kMaxCpl >= 4)
                if (s.cpl == 4) return batched_cpl<Q, A, COLL, 4>(s);
        }
        return hipErrorInvalidValue;
    }
};

}  // namespace lbm
