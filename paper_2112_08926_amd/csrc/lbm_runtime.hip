// lbm_runtime.hip -- host runtime behind the C interface of include/lbm.h:
// handles, device memory, flags pre-pass, launch configuration, HIP graphs,
// autotuning, encoder tables, diagnostics, codec and copy-probe kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "lbm.h"
#include "lbm_codecs.h"
#include "lbm_internal.h"
#include "lbm_kernels.h"

using namespace lbm;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static lbm_status fail(lbm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

extern "C" const char* lbm_last_error(void) { return g_err.c_str(); }

#include "lbm_enc_table.h"

// FP16C encodes arithmetically; the posits through a table
static bool uses_table(int storage) { return storage >= S_P16_0S && storage <= S_P16_2C; }

static int ddf_bytes(int storage) { return storage == S_FP64 ? 8 : (storage == S_FP32 ? 4 : 2); }

// Per-process device tables of the software encoders (one per format).
struct EncTables {
    EncEntry* dev[8] = {nullptr};
    int device = -1;
};
static EncTables g_tables;

static lbm_status device_table(int storage, const EncEntry** out) {
    *out = nullptr;
    if (!uses_table(storage)) return LBM_OK;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (g_tables.device != dev) {
        g_tables = EncTables{};
        g_tables.device = dev;
    }
    if (!g_tables.dev[storage]) {
        EncEntry host[kEncEntries];
        std::string why;
        if (!build_encoder_table(storage, host, &why))
            return fail(LBM_EDEVICE, "encoder table of format %d: %s", storage, why.c_str());
        EncEntry* d = nullptr;
        HIP_TRY(hipMalloc(&d, sizeof host));
        const hipError_t e = hipMemcpy(d, host, sizeof host, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return fail(LBM_EDEVICE, "encoder table upload: %s", hipGetErrorString(e));
        }
        g_tables.dev[storage] = d;
    }
    *out = g_tables.dev[storage];
    return LBM_OK;
}

// ------------------------------------------------------------------ dispatch by format
#define LBM_FORMAT_SWITCH(storage, EXPR_OF)                    \
    switch (storage) {                                         \
    case S_FP64: return EXPR_OF(fp64);                         \
    case S_FP32: return EXPR_OF(fp32);                         \
    case S_FP16: return EXPR_OF(fp16);                         \
    case S_FP16S: return EXPR_OF(fp16s);                       \
    case S_FP16C: return EXPR_OF(fp16c);                       \
    case S_P16_0S: return EXPR_OF(p16_0s);                     \
    case S_P16_1S: return EXPR_OF(p16_1s);                     \
    case S_P16_2C: return EXPR_OF(p16_2c);                     \
    default: return hipErrorInvalidValue;                      \
    }

namespace lbm {
hipError_t launch_step_single(const StepLaunch& s, const LatDev& lat) {
#define E(N) step_single_##N(s, lat)
    LBM_FORMAT_SWITCH(s.storage, E)
#undef E
}
hipError_t launch_step_batched(const StepLaunch& s) {
#define E(N) step_batched_##N(s)
    LBM_FORMAT_SWITCH(s.storage, E)
#undef E
}
hipError_t launch_init(int q, int storage, int arith, const LatDev& lat, const double* rho, const double* u,
                       const EncEntry* enc, hipStream_t st) {
#define E(N) init_##N(q, arith, lat, rho, u, enc, st)
    LBM_FORMAT_SWITCH(storage, E)
#undef E
}
hipError_t launch_moments(int q, int storage, int arith, const LatDev& lat, int parity, double* rho, double* u,
                          hipStream_t st) {
#define E(N) moments_##N(q, arith, lat, parity, rho, u, st)
    LBM_FORMAT_SWITCH(storage, E)
#undef E
}
hipError_t launch_eq_codes(int q, int storage, int arith, const LatDev& lat, void* out, const EncEntry* enc,
                           hipStream_t st) {
#define E(N) eq_codes_##N(q, arith, lat, out, enc, st)
    LBM_FORMAT_SWITCH(storage, E)
#undef E
}
}  // namespace lbm

// ------------------------------------------------------------------ small kernels
// Later passes of the diagnostics: workgroup b sums the partials
// b*chunk .. min((b+1)*chunk, count) - 1 (the last field by max) into out[b],
// thread t the partials t, t + 256, ... of that range, then a fixed tree, so
// repeated calls give identical results.  Run with many workgroups over the
// first pass's partials, then with one workgroup over theirs.
__global__ void __launch_bounds__(256) k_diag_reduce(const double* __restrict__ in, uint32_t count, uint32_t chunk,
                                                     double* __restrict__ out) {
    __shared__ double s[kDiagFields][256];
    const int t = threadIdx.x;
    const uint32_t begin = blockIdx.x * chunk;
    const uint32_t end = min(begin + chunk, count);
#pragma unroll
    for (int k = 0; k < kDiagFields; k++) {
        double v = 0.0;
        for (uint32_t b = begin + t; b < end; b += 256) {
            const double p = in[(size_t)b * kDiagFields + k];
            v = (k == kDiagFields - 1) ? fmax(v, p) : v + p;
        }
        s[k][t] = v;
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int k = 0; k < kDiagFields; k++)
                s[k][t] = (k == kDiagFields - 1) ? fmax(s[k][t], s[k][t + w]) : s[k][t] + s[k][t + w];
        }
        __syncthreads();
    }
    if (t < kDiagFields) out[(size_t)blockIdx.x * kDiagFields + t] = s[t][0];
}

__global__ void __launch_bounds__(256) k_encode(int storage, const float* __restrict__ in,
                                                uint16_t* __restrict__ out, int64_t n,
                                                const EncEntry* __restrict__ enc) {
    __shared__ EncEntry s_tab[kEncEntries];
    if (enc) {
        for (int k = threadIdx.x; k < kEncEntries; k += blockDim.x) s_tab[k] = enc[k];
        __syncthreads();
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = in[i];
        uint16_t c;
        switch (storage) {
        case S_FP16: c = Codec<S_FP16>::store<float>(x, nullptr); break;
        case S_FP16S: c = Codec<S_FP16S>::store<float>(x, nullptr); break;
        case S_FP16C: c = Codec<S_FP16C>::store<float>(x, nullptr); break;
        case S_P16_0S:
            // as the step encodes: the arithmetic encoder in wavefronts whose
            // inputs all lie in its range, else the table
            c = __all(__builtin_fabsf(x) < FixedRange<S_P16_0S>::kBound) ? FixedRange<S_P16_0S>::store(x)
                                                                           : table_encode(x, s_tab, enc_window_lo(storage));
            break;
        default: c = table_encode(x, s_tab, enc_window_lo(storage)); break;
        }
        out[i] = c;
    }
}

__global__ void __launch_bounds__(256) k_decode(int storage, const uint16_t* __restrict__ in,
                                                float* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = decode16(storage, in[i]);
}

// NEAR bit of every fluid cell with a SOLID cell among its q-1 periodic
// neighbours, and its wall mask (bit i: the source x - c_i is SOLID; bit 31:
// one of those sources is MOVING); reads the caller's flags from `raw`.
template <int Q>
__global__ void __launch_bounds__(256) k_mark_near(const uint8_t* __restrict__ raw, uint8_t* __restrict__ out,
                                                   uint32_t* __restrict__ mask, uint32_t nx, uint32_t ny,
                                                   uint32_t nz) {
    const size_t N = (size_t)nx * ny * nz;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    uint8_t f = raw[n];
    uint32_t m = 0;
    if (!(f & (F_SOLID | F_EQ))) {
        const uint32_t x = (uint32_t)(n % nx), yz = (uint32_t)(n / nx), y = yz % ny, z = yz / ny;
        for (int i = 1; i < Q; i++) {
            const uint32_t sx = (x + nx - VelSet<Q>::c[i][0]) % nx;
            const uint32_t sy = (y + ny - VelSet<Q>::c[i][1]) % ny;
            const uint32_t sz = (z + nz - VelSet<Q>::c[i][2]) % nz;
            const uint8_t fs = raw[sx + (size_t)nx * (sy + (size_t)ny * sz)];
            if (fs & F_SOLID) {
                m |= 1u << i;
                if (fs & F_MOVING) m |= 0x80000000u;
            }
        }
        if (m) f |= F_NEAR;
    }
    out[n] = f;
    mask[n] = m;
}

// Bit g (bit g % 32 of word g / 32) of `bits`: one of the cells 64g ..
// 64g+63 (below N) has a wall source (F_NEAR).  One lane per group of 64
// cells; each wavefront's 64 bits are two whole words, written by its first
// lane.  `waves` wavefronts cover every group plus one pair of zero words,
// which the step's two-word read at the last group reaches.
__global__ void __launch_bounds__(256) k_near_groups(const uint8_t* __restrict__ flags, uint32_t* __restrict__ bits,
                                                     size_t N, size_t waves) {
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t wave = g >> 6;
    if (wave >= waves) return;                       // whole wavefronts
    bool near = false;
    const size_t n0 = g * 64;
    if (n0 + 64 <= N) {
        const uint4* p = (const uint4*)(flags + n0);  // 16-byte aligned: n0 is a multiple of 64
        for (int k = 0; k < 4; k++) {
            const uint4 v = p[k];
            near |= ((v.x | v.y | v.z | v.w) & 0x08080808u) != 0;   // F_NEAR in any byte
        }
    } else {
        for (size_t n = n0; n < N; n++) near |= (flags[n] & F_NEAR) != 0;
    }
    const uint64_t b = __ballot(near);
    if ((threadIdx.x & 63) == 0) {
        bits[2 * wave] = (uint32_t)b;
        bits[2 * wave + 1] = (uint32_t)(b >> 32);
    }
}

// Words of the group bitmap of a lattice of N cells (see k_near_groups).
static size_t near_words(size_t N) {
    const size_t groups = (N + 63) / 64;
    return 2 * ((groups + 63) / 64 + 1);
}

// One 16-byte element per lane, streamed with nontemporal loads and stores
// (the fastest plain copy form measured on gfx950); grid-stride only beyond
// 2^31 workgroups.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy(const f32x4* __restrict__ src, f32x4* __restrict__ dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Memory microbenchmarks (the paper's appendix, Fig. 13: coalesced and
// misaligned reads and writes, one 4-byte element per lane as the DDF
// accesses of a stream-collide kernel).  Misaligned: the element index is
// shifted by one, so every wavefront's 256 bytes straddle two 128-byte
// lines, as the x-shifted pull reads of the step do.  Reads accumulate their
// elements (xor) and write one word per lane only if it equals a value the
// caller never stores, so the loads cannot be dropped and nothing is
// written in practice.  A thread that reads nothing keeps acc = 0 and
// writes nothing, so sink indices stay below n.
// Each thread handles kMemUnroll elements per pass, issued before any is
// used, so that enough loads are in flight to cover the memory latency.
constexpr int kMemUnroll = 8;
__global__ void __launch_bounds__(256) k_mem_read(const uint32_t* __restrict__ src, uint32_t* __restrict__ sink,
                                                  size_t n, uint32_t shift) {
    const size_t T = (size_t)gridDim.x * blockDim.x;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t* s = src + shift;
    uint32_t acc = 0;
    size_t i = t;
    for (; i + (kMemUnroll - 1) * T < n; i += kMemUnroll * T) {
        uint32_t v[kMemUnroll];
#pragma unroll
        for (int k = 0; k < kMemUnroll; k++) v[k] = __builtin_nontemporal_load(s + i + k * T);
#pragma unroll
        for (int k = 0; k < kMemUnroll; k++) acc ^= v[k];
    }
    for (; i < n; i += T) acc ^= __builtin_nontemporal_load(s + i);
    if (acc == 0x9E3779B9u) sink[t] = acc;
}
__global__ void __launch_bounds__(256) k_mem_write(uint32_t* __restrict__ dst, size_t n, uint32_t shift) {
    const size_t T = (size_t)gridDim.x * blockDim.x;
    uint32_t* d = dst + shift;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kMemUnroll - 1) * T < n; i += kMemUnroll * T) {
#pragma unroll
        for (int k = 0; k < kMemUnroll; k++) __builtin_nontemporal_store((uint32_t)(i + k * T), d + i + k * T);
    }
    for (; i < n; i += T) __builtin_nontemporal_store((uint32_t)i, d + i);
}

// ------------------------------------------------------------------ static scratch
// Device memory of lbm_diagnostics_noalloc: the reduction's partials (one set
// of kDiagFields doubles per row tile of the first pass, then per workgroup of
// the second, then the results), in a file-scope device array instead of
// memory of the handle, so that the entry point allocates nothing.  32 MiB:
// lattices of up to 349,000 row tiles (a 512^3 lattice has 262,144).  Each GPU
// holds its own copy for the life of the process.  In host code the array's
// name is not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device, kept per device below.
constexpr size_t kScratchDoubles = (size_t)4 << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices];

// Address of the current device's scratch array, looked up once per device
// (at handle creation, with that device current).
static lbm_status scratch_address(double** out) {
    *out = nullptr;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBM_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

// ------------------------------------------------------------------ handle
struct Lattice {
    lbm_params p{};
    size_t N = 0;
    uint32_t plane = 0;
    void* f[2] = {nullptr, nullptr};
    uint8_t* flags = nullptr;
    uint32_t* wall_mask = nullptr;
    uint32_t* near_bits = nullptr;   // one bit per 64 cells: some cell has a wall source
    size_t near_words = 0;
    void* eq_codes = nullptr;   // q codes of the EQ state
    LatDev dev{};
    // host copy of the caller's flags (empty: no walls), for the tile tables:
    // tiles of wall cells only need no work (their DDFs stay zero) and are
    // left out; tiles with EQ cells are kept, so that every launch mode
    // writes the same equilibrium codes there
    std::vector<uint8_t> host_flags;
    bool needs_step(size_t n0, size_t count) const {
        if (host_flags.empty()) return true;
        const size_t end = std::min(n0 + count, N);
        for (size_t n = n0; n < end; n++)
            if (!(host_flags[n] & LBM_FLAG_SOLID)) return true;
        return false;
    }
};

struct lbm_handle {
    hipStream_t stream = nullptr;
    lbm_alloc_fn alloc = nullptr;
    lbm_free_fn free_ = nullptr;
    void* ctx = nullptr;
    int q = 19, storage = 1, arith = 0, collision = 0;
    std::vector<Lattice> lats;
    int parity = 0;
    int64_t step = 0;
    int64_t device_bytes = 0;
    int num_cus = 256;
    lbm_launch launch{};
    const EncEntry* enc = nullptr;
    // batched launch
    LatDev* d_lats = nullptr;
    Tile* d_tiles = nullptr;
    uint32_t ntiles = 0;
    int tiles_block = 0;
    // graph
    hipGraphExec_t graph = nullptr;
    int graph_steps = 0;
    // diagnostics: partials and results of the reduction (largest lattice)
    double* d_partials = nullptr;
    // per lattice: cell updates with a non-finite density or velocity before
    // the clamp since the lattice was last initialised
    unsigned long long* d_nonfinite = nullptr;
    // size of every device allocation the handle holds (for device_bytes)
    std::unordered_map<void*, size_t> sizes;
    // this device's static scratch array (lbm_diagnostics_noalloc)
    double* scratch = nullptr;
};

// Reduction layout of lattice L: `tiles` first-pass partials (one per row
// tile of kDiagThreads cells, segs per row), `groups` second-pass partials,
// then the results; diag_doubles() is the scratch this needs.
struct DiagLayout {
    uint32_t segs, tiles, groups, chunk;
};
static DiagLayout diag_layout(const Lattice& L) {
    DiagLayout d;
    d.segs = (uint32_t)((L.p.nx + kDiagThreads - 1) / kDiagThreads);
    d.tiles = (uint32_t)L.p.ny * (uint32_t)L.p.nz * d.segs;
    d.groups = std::min<uint32_t>(d.tiles, kDiagReduceBlocks);
    d.chunk = (d.tiles + d.groups - 1) / d.groups;
    return d;
}
static size_t diag_doubles(const DiagLayout& d) {
    return ((size_t)d.tiles + d.groups + 1) * kDiagFields;
}

// Device memory of a handle, through the caller's allocator hooks if given.
// Every allocation the library makes for a handle goes through here, also
// short-lived staging buffers, so that a caller's allocator sees all of it.
static void* dev_alloc(lbm_handle* h, size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    if (h->alloc) p = h->alloc(bytes, h->ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) {
        h->device_bytes += (int64_t)bytes;
        h->sizes[p] = bytes;
    }
    return p;
}
static void dev_free(lbm_handle* h, void* p) {
    if (!p) return;
    auto it = h->sizes.find(p);
    if (it != h->sizes.end()) {
        h->device_bytes -= (int64_t)it->second;
        h->sizes.erase(it);
    }
    if (h->free_) h->free_(p, h->ctx);
    else (void)hipFree(p);
}

static void drop_graph(lbm_handle* h) {
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    h->graph_steps = 0;
}

static void fill_dev(Lattice& L, int arith) {
    (void)arith;
    LatDev& d = L.dev;
    d.f[0] = L.f[0];
    d.f[1] = L.f[1];
    d.flags = L.flags;
    d.wall_mask = L.wall_mask;
    d.near_bits = nullptr;           // no walls until lbm_set_boundaries says otherwise
    d.eq_codes = L.eq_codes;
    d.nx = (uint32_t)L.p.nx;
    d.ny = (uint32_t)L.p.ny;
    d.nz = (uint32_t)L.p.nz;
    d.plane = L.plane;
    d.omega = 1.0 / L.p.tau;
    d.omega_m = 1.0 / (0.5 + L.p.trt_magic / (L.p.tau - 0.5));
    for (int a = 0; a < 3; a++) {
        d.force[a] = L.p.force[a];
        d.wall_u[a] = L.p.wall_u[a];
        d.eq_u[a] = L.p.eq_u[a];
    }
    d.eq_rho = L.p.eq_rho;
    d.shift = L.p.unshifted ? 0.0 : 1.0;
    d.forced = (L.p.force[0] != 0.0 || L.p.force[1] != 0.0 || L.p.force[2] != 0.0) ? 1 : 0;
    d.inv_nx = 1.0f / (float)L.p.nx;
    d.inv_ny = 1.0f / (float)L.p.ny;
}

static lbm_status check_params(const lbm_params& p, int k) {
    if (p.q != 9 && p.q != 15 && p.q != 19 && p.q != 27)
        return fail(LBM_EINVAL, "lattice %d: q must be 9 (D2Q9), 15, 19 or 27", k);
    if (p.q == 9 && p.nz != 1) return fail(LBM_EINVAL, "lattice %d: D2Q9 needs nz = 1", k);
    if (p.collision != LBM_SRT && p.collision != LBM_TRT && p.collision != LBM_MRT)
        return fail(LBM_EINVAL, "lattice %d: unknown collision", k);
    if (p.collision == LBM_MRT && p.q != 19)
        return fail(LBM_EUNSUPPORTED, "lattice %d: MRT is built for D3Q19", k);
    if (p.storage < LBM_FP64 || p.storage > LBM_P16_2C) return fail(LBM_EINVAL, "lattice %d: unknown storage", k);
    if (p.arith != LBM_ARITH_FP32 && p.arith != LBM_ARITH_FP64) return fail(LBM_EINVAL, "lattice %d: unknown arith", k);
    if (p.unshifted != 0 && p.unshifted != 1) return fail(LBM_EINVAL, "lattice %d: unshifted must be 0 or 1", k);
    if (!(p.tau > 0.5) || !std::isfinite(p.tau)) return fail(LBM_EINVAL, "lattice %d: tau must be > 0.5", k);
    if (p.collision == LBM_TRT && !(p.trt_magic > 0.0)) return fail(LBM_EINVAL, "lattice %d: trt_magic must be > 0", k);
    if (p.nx < 1 || p.ny < 1 || p.nz < 1 || p.nx > 65535 || p.ny > 65535 || p.nz > 65535)
        return fail(LBM_EINVAL, "lattice %d: sizes must be in [1, 65535]", k);
    const double N = (double)p.nx * p.ny * p.nz;
    if (N >= 2147483648.0 || N * ddf_bytes(p.storage) >= 4294967296.0)
        return fail(LBM_EINVAL, "lattice %d: too many cells for 32-bit per-plane offsets", k);
    if (p.arith == LBM_ARITH_FP64 && p.storage != LBM_FP64 && p.storage != LBM_FP32)
        return fail(LBM_EUNSUPPORTED, "lattice %d: FP64 arithmetic needs FP64 or FP32 storage", k);
    if (p.arith == LBM_ARITH_FP32 && p.storage == LBM_FP64)
        return fail(LBM_EUNSUPPORTED, "lattice %d: FP64 storage is built with FP64 arithmetic only", k);
    return LBM_OK;
}

static lbm_status run_init(lbm_handle* h, Lattice& L, const double* d_rho, const double* d_u) {
    HIP_TRY(launch_init(h->q, h->storage, h->arith, L.dev, d_rho, d_u, h->enc, h->stream));
    return LBM_OK;
}

static lbm_status rebuild_tiles(lbm_handle* h);

// Elements between consecutive direction planes: the plane rounded up to an
// odd number of pages of max(4 KiB, 1024 DDFs).  A wavefront's 2Q streams
// sit at the same offset in their planes; with a power-of-two plane size (a
// 512^3 plane of 16-bit codes is 2^28 bytes) they meet the same memory
// channels at once.  Measured on the bare access pattern of the D3Q19 step
// (512^3): 16-bit streams move 4.8 TB/s with no gap between planes, 5.7 with
// 4 KiB (12 KiB: 5.7; 8 and 16 KiB: 5.2-5.3); 32-bit 5.5 -> 5.7 with 4 or
// 8 KiB; 64-bit 5.34 -> 5.46 with 8 KiB (4 KiB: 5.17).
static uint32_t plane_elements(size_t N, int bytes_per_ddf) {
    const size_t page = bytes_per_ddf * 1024 > 4096 ? (size_t)bytes_per_ddf * 1024 : 4096;
    size_t pages = (N * (size_t)bytes_per_ddf + page - 1) / page;
    pages |= 1;
    return (uint32_t)(pages * page / (size_t)bytes_per_ddf);
}

extern "C" lbm_status lbm_create(const lbm_params* params, int32_t n_lattices, void* stream,
                                 lbm_alloc_fn alloc, lbm_free_fn free_, void* alloc_ctx, lbm_handle** out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || n_lattices < 1 || n_lattices > 65535) return fail(LBM_EINVAL, "need 1..65535 lattices");
    if ((alloc == nullptr) != (free_ == nullptr)) return fail(LBM_EINVAL, "alloc and free_ go together");
    for (int k = 0; k < n_lattices; k++) {
        lbm_status st = check_params(params[k], k);
        if (st != LBM_OK) return st;
        const lbm_params& a = params[0];
        const lbm_params& b = params[k];
        if (a.q != b.q || a.collision != b.collision || a.storage != b.storage || a.arith != b.arith)
            return fail(LBM_EUNSUPPORTED, "lattice %d: q, collision, storage and arith must match lattice 0", k);
    }
    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) return fail(LBM_ENOMEM, "out of host memory");
    h->stream = (hipStream_t)stream;
    h->alloc = alloc;
    h->free_ = free_;
    h->ctx = alloc_ctx;
    h->q = params[0].q;
    h->storage = params[0].storage;
    h->arith = params[0].arith;
    h->collision = params[0].collision;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete h;
        return fail(LBM_EDEVICE, "no HIP device");
    }
    h->num_cus = prop.multiProcessorCount;
    lbm_status sst = scratch_address(&h->scratch);
    if (sst != LBM_OK) {
        delete h;
        return sst;
    }
    h->launch = {n_lattices > 1 ? LBM_LAUNCH_BATCHED : LBM_LAUNCH_PER_LATTICE, 256, 1, 0, 0};
    lbm_status st = device_table(h->storage, &h->enc);
    if (st != LBM_OK) { delete h; return st; }
    const int b = ddf_bytes(h->storage);
    h->lats.resize(n_lattices);
    h->d_nonfinite = (unsigned long long*)dev_alloc(h, sizeof(unsigned long long) * n_lattices);
    if (!h->d_nonfinite || hipMemsetAsync(h->d_nonfinite, 0, sizeof(unsigned long long) * n_lattices,
                                          h->stream) != hipSuccess) {
        lbm_destroy(h);
        return fail(LBM_ENOMEM, "device allocation of the non-finite counters failed");
    }
    for (int k = 0; k < n_lattices; k++) {
        Lattice& L = h->lats[k];
        L.p = params[k];
        L.N = (size_t)L.p.nx * L.p.ny * L.p.nz;
        L.plane = plane_elements(L.N, b);
        const size_t bytes = (size_t)L.plane * h->q * b;
        L.f[0] = dev_alloc(h, bytes);
        L.f[1] = dev_alloc(h, bytes);
        L.flags = (uint8_t*)dev_alloc(h, L.N);
        L.wall_mask = (uint32_t*)dev_alloc(h, L.N * 4);
        L.near_words = near_words(L.N);
        L.near_bits = (uint32_t*)dev_alloc(h, L.near_words * 4);
        L.eq_codes = dev_alloc(h, 27 * 8);
        if (!L.f[0] || !L.f[1] || !L.flags || !L.wall_mask || !L.near_bits || !L.eq_codes) {
            lbm_destroy(h);
            return fail(LBM_ENOMEM, "device allocation of lattice %d (%zu bytes per buffer) failed", k, bytes);
        }
        if (hipMemsetAsync(L.flags, 0, L.N, h->stream) != hipSuccess ||
            hipMemsetAsync(L.wall_mask, 0, L.N * 4, h->stream) != hipSuccess ||
            hipMemsetAsync(L.near_bits, 0, L.near_words * 4, h->stream) != hipSuccess ||
            hipMemsetAsync(L.f[0], 0, bytes, h->stream) != hipSuccess ||
            hipMemsetAsync(L.f[1], 0, bytes, h->stream) != hipSuccess) {
            lbm_destroy(h);
            return fail(LBM_EDEVICE, "hipMemsetAsync failed");
        }
        fill_dev(L, h->arith);
        L.dev.nonfinite = h->d_nonfinite + k;
        if (launch_eq_codes(h->q, h->storage, h->arith, L.dev, L.eq_codes, h->enc, h->stream) != hipSuccess) {
            lbm_destroy(h);
            return fail(LBM_EDEVICE, "equilibrium code table failed");
        }
        st = run_init(h, L, nullptr, nullptr);
        if (st != LBM_OK) { lbm_destroy(h); return st; }
    }
    size_t diag_work = 0;
    for (const Lattice& L : h->lats) diag_work = std::max(diag_work, diag_doubles(diag_layout(L)));
    h->d_partials = (double*)dev_alloc(h, sizeof(double) * diag_work);
    h->d_lats = (LatDev*)dev_alloc(h, sizeof(LatDev) * n_lattices);
    if (!h->d_partials || !h->d_lats) {
        lbm_destroy(h);
        return fail(LBM_ENOMEM, "device allocation failed");
    }
    std::vector<LatDev> descs(n_lattices);
    for (int k = 0; k < n_lattices; k++) descs[k] = h->lats[k].dev;
    if (hipMemcpyAsync(h->d_lats, descs.data(), sizeof(LatDev) * n_lattices, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        lbm_destroy(h);
        return fail(LBM_EDEVICE, "descriptor upload failed");
    }
    st = rebuild_tiles(h);
    if (st != LBM_OK) { lbm_destroy(h); return st; }
    *out = h;
    return LBM_OK;
}

extern "C" void lbm_destroy(lbm_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    for (auto& L : h->lats) {
        dev_free(h, L.f[0]);
        dev_free(h, L.f[1]);
        dev_free(h, L.flags);
        dev_free(h, L.wall_mask);
        dev_free(h, L.near_bits);
        dev_free(h, L.eq_codes);
    }
    dev_free(h, h->d_partials);
    dev_free(h, h->d_lats);
    dev_free(h, h->d_tiles);
    dev_free(h, h->d_nonfinite);
    delete h;
}

// Clears a lattice's count of non-finite updates (when it is initialised).
static hipError_t reset_nonfinite(lbm_handle* h, int32_t k) {
    return hipMemsetAsync(h->d_nonfinite + k, 0, sizeof(unsigned long long), h->stream);
}

static lbm_status check_lattice(lbm_handle* h, int32_t k) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (k < 0 || k >= (int)h->lats.size()) return fail(LBM_EINVAL, "lattice index %d out of range", k);
    return LBM_OK;
}

// ------------------------------------------------------------------ tiles
// Tile table of the batched launch for the current block size: row segments
// of `block` cells, lattice by lattice, row by row.  The old table is
// withdrawn before anything can fail (with any graph that was captured with
// it), and the new one is published only once it is on the device, so after
// a failure the handle holds no table and lbm_step refuses batched launches
// instead of reading a freed or short table.
static lbm_status rebuild_tiles(lbm_handle* h) {
    const int T = h->launch.block * h->launch.cells_per_lane;
    const bool dense = h->launch.mode == LBM_LAUNCH_DENSE;
    const int key = 2 * T + (dense ? 1 : 0);
    if (h->d_tiles && h->tiles_block == key) return LBM_OK;
    std::vector<Tile> tiles;
    for (size_t k = 0; k < h->lats.size(); k++) {
        const lbm_params& p = h->lats[k].p;
        const Lattice& L = h->lats[k];
        if (dense) {
            // T consecutive cells each, from the start cell's coordinates
            const size_t N = L.N, row = (size_t)p.nx, slab = row * p.ny;
            for (size_t n0 = 0; n0 < N; n0 += T)
                if (L.needs_step(n0, T))
                    tiles.push_back(Tile{(uint16_t)k, (uint16_t)(n0 % row), (uint16_t)((n0 / row) % p.ny),
                                         (uint16_t)(n0 / slab)});
            continue;
        }
        for (int z = 0; z < p.nz; z++)
            for (int y = 0; y < p.ny; y++)
                for (int x0 = 0; x0 < p.nx; x0 += T) {
                    const size_t n0 = (size_t)x0 + (size_t)p.nx * ((size_t)y + (size_t)p.ny * z);
                    if (L.needs_step(n0, std::min<size_t>(T, p.nx - x0)))
                        tiles.push_back(Tile{(uint16_t)k, (uint16_t)x0, (uint16_t)y, (uint16_t)z});
                }
    }
    drop_graph(h);
    Tile* old = h->d_tiles;
    h->d_tiles = nullptr;
    h->ntiles = 0;
    h->tiles_block = 0;
    dev_free(h, old);
    if (tiles.size() >= 0xFFFFFFFFull) return fail(LBM_EINVAL, "too many tiles");
    Tile* t = (Tile*)dev_alloc(h, sizeof(Tile) * std::max<size_t>(tiles.size(), 1));   // may be empty
    if (!t) return fail(LBM_ENOMEM, "tile table allocation failed");
    hipError_t e = hipMemcpyAsync(t, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        dev_free(h, t);
        return fail(LBM_EDEVICE, "tile table upload failed: %s", hipGetErrorString(e));
    }
    h->d_tiles = t;
    h->ntiles = (uint32_t)tiles.size();
    h->tiles_block = key;
    return LBM_OK;
}

// ------------------------------------------------------------------ stepping
static StepLaunch make_launch(lbm_handle* h, const lbm_launch& cfg, int parity) {
    StepLaunch s{};
    s.q = h->q;
    s.storage = h->storage;
    s.arith = h->arith;
    s.collision = h->collision;
    s.block = cfg.block;
    s.cpl = cfg.cells_per_lane;
    s.dense = cfg.mode == LBM_LAUNCH_DENSE ? 1 : 0;
    s.parity = parity;
    s.lats = h->d_lats;
    s.tiles = h->d_tiles;
    s.ntiles = h->ntiles;
    s.grid = cfg.persistent > 0 ? (uint32_t)std::min<int64_t>((int64_t)cfg.persistent * h->num_cus, h->ntiles)
                                : h->ntiles;
    s.enc = h->enc;
    s.stream = h->stream;
    return s;
}

// Enqueue one time step with the given configuration, reading buffer `parity`.
// Batched launches need the tile table (absent only after a failed rebuild).
static hipError_t enqueue_step(lbm_handle* h, const lbm_launch& cfg, int parity) {
    const StepLaunch s = make_launch(h, cfg, parity);
    if (cfg.mode != LBM_LAUNCH_PER_LATTICE) {
        if (!h->d_tiles) return hipErrorInvalidValue;
        return s.ntiles ? launch_step_batched(s) : hipSuccess;
    }
    for (auto& L : h->lats) {
        hipError_t e = launch_step_single(s, L.dev);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static lbm_status ensure_graph(lbm_handle* h) {
    const int K = h->launch.graph_steps;
    if (K <= 0 || (h->graph && h->graph_steps == K)) return LBM_OK;
    drop_graph(h);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int s = 0; s < K && e == hipSuccess; s++) e = enqueue_step(h, h->launch, s & 1);
    hipError_t e2 = hipStreamEndCapture(h->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(LBM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    h->graph = ex;
    h->graph_steps = K;
    return LBM_OK;
}

extern "C" lbm_status lbm_step(lbm_handle* h, int64_t n) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (n < 0) return fail(LBM_EINVAL, "n_steps must be >= 0");
    if (h->launch.mode != LBM_LAUNCH_PER_LATTICE && !h->d_tiles)
        return fail(LBM_EINVAL, "no tile table for the batched launch (a previous call failed to build it); "
                                "set the launch configuration again");
    lbm_status st = ensure_graph(h);
    if (st != LBM_OK) return st;
    const int K = h->graph ? h->graph_steps : 0;
    while (n > 0) {
        if (K > 0 && h->parity == 0 && n >= K) {
            HIP_TRY(hipGraphLaunch(h->graph, h->stream));
            n -= K;
            h->step += K;       // K is even: parity unchanged
            continue;
        }
        HIP_TRY(enqueue_step(h, h->launch, h->parity));
        h->parity ^= 1;
        h->step += 1;
        n -= 1;
    }
    return LBM_OK;
}

// ------------------------------------------------------------------ boundaries and state
extern "C" lbm_status lbm_set_boundaries(lbm_handle* h, int32_t k, const uint8_t* flags) {
    lbm_status st = check_lattice(h, k);
    if (st != LBM_OK) return st;
    if (!flags) return fail(LBM_EINVAL, "flags is NULL");
    Lattice& L = h->lats[k];
    std::vector<uint8_t> fl(L.N);
    for (size_t n = 0; n < L.N; n++) {
        const uint8_t f = flags[n];
        if (f & ~(LBM_FLAG_SOLID | LBM_FLAG_EQ | LBM_FLAG_MOVING))
            return fail(LBM_EINVAL, "cell %zu: unknown flag bits 0x%x", n, f);
        if ((f & LBM_FLAG_MOVING) && !(f & LBM_FLAG_SOLID))
            return fail(LBM_EINVAL, "cell %zu: MOVING without SOLID", n);
        if ((f & LBM_FLAG_EQ) && (f & LBM_FLAG_SOLID))
            return fail(LBM_EINVAL, "cell %zu: EQ together with SOLID", n);
        fl[n] = f;
    }
    // NEAR (fluid cell with a SOLID cell among its q-1 neighbours) is marked on
    // the device from a staging copy of the caller's flags.
    uint8_t* d_raw = (uint8_t*)dev_alloc(h, L.N);
    if (!d_raw) return fail(LBM_ENOMEM, "flags staging buffer");
    hipError_t e = hipMemcpyAsync(d_raw, fl.data(), L.N, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        const dim3 grid((unsigned)((L.N + 255) / 256));
        switch (h->q) {
#define LBM_MARK(QQ) case QQ: hipLaunchKernelGGL(k_mark_near<QQ>, grid, dim3(256), 0, h->stream, d_raw, L.flags, \
                                                 L.wall_mask, L.dev.nx, L.dev.ny, L.dev.nz); break;
        LBM_MARK(9) LBM_MARK(15) LBM_MARK(19) LBM_MARK(27)
#undef LBM_MARK
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        const size_t waves = L.near_words / 2;
        hipLaunchKernelGGL(k_near_groups, dim3((unsigned)((waves * 64 + 255) / 256)), dim3(256), 0, h->stream,
                           L.flags, L.near_bits, L.N, waves);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = reset_nonfinite(h, k);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);   // fl is a local buffer
    dev_free(h, d_raw);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "flag upload failed: %s", hipGetErrorString(e));
    drop_graph(h);
    L.host_flags.assign(flags, flags + L.N);
    // Lattices without walls skip the group bitmap in the step (its read is
    // the one thing a wavefront waits for before its first DDF load).
    bool any_solid = false;
    for (size_t n = 0; n < L.N && !any_solid; n++) any_solid = (flags[n] & LBM_FLAG_SOLID) != 0;
    L.dev.near_bits = any_solid ? L.near_bits : nullptr;
    if (hipMemcpyAsync(h->d_lats + k, &L.dev, sizeof(LatDev), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return fail(LBM_EDEVICE, "descriptor upload failed");
    h->tiles_block = 0;                  // the tile tables depend on the flags
    st = rebuild_tiles(h);
    if (st != LBM_OK) return st;
    st = run_init(h, L, nullptr, nullptr);
    if (st != LBM_OK) return st;
    h->step = 0;
    return LBM_OK;
}

// The initialisation writes both buffers, so the current parity stays valid.
extern "C" lbm_status lbm_set_rho_u(lbm_handle* h, int32_t k, const double* rho, const double* u) {
    lbm_status st = check_lattice(h, k);
    if (st != LBM_OK) return st;
    Lattice& L = h->lats[k];
    double* d_rho = rho ? (double*)dev_alloc(h, L.N * sizeof(double)) : nullptr;
    double* d_u = u ? (double*)dev_alloc(h, 3 * L.N * sizeof(double)) : nullptr;
    if ((rho && !d_rho) || (u && !d_u)) {
        dev_free(h, d_rho);
        dev_free(h, d_u);
        return fail(LBM_ENOMEM, "rho/u upload buffers");
    }
    hipError_t e = hipSuccess;
    if (rho) e = hipMemcpyAsync(d_rho, rho, L.N * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(d_u, u, 3 * L.N * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = reset_nonfinite(h, k);
    st = e == hipSuccess ? run_init(h, L, d_rho, d_u) : LBM_OK;
    const hipError_t es = hipStreamSynchronize(h->stream);    // the uploads read the caller's buffers
    if (e == hipSuccess) e = es;
    dev_free(h, d_rho);
    dev_free(h, d_u);
    if (st != LBM_OK) return st;
    if (e != hipSuccess) return fail(LBM_EDEVICE, "initialisation failed: %s", hipGetErrorString(e));
    h->step = 0;
    return LBM_OK;
}

extern "C" lbm_status lbm_get_rho_u(lbm_handle* h, int32_t k, double* rho, double* u) {
    lbm_status st = check_lattice(h, k);
    if (st != LBM_OK) return st;
    Lattice& L = h->lats[k];
    double* d = (double*)dev_alloc(h, 4 * L.N * sizeof(double));
    if (!d) return fail(LBM_ENOMEM, "moments buffer");
    hipError_t e = launch_moments(h->q, h->storage, h->arith, L.dev, h->parity, d, d + L.N, h->stream);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, d, L.N * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, d + L.N, 3 * L.N * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    dev_free(h, d);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "moments failed: %s", hipGetErrorString(e));
    return LBM_OK;
}

extern "C" lbm_status lbm_set_ddf(lbm_handle* h, int32_t k, const void* host) {
    lbm_status st = check_lattice(h, k);
    if (st != LBM_OK) return st;
    if (!host) return fail(LBM_EINVAL, "host buffer is NULL");
    Lattice& L = h->lats[k];
    const size_t b = ddf_bytes(h->storage);
    // both buffers, so that the cells a step never writes (SOLID, EQ) agree
    for (int buf = 0; buf < 2; buf++)
        for (int i = 0; i < h->q; i++)
            HIP_TRY(hipMemcpyAsync((char*)L.f[buf] + (size_t)i * L.plane * b, (const char*)host + (size_t)i * L.N * b,
                                   L.N * b, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(reset_nonfinite(h, k));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

extern "C" lbm_status lbm_get_ddf(lbm_handle* h, int32_t k, void* host) {
    lbm_status st = check_lattice(h, k);
    if (st != LBM_OK) return st;
    if (!host) return fail(LBM_EINVAL, "host buffer is NULL");
    Lattice& L = h->lats[k];
    const size_t b = ddf_bytes(h->storage);
    for (int i = 0; i < h->q; i++)
        HIP_TRY(hipMemcpyAsync((char*)host + (size_t)i * L.N * b, (const char*)L.f[h->parity] + (size_t)i * L.plane * b,
                               L.N * b, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// The FP64 diagnostics of lattice k: the first pass, the two reduction
// passes, then the results and the lattice's count of non-finite updates to
// the host.  `work`: device memory of at least diag_doubles() doubles for
// the partials and results.  Synchronises.  d_ref: device u_ref or null.
// with_step: the first pass is the fused step (k_step_diag) instead of
// k_diag: the diagnostics are those of the state the step reads, and the
// handle has advanced one step when this returns.
static lbm_status run_diagnostics(lbm_handle* h, int32_t k, const double* d_ref, double* work, lbm_diag* out,
                                  bool with_step = false) {
    Lattice& L = h->lats[k];
    const DiagLayout dl = diag_layout(L);
    double* partials = work;
    double* groups = work + (size_t)dl.tiles * kDiagFields;
    double* res_dev = groups + (size_t)dl.groups * kDiagFields;
    const uint32_t segs = dl.segs;
    double res[kDiagFields];
    unsigned long long nonfinite_updates = 0;
    const int64_t step = h->step;
    hipError_t e;
    if (with_step) {
        const StepLaunch s = make_launch(h, h->launch, h->parity);
#define E(N) step_diag_##N(s, L.dev, d_ref, partials, segs)
        switch (h->storage) {
        case S_FP64: e = E(fp64); break;
        case S_FP32: e = E(fp32); break;
        case S_FP16: e = E(fp16); break;
        case S_FP16S: e = E(fp16s); break;
        case S_FP16C: e = E(fp16c); break;
        case S_P16_0S: e = E(p16_0s); break;
        case S_P16_1S: e = E(p16_1s); break;
        default: e = E(p16_2c); break;
        }
#undef E
        if (e == hipSuccess) {
            h->parity ^= 1;
            h->step += 1;
        }
    } else {
#define E(N) diag_##N(h->q, h->arith, L.dev, h->parity, d_ref, partials, segs, h->stream)
        switch (h->storage) {
        case S_FP64: e = E(fp64); break;
        case S_FP32: e = E(fp32); break;
        case S_FP16: e = E(fp16); break;
        case S_FP16S: e = E(fp16s); break;
        case S_FP16C: e = E(fp16c); break;
        case S_P16_0S: e = E(p16_0s); break;
        case S_P16_1S: e = E(p16_1s); break;
        default: e = E(p16_2c); break;
        }
#undef E
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_diag_reduce, dim3(dl.groups), dim3(256), 0, h->stream, partials, dl.tiles, dl.chunk,
                           groups);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_diag_reduce, dim3(1), dim3(256), 0, h->stream, groups, dl.groups, dl.groups, res_dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(res, res_dev, sizeof res, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&nonfinite_updates, h->d_nonfinite + k, sizeof nonfinite_updates, hipMemcpyDeviceToHost,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "diagnostics failed: %s", hipGetErrorString(e));
    out->mass = res[0];
    out->momentum[0] = res[1];
    out->momentum[1] = res[2];
    out->momentum[2] = res[3];
    out->kinetic_energy = res[4];
    out->l2_error = d_ref ? (res[6] > 0 ? std::sqrt(res[5] / res[6]) : 0.0) : -1.0;
    out->force_on_solid[0] = res[7];
    out->force_on_solid[1] = res[8];
    out->force_on_solid[2] = res[9];
    out->nonfinite_cells = (int64_t)res[10];
    out->u_max = std::sqrt(res[11]);
    out->step = step;
    out->nonfinite_updates = (int64_t)nonfinite_updates;
    if (out->nonfinite_cells > 0 || out->nonfinite_updates > 0)
        return fail(LBM_ENONFINITE, "lattice %d: %lld fluid cells with non-finite fields now, %lld cell updates "
                    "with a non-finite density or velocity since the last initialisation", k,
                    (long long)out->nonfinite_cells, (long long)out->nonfinite_updates);
    return LBM_OK;
}

extern "C" lbm_status lbm_diagnostics(lbm_handle* h, int32_t k, const double* u_ref, lbm_diag* out) {
    lbm_status st = check_lattice(h, k);
    if (st != LBM_OK) return st;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    Lattice& L = h->lats[k];
    double* d_ref = nullptr;
    if (u_ref) {
        d_ref = (double*)dev_alloc(h, 3 * L.N * sizeof(double));
        if (!d_ref) return fail(LBM_ENOMEM, "u_ref buffer");
        const hipError_t e = hipMemcpyAsync(d_ref, u_ref, 3 * L.N * sizeof(double), hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) {
            dev_free(h, d_ref);
            return fail(LBM_EDEVICE, "u_ref upload failed: %s", hipGetErrorString(e));
        }
    }
    st = run_diagnostics(h, k, d_ref, h->d_partials, out);
    dev_free(h, d_ref);
    return st;
}

extern "C" lbm_status lbm_step_diagnostics(lbm_handle* h, const double* u_ref_dev, lbm_diag* out) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    if (h->lats.size() != 1)
        return fail(LBM_EUNSUPPORTED, "lbm_step_diagnostics steps a handle of one lattice (this one has %zu)",
                    h->lats.size());
    return run_diagnostics(h, 0, u_ref_dev, h->d_partials, out, true);
}

extern "C" lbm_status lbm_diagnostics_noalloc(lbm_handle* h, int32_t k, const double* u_ref_dev, lbm_diag* out) {
    lbm_status st = check_lattice(h, k);
    if (st != LBM_OK) return st;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    const size_t need = diag_doubles(diag_layout(h->lats[k]));
    if (need > kScratchDoubles)
        return fail(LBM_EINVAL, "lattice %d needs %zu bytes of reduction scratch; the static array holds %zu "
                    "(lbm_diagnostics has no such limit)", k, need * sizeof(double), kScratchDoubles * sizeof(double));
    // every first-pass workgroup writes all of its slot and each later pass
    // writes every slot the next one reads, so nothing needs clearing
    return run_diagnostics(h, k, u_ref_dev, h->scratch, out);
}

// ------------------------------------------------------------------ launch configuration
static lbm_status check_launch(lbm_handle* h, const lbm_launch& c) {
    if (c.mode != LBM_LAUNCH_PER_LATTICE && c.mode != LBM_LAUNCH_BATCHED && c.mode != LBM_LAUNCH_DENSE)
        return fail(LBM_EINVAL, "unknown launch mode");
    if (c.block != 64 && c.block != 128 && c.block != 256 && c.block != 512) return fail(LBM_EINVAL, "block must be 64..512");
    if (c.mode == LBM_LAUNCH_DENSE && c.cells_per_lane != 1)
        return fail(LBM_EINVAL, "cell-contiguous tiles take one cell per lane");
    if (c.cells_per_lane != 1 && c.cells_per_lane != 2 && c.cells_per_lane != 4)
        return fail(LBM_EINVAL, "cells_per_lane must be 1, 2 or 4");
    if ((h->q != 19 && h->q != 27) && c.cells_per_lane != 1)
        return fail(LBM_EUNSUPPORTED, "several cells per lane are built for D3Q19 and D3Q27");
    if (h->collision == LBM_MRT && c.cells_per_lane != 1)
        return fail(LBM_EUNSUPPORTED, "MRT runs one cell per lane");
    if (c.cells_per_lane == 4 && ddf_bytes(h->storage) != 2)
        return fail(LBM_EUNSUPPORTED, "cells_per_lane 4 needs 16-bit storage");
    if (c.cells_per_lane > 1 && ddf_bytes(h->storage) == 8)
        return fail(LBM_EUNSUPPORTED, "FP64 storage runs one cell per lane");
    for (size_t k = 0; k < h->lats.size(); k++)
        if (h->lats[k].p.nx % c.cells_per_lane)
            return fail(LBM_EINVAL, "lattice %zu: nx = %d is not a multiple of cells_per_lane", k,
                        h->lats[k].p.nx);
    if (c.persistent < 0 || c.persistent > 64) return fail(LBM_EINVAL, "persistent must be in [0, 64]");
    if (c.graph_steps < 0 || (c.graph_steps & 1) || c.graph_steps > 100000)
        return fail(LBM_EINVAL, "graph_steps must be even and >= 0");
    if (c.graph_steps > 0 && h->stream == nullptr)
        return fail(LBM_EINVAL, "HIP graphs need a non-null stream (the null stream cannot be captured)");
    return LBM_OK;
}

extern "C" lbm_status lbm_set_launch(lbm_handle* h, const lbm_launch* cfg) {
    if (!h || !cfg) return fail(LBM_EINVAL, "NULL argument");
    lbm_status st = check_launch(h, *cfg);
    if (st != LBM_OK) return st;
    drop_graph(h);
    const lbm_launch keep = h->launch;
    h->launch = *cfg;
    st = rebuild_tiles(h);
    if (st != LBM_OK) {
        // back to the previous configuration; should its table fail too,
        // lbm_step refuses batched launches until a launch is set again
        const std::string why = g_err;
        h->launch = keep;
        (void)rebuild_tiles(h);
        g_err = why;
    }
    return st;
}

extern "C" lbm_status lbm_get_launch(lbm_handle* h, lbm_launch* cfg) {
    if (!h || !cfg) return fail(LBM_EINVAL, "NULL argument");
    *cfg = h->launch;
    return LBM_OK;
}

extern "C" lbm_status lbm_autotune(lbm_handle* h, int32_t trial_steps, lbm_launch* best) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (trial_steps < 1) return fail(LBM_EINVAL, "trial_steps must be >= 1");
    const lbm_launch keep = h->launch;
    std::vector<lbm_launch> cands;
    const int blocks[] = {64, 128, 256, 512};
    // one or two cells per lane (four never won on the workloads measured)
    for (int cpl : {1, 2}) {
        for (int b : blocks) {
            const lbm_launch c{LBM_LAUNCH_PER_LATTICE, b, cpl, 0, keep.graph_steps};
            if (check_launch(h, c) != LBM_OK) continue;
            cands.push_back(c);
            // persistent grids of half and full occupancy (2048 threads per CU)
            const int pers[] = {0, 1024 / b, 2048 / b};
            for (int pz : pers) {
                if (h->lats.size() > 1) cands.push_back({LBM_LAUNCH_BATCHED, b, cpl, pz, keep.graph_steps});
                if (cpl == 1) cands.push_back({LBM_LAUNCH_DENSE, b, 1, pz, keep.graph_steps});
            }
        }
    }
    g_err.clear();
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 1e30f;
    lbm_launch best_cfg = keep;
    for (const lbm_launch& c : cands) {
        h->launch = c;
        if (rebuild_tiles(h) != LBM_OK) continue;      // e.g. no memory for its tile tables: skip it
        // warm-up, then the better of two timed runs (one run alone is
        // noisy enough to flip close candidates); always reading the
        // current buffer
        hipError_t e = enqueue_step(h, c, h->parity);
        float ms = 1e30f;
        for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {
            e = hipEventRecord(e0, h->stream);
            for (int s = 0; s < trial_steps && e == hipSuccess; s++) e = enqueue_step(h, c, h->parity);
            if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e == hipSuccess) ms = std::min(ms, t);
        }
        if (e != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            drop_graph(h);
            h->launch = keep;
            (void)rebuild_tiles(h);
            return fail(LBM_EDEVICE, "autotune launch failed: %s", hipGetErrorString(e));
        }
        // ties go to the smaller workgroup (candidates are in increasing size)
        if (ms < best_ms * 0.995f) {
            best_ms = ms;
            best_cfg = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graph(h);
    h->launch = best_cfg;
    lbm_status st = rebuild_tiles(h);
    if (st != LBM_OK) return st;
    if (best) *best = best_cfg;
    return LBM_OK;
}

extern "C" lbm_status lbm_info_get(lbm_handle* h, lbm_info* out) {
    if (!h || !out) return fail(LBM_EINVAL, "NULL argument");
    int64_t cells = 0;
    for (auto& L : h->lats) cells += (int64_t)L.N;
    out->cells = cells;
    out->device_bytes = h->device_bytes;
    out->n_lattices = (int32_t)h->lats.size();
    out->bytes_per_ddf = ddf_bytes(h->storage);
    out->step = h->step;
    return LBM_OK;
}

extern "C" lbm_status lbm_synchronize(lbm_handle* h) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// ------------------------------------------------------------------ codecs and probe
extern "C" lbm_status lbm_encode(int32_t storage, const float* d_in, uint16_t* d_out, int64_t n, void* stream) {
    if (storage < LBM_FP16 || storage > LBM_P16_2C) return fail(LBM_EINVAL, "not a 16-bit format");
    if (n < 0 || (n > 0 && (!d_in || !d_out))) return fail(LBM_EINVAL, "bad arguments");
    if (n == 0) return LBM_OK;
    const EncEntry* enc = nullptr;
    lbm_status st = device_table(storage, &enc);
    if (st != LBM_OK) return st;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_encode, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, storage, d_in, d_out, n, enc);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

extern "C" lbm_status lbm_decode(int32_t storage, const uint16_t* d_in, float* d_out, int64_t n, void* stream) {
    if (storage < LBM_FP16 || storage > LBM_P16_2C) return fail(LBM_EINVAL, "not a 16-bit format");
    if (n < 0 || (n > 0 && (!d_in || !d_out))) return fail(LBM_EINVAL, "bad arguments");
    if (n == 0) return LBM_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_decode, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, storage, d_in, d_out, n);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

extern "C" lbm_status lbm_memory_probe(int32_t kind, const void* d_src, void* d_dst, size_t bytes, void* stream) {
    if (kind == LBM_PROBE_COPY) return lbm_copy_probe(d_src, d_dst, bytes, stream);
    if (kind < LBM_PROBE_READ || kind > LBM_PROBE_WRITE_MISALIGNED) return fail(LBM_EINVAL, "unknown probe kind %d", kind);
    const bool read = kind == LBM_PROBE_READ || kind == LBM_PROBE_READ_MISALIGNED;
    const uint32_t shift = (kind == LBM_PROBE_READ_MISALIGNED || kind == LBM_PROBE_WRITE_MISALIGNED) ? 1u : 0u;
    if ((read && !d_src) || !d_dst || (bytes % 4) || ((uintptr_t)d_src % 4) || ((uintptr_t)d_dst % 4) || bytes < 8)
        return fail(LBM_EINVAL, "memory probe needs 4-byte aligned pointers and a size of at least 8, a multiple of 4");
    const size_t n = bytes / 4 - shift;            // elements accessed, shift .. shift + n - 1
    // a grid of 64 workgroups of 256 threads per CU (enough waves in flight;
    // each thread then walks the buffer in strides of the whole grid)
    const size_t threads = 256;
    const size_t blocks = std::min<size_t>((n + threads - 1) / threads, (size_t)64 * 256);
    if (read) {
        hipLaunchKernelGGL(k_mem_read, dim3((unsigned)blocks), dim3(threads), 0, (hipStream_t)stream,
                           (const uint32_t*)d_src, (uint32_t*)d_dst, n, shift);
    } else {
        hipLaunchKernelGGL(k_mem_write, dim3((unsigned)blocks), dim3(threads), 0, (hipStream_t)stream, (uint32_t*)d_dst,
                           n, shift);
    }
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

extern "C" lbm_status lbm_copy_probe(const void* d_src, void* d_dst, size_t bytes, void* stream) {
    if (!d_src || !d_dst || (bytes % 16) || ((uintptr_t)d_src % 16) || ((uintptr_t)d_dst % 16))
        return fail(LBM_EINVAL, "copy probe needs 16-byte aligned pointers and size");
    const size_t n = bytes / 16;
    if (n == 0) return LBM_OK;
    const size_t blocks = std::min<size_t>((n + 255) / 256, (size_t)1 << 31);
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (const f32x4*)d_src,
                       (f32x4*)d_dst, n);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}
