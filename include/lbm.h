/*
 * lbm.h -- C interface of liblbm.so, an MI355X (gfx950) implementation of the
 * lattice Boltzmann hot path of Lehmann, Krause, Amati, Sega, Harting, Gekle,
 * "On the accuracy and performance of the lattice Boltzmann method with
 * 64-bit, 32-bit and novel 16-bit number formats" (arXiv 2112.08926).
 *
 * What the library computes (paper references by section/equation/table):
 *   - the fused pull stream-collide step of the appendix "LBM equations in a
 *     nutshell" (streaming, fields, equilibrium, collision) with DDF shifting
 *     (Sec. 2.2: DDFs stored as f_i - w_i, shifted equilibrium in its 3-FMA
 *     order, density summed with the 1 added last, velocity summed with
 *     alternating signs), the velocity clamp and mid-grid bounce-back of the
 *     paper's D3Q19 SRT kernel listing;
 *   - velocity sets D2Q9, D3Q15, D3Q19 and D3Q27 (Table 1), collision SRT
 *     (BGK), TRT or, for D3Q19, MRT; Guo body force, stationary and moving
 *     bounce-back walls, cells held at a fixed equilibrium;
 *   - FP32 arithmetic with DDFs stored as FP32, IEEE FP16, FP16S, FP16C,
 *     P16_0S, P16_1S or P16_2C (Sec. 3, Table 2), and an FP64 arithmetic path
 *     with FP64 or FP32 storage;
 *   - FP64 reductions of mass, momentum, kinetic energy (Sec. 4.2), the L2
 *     velocity error of Sec. 4.1 and the momentum-exchange force on walls;
 *   - ensembles of independent lattices of different sizes advanced together.
 *
 * Conventions for every function:
 *   - Status codes are returned, never thrown; lbm_last_error() gives a
 *     thread-local message for the last failure in the calling thread.
 *   - Host arrays passed in are borrowed for the duration of the call only.
 *   - The library owns all device memory it allocates (through the optional
 *     allocator hooks of lbm_create, else hipMalloc) and frees it in
 *     lbm_destroy.
 *   - All device work of a handle is enqueued on the stream given to
 *     lbm_create.  Only functions that return host data synchronise it.
 *   - A handle may be used by one thread at a time.
 *   - Cell index n = x + (y + z*ny)*nx; per-cell vector fields are stored
 *     component-major: u[0*N + n] = u_x, u[1*N + n] = u_y, u[2*N + n] = u_z.
 *   - All faces are periodic; walls and inflow/outflow are made with cell
 *     flags.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_handle lbm_handle;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,        /* invalid argument (message says which) */
    LBM_ENOMEM = -2,        /* device or host allocation failed */
    LBM_EDEVICE = -3,       /* a HIP call failed */
    LBM_EUNSUPPORTED = -4,  /* valid but not built combination */
    LBM_ENONFINITE = -5     /* diagnostics found non-finite fields */
} lbm_status;

/* Velocity sets (Sec. 2.1, Table 1), named by their number of directions:
 * rest first, then opposite pairs (2k-1, 2k).  D2Q9 needs nz = 1.  Several
 * cells per lane exist for D3Q19 and D3Q27.  (D3Q7
 * and D3Q13 of Table 1 are not offered: with the equilibrium of Sec. 2.2
 * D3Q7 does not conserve momentum (its c_s^2 is 1/4) and D3Q13 lacks the
 * fourth-order isotropy of the viscous stress.) */
typedef enum { LBM_D2Q9 = 9, LBM_D3Q15 = 15, LBM_D3Q19 = 19, LBM_D3Q27 = 27 } lbm_velset;
/* Collision operators (Sec. 2.1 names SRT, TRT and MRT; the paper defines
 * none beyond its SRT listing).  TRT: the pairs' symmetric parts relax with
 * 1/tau, the antisymmetric parts with the rate from trt_magic.  MRT (D3Q19
 * only): the moment basis of d'Humieres et al. (2002) with rates 0 for rho
 * and j, 1/tau for the five shear moments, 1.19 (e), 1.4 (eps, 3pi_xx,
 * pi_ww), 1.2 (q) and 1.98 (m); the Guo source is added in moment space
 * scaled by 1 - s/2. */
typedef enum { LBM_SRT = 0, LBM_TRT = 1, LBM_MRT = 2 } lbm_collision;

/* DDF storage formats (Sec. 3, Table 2).  Codes of the 16-bit formats:
 * FP16 IEEE binary16 (round to nearest even); FP16S binary16 of x*2^15;
 * FP16C 1|4|11 bits, bias 15, no Inf/NaN; P16_0S and P16_1S posits with 0/1
 * exponent bits in sign-magnitude form holding x*2^7; P16_2C the asymmetric
 * posit with 2 exponent bits.  FP16C and the posits round to the nearest
 * value with ties away from zero and saturate at their largest value. */
typedef enum {
    LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16 = 2, LBM_FP16S = 3, LBM_FP16C = 4,
    LBM_P16_0S = 5, LBM_P16_1S = 6, LBM_P16_2C = 7
} lbm_storage;

/* Arithmetic precision.  LBM_ARITH_FP64 requires FP64 or FP32 storage. */
typedef enum { LBM_ARITH_FP32 = 0, LBM_ARITH_FP64 = 1 } lbm_arith;

/* Cell flags (one byte per cell). */
#define LBM_FLAG_SOLID  1u   /* bounce-back wall cell; never updated */
#define LBM_FLAG_EQ     2u   /* held at the equilibrium of eq_rho, eq_u */
#define LBM_FLAG_MOVING 4u   /* with SOLID: wall moving with wall_u */

typedef struct {
    int32_t nx, ny, nz;      /* cells per axis in [1, 65535]; N = nx*ny*nz with
                                N < 2^31 and N * bytes per DDF < 2^32 */
    int32_t q;               /* lbm_velset */
    int32_t collision;       /* lbm_collision */
    int32_t storage;         /* lbm_storage */
    int32_t arith;           /* lbm_arith */
    int32_t unshifted;       /* 0: DDFs stored shifted, f_i - w_i (Sec. 2.2, the
                                default); 1: ablation storing f_i itself */
    double tau;              /* relaxation time, > 0.5 (nu = (tau - 1/2)/3) */
    double trt_magic;        /* TRT Lambda = (tau - 1/2)(tau_minus - 1/2); 0.25 */
    double force[3];         /* Guo body force per volume (lattice units) */
    double wall_u[3];        /* velocity of MOVING wall cells (wall density 1) */
    double eq_rho;           /* density of EQ cells */
    double eq_u[3];          /* velocity of EQ cells */
} lbm_params;

/* FP64 diagnostics of one lattice, summed over fluid cells (neither SOLID
 * nor EQ) in a fixed order, so repeated calls give identical results.  The
 * sums are the discrete sums of the paper's diagnostics: the kinetic energy
 * of the Taylor-Green runs (Sec. 4.2) and the velocity error norm of the
 * Poiseuille runs (Sec. 4.1); mass and momentum are what the collision
 * conserves (appendix "LBM equations in a nutshell"). */
typedef struct {
    double mass;             /* sum of rho */
    double momentum[3];      /* sum of rho u */
    double kinetic_energy;   /* sum of rho |u|^2 / 2 */
    double u_max;            /* max |u| */
    double l2_error;         /* sqrt(sum |u - u_ref|^2 / sum |u_ref|^2); -1 without u_ref */
    double force_on_solid[3];/* momentum exchange into SOLID cells, this time step */
    int64_t nonfinite_cells; /* fluid cells with non-finite rho or u (decoded state) */
    int64_t step;            /* time steps taken since the last initialisation */
    int64_t nonfinite_updates; /* cell updates since the last initialisation whose
                                  density or velocity before the velocity clamp was
                                  not finite, counted by the step before encoding:
                                  the only sign of a blow-up in FP16C and the
                                  posits, which have no NaN or Inf and saturate */
} lbm_diag;

/* How lbm_step launches the stream-collide kernel. */
/* PER_LATTICE: one launch per lattice per step over row tiles.  BATCHED:
 * one launch per step over a table of row tiles (block * cells_per_lane cells
 * of one row) of every lattice.  DENSE: one launch per step over tiles of
 * `block` consecutive cells in index order, which may span rows, so short
 * rows leave no lanes idle (one cell per lane). */
typedef enum { LBM_LAUNCH_PER_LATTICE = 0, LBM_LAUNCH_BATCHED = 1, LBM_LAUNCH_DENSE = 2 } lbm_launch_mode;
typedef struct {
    int32_t mode;            /* lbm_launch_mode */
    int32_t block;           /* threads per workgroup: 64, 128, 256, 512 */
    int32_t cells_per_lane;  /* consecutive x cells per thread: 1, 2 (not FP64
                                storage) or 4 (16-bit storage); every nx must
                                be a multiple of it */
    int32_t persistent;      /* BATCHED/DENSE: workgroups per CU of a persistent
                                grid walking the tile table; 0 = one workgroup
                                per tile */
    int32_t graph_steps;     /* > 0 (even): lbm_step replays a HIP graph of
                                this many steps (needs a non-null stream);
                                0 = direct launches */
} lbm_launch;

typedef struct {
    int64_t cells;           /* total cells of all lattices */
    int64_t device_bytes;    /* device memory held by the handle */
    int32_t n_lattices;
    int32_t bytes_per_ddf;   /* 8, 4 or 2 */
    int64_t step;
} lbm_info;

typedef void* (*lbm_alloc_fn)(size_t bytes, void* ctx);
typedef void (*lbm_free_fn)(void* ptr, void* ctx);

/* Create n_lattices >= 1 lattices described by params[0..n_lattices-1]: the
 * state of the paper's kernels (two DDF buffers for the one-step pull
 * scheme, Sec. 5 and Table 3; a flag byte per cell).
 * All must share q, collision, storage and arith (else LBM_EUNSUPPORTED).
 * stream: a hipStream_t, or NULL for the null stream.  alloc/free_: optional
 * device allocator (both or neither); alloc_ctx is passed back to them.
 * Every cell starts as fluid at rest (rho = 1, u = 0).
 * Errors: LBM_EINVAL for tau <= 0.5, sizes out of range, unshifted not 0/1
 * or unknown enums; LBM_ENOMEM; LBM_EDEVICE. */
lbm_status lbm_create(const lbm_params* params, int32_t n_lattices, void* stream,
                      lbm_alloc_fn alloc, lbm_free_fn free_, void* alloc_ctx,
                      lbm_handle** out);

/* Set the cell flags of one lattice from host uint8[N] (bits LBM_FLAG_*;
 * MOVING without SOLID, and EQ with SOLID, are LBM_EINVAL), then
 * re-initialise that lattice to rest with EQ cells at their equilibrium.
 * Wall cells hold zero DDFs.  The flags are what the paper's kernel reads
 * per cell and per neighbour (its flag checks before streaming); the
 * near-wall marks and masks the step uses are derived from them here, on
 * the device.  Synchronises.  Errors: LBM_EINVAL (NULL handle or flags,
 * lattice out of range, bad flag bits), LBM_ENOMEM (staging buffer),
 * LBM_EDEVICE. */
lbm_status lbm_set_boundaries(lbm_handle* h, int32_t lattice, const uint8_t* flags);

/* Initialise one lattice's DDFs to the equilibrium of host fields rho[N] and
 * u[3*N] (either may be NULL: rho = 1, u = 0), stored in the lattice's
 * format (the paper's initialize kernel).  EQ cells take eq_rho/eq_u, SOLID
 * cells zero.  Resets the step counter of the handle. */
lbm_status lbm_set_rho_u(lbm_handle* h, int32_t lattice, const double* rho, const double* u);

/* Advance every lattice by n_steps >= 0 time steps of the fused pull
 * stream-collide update (the appendix "LBM equations in a nutshell", with
 * DDF shifting of Sec. 2.2), alternating the two DDF buffers.  Asynchronous.
 * Errors: LBM_EINVAL (NULL handle, n_steps < 0), LBM_EDEVICE (a launch or
 * the graph capture failed; steps already enqueued stay enqueued). */
lbm_status lbm_step(lbm_handle* h, int64_t n_steps);

/* Density and velocity of the current state: the sums the paper's fields()
 * takes (Sec. 2.2: density with the 1 of the shift added last, velocity by
 * alternating pair sums), over what the next step sees after streaming;
 * velocity includes half the body force, not clamped.  SOLID
 * cells report rho = 1 and the wall velocity, EQ cells their own moments.
 * rho: host double[N] or NULL; u: host double[3*N] or NULL.  Synchronises.
 * Errors: LBM_EINVAL (NULL handle, lattice out of range), LBM_ENOMEM
 * (device scratch of 4*N doubles), LBM_EDEVICE. */
lbm_status lbm_get_rho_u(lbm_handle* h, int32_t lattice, double* rho, double* u);

/* Raw DDF codes of the current state: host buffer of q*N elements of the
 * storage type (double, float or uint16), direction-major [i*N + n].
 * set: copies in, to both DDF buffers (used for checkpoints and exact
 * comparisons); get: copies out.  Both synchronise.  Every step writes the
 * code of +0 into SOLID cells and the stored equilibrium of eq_rho/eq_u
 * into EQ cells (what lbm_set_rho_u puts there), so codes set into those
 * cells other than these last until the next step: EQ codes are streamed
 * to the neighbours once, SOLID codes are never read. */
/* Errors: LBM_EINVAL (NULL handle or host, lattice out of range),
 * LBM_EDEVICE. */
lbm_status lbm_set_ddf(lbm_handle* h, int32_t lattice, const void* host);
lbm_status lbm_get_ddf(lbm_handle* h, int32_t lattice, void* host);

/* FP64 diagnostics of one lattice (see lbm_diag: the kinetic-energy sum of
 * Sec. 4.2, the error norm of Sec. 4.1, conserved sums, momentum-exchange
 * force).  u_ref: NULL or host double[3*N] for the L2 error.  Fills *out;
 * returns LBM_ENONFINITE (after filling) if out->nonfinite_cells > 0 or
 * out->nonfinite_updates > 0.  Synchronises.  Other errors: LBM_EINVAL
 * (NULL handle or out, lattice out of range), LBM_ENOMEM (device copy of
 * u_ref), LBM_EDEVICE. */
lbm_status lbm_diagnostics(lbm_handle* h, int32_t lattice, const double* u_ref, lbm_diag* out);

/* One time step fused with the diagnostics of the state it reads (the
 * paper's runs sample the kinetic energy of Sec. 4.2 or the drag and lift of
 * Sec. 4.3 every few steps): the step's kernel pulls each cell once for both,
 * so a diagnostic step costs little more than a plain one.  *out is
 * bit-identical to lbm_diagnostics called before the step (out->step is the
 * step number of that state), the DDFs written to a plain lbm_step; the
 * handle has advanced one step on return, and out->nonfinite_updates
 * includes the step just taken.  u_ref_dev: NULL or a DEVICE array of 3*N
 * doubles laid out as lbm_diagnostics' u_ref (owned by the caller).  Runs
 * with workgroups of 512 threads whatever the launch configuration, outside
 * any captured graph.  Allocates nothing.  Synchronises.  Returns
 * LBM_ENONFINITE (after filling *out and stepping) like lbm_diagnostics.
 * Errors: LBM_EINVAL (NULL handle or out), LBM_EUNSUPPORTED (a handle of
 * more than one lattice), LBM_EDEVICE. */
lbm_status lbm_step_diagnostics(lbm_handle* h, const double* u_ref_dev, lbm_diag* out);

/* For callers that cannot allocate device memory (code around a HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * diagnostics of lbm_diagnostics without any allocation.  u_ref_dev: NULL
 * or a DEVICE array of 3*N doubles laid out as lbm_diagnostics' u_ref (owned
 * by the caller).  The reduction's partial sums and results go to a static
 * device array of the library (32 MiB per GPU, held until the process ends)
 * instead of memory of the handle: 12 doubles per row tile of up to 512
 * cells (ny * nz * ceil(nx / 512) tiles) plus 513 * 12 doubles, so lattices
 * of up to about 349,000 row tiles (a 512^3 lattice has 262,144); a larger
 * lattice is refused with LBM_EINVAL and a message giving both sizes.
 * Every call on one GPU shares the array and leaves its contents there, so
 * calls that overlap on one GPU (from other threads, or on other streams)
 * race and must be serialised by the caller.  Results are bit-identical to
 * lbm_diagnostics with the same reference field.  Synchronises.  Errors:
 * as lbm_diagnostics (LBM_ENONFINITE after filling *out). */
lbm_status lbm_diagnostics_noalloc(lbm_handle* h, int32_t lattice, const double* u_ref_dev, lbm_diag* out);

/* Launch configuration (see lbm_launch); invalid values are LBM_EINVAL and
 * leave the current configuration in place.  Setting one drops a captured
 * graph (it is captured again at the next lbm_step).  If the batched tile
 * table cannot be built (LBM_ENOMEM, LBM_EDEVICE) the previous configuration
 * is restored; should that fail too, lbm_step returns LBM_EINVAL for batched
 * launches until a configuration is set successfully. */
lbm_status lbm_set_launch(lbm_handle* h, const lbm_launch* cfg);
lbm_status lbm_get_launch(lbm_handle* h, lbm_launch* cfg);

/* Time every launch configuration on the handle's own lattices (one warm-up
 * launch, then the better of two runs of trial_steps launches, each reading
 * the current state and writing the other buffer, so the state is left
 * unchanged), keep the fastest (ties within 0.5 % go to the candidate tried
 * first, the smaller workgroup) and return it (best may be NULL).  The graph
 * setting of the current configuration is kept; candidates the handle's
 * lattices do not admit are skipped.  Errors: LBM_EINVAL (NULL handle,
 * trial_steps < 1), LBM_EDEVICE (a trial launch failed; the previous
 * configuration is restored). */
lbm_status lbm_autotune(lbm_handle* h, int32_t trial_steps, lbm_launch* best);

/* Sizes, device memory and step counter of a handle.  LBM_EINVAL for NULL. */
lbm_status lbm_info_get(lbm_handle* h, lbm_info* out);
/* Wait for all work enqueued on the handle's stream.  LBM_EINVAL for NULL,
 * LBM_EDEVICE if the stream reports an error. */
lbm_status lbm_synchronize(lbm_handle* h);
/* Wait for the handle's stream, then free everything it holds (NULL: no-op). */
void lbm_destroy(lbm_handle* h);
/* Message of the last failure in the calling thread; never NULL (empty
 * before any failure); valid until that thread's next library call. */
const char* lbm_last_error(void);

/* Storage codecs on device arrays (Sec. 3): encode n floats into n codes of
 * a 16-bit format, or decode n codes into floats.  d_in/d_out: device
 * pointers; stream: hipStream_t or NULL.  Asynchronous.  LBM_EINVAL for a
 * non-16-bit format or n < 0. */
lbm_status lbm_encode(int32_t storage, const float* d_in, uint16_t* d_out, int64_t n, void* stream);
lbm_status lbm_decode(int32_t storage, const uint16_t* d_in, float* d_out, int64_t n, void* stream);

/* Plain device copy of `bytes` bytes (multiple of 16, 16-byte aligned
 * pointers): the reference kernel for calibrating memory-traffic counters
 * and achievable HBM bandwidth.  Asynchronous. */
lbm_status lbm_copy_probe(const void* d_src, void* d_dst, size_t bytes, void* stream);

/* Memory microbenchmarks of the paper's appendix (its memory benchmarks,
 * Fig. 13, and the coalesced/misaligned read/write columns of Table 5): one
 * kernel of the given kind over device buffers, one 4-byte element per
 * thread (as a stream-collide kernel accesses DDFs).  Coalesced: element i at
 * i; misaligned: at i + 1, so each wavefront's accesses straddle cache lines
 * as the x-shifted pull reads do.  READ kinds read bytes/4 (- 1) elements of
 * d_src and use d_dst (also `bytes` long) as a sink that is written only in
 * the case, which the caller avoids, that the xor of a thread's elements is
 * 0x9E3779B9 (all-zero sources are safe); WRITE kinds write
 * d_dst[i (+ 1)] = i; COPY is lbm_copy_probe.  Bytes moved: the elements read
 * or written (both for COPY).  Asynchronous.  LBM_EINVAL for an unknown kind,
 * NULL or misaligned pointers, or sizes below 8 or not a multiple of 4. */
typedef enum {
    LBM_PROBE_COPY = 0, LBM_PROBE_READ = 1, LBM_PROBE_READ_MISALIGNED = 2,
    LBM_PROBE_WRITE = 3, LBM_PROBE_WRITE_MISALIGNED = 4
} lbm_probe_kind;
lbm_status lbm_memory_probe(int32_t kind, const void* d_src, void* d_dst, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
