/*
 * lbm.h -- C ABI of the MI355X lattice Boltzmann library (liblbm.so).
 *
 * The library advances a distribution f_i(x, t) on a periodic D-dimensional
 * lattice with the lattice Boltzmann equation in lattice units (dx = dt = 1):
 *
 *     f_i(x + c_i, t + 1) = f^eq_i(x, t) + (1 - 1/tau) fhat^neq_i(x, t)
 *
 * (eq. lbe in the introduction, in its regularised form eq. lbe-reg), where
 * the equilibrium is the Hermite expansion eq. hermite and the filtered
 * non-equilibrium part is the Galilean-invariant expansion eq. hermite-coll,
 * both truncated at Hermite order K (default: 3 on D2Q9, D3Q15 and D3Q19,
 * whose isotropy order is 2N = 4, giving eq. filter-1st; 4 on D3Q39, 2N = 6,
 * giving eq. filter-2nd).  rho and u are the zeroth and first moments (eq. mme) and
 * Pi^neq the non-equilibrium momentum flux (eq. coeff-2 / eq. Pi_def).
 *
 * Conventions for every call:
 *   - Return value: lbm_status; LBM_OK (0) on success, a negative code on
 *     failure.  No C++ exception crosses the ABI.  lbm_last_error() gives a
 *     thread-local message for the most recent failure on that thread.
 *   - Arguments are validated on the host before any device work, so a call
 *     that returns LBM_EINVAL or LBM_ESTATE has changed nothing.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Field layout: rho is [nz][ny][nx] (x fastest) float64; u is
 *     [D][nz][ny][nx] float64 (component-major).  A batch concatenates its
 *     boxes in creation order, each in that layout (rho: all boxes' sites;
 *     u: component a of every box is the a-th block of total-site length).
 *   - Device work runs on the handle's stream (lbm_set_stream); calls that
 *     return host data synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx* lbm_t;

/* Velocity sets.  D2Q9, D3Q15 and D3Q19: T0 = 1/3, 2N = 4.  D3Q39: T0 = 2/3,
 * 2N = 6 (eq. iso and the lattice catalogue that follows it). */
typedef enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1, LBM_D3Q39 = 2, LBM_D3Q15 = 3 } lbm_lattice;

/* Storage type of the populations.  Every type stores S (f_i - w_i): the
 * deviation from the rest weights in units of the weight quantum 1/S (S = 36
 * for D2Q9 and D3Q19, 72 for D3Q15, 6480 for D3Q39), so every weight is the
 * exact integer S w_i.  Arithmetic: FP64 computes in double; FP32, FP16 and
 * BF16 compute in float. */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16 = 2, LBM_BF16 = 3 } lbm_dtype;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,   /* bad argument (tau <= 1/2, bad dims, unknown enum, NULL pointer, ...) */
    LBM_ENOMEM = -2,   /* device or host allocation failed */
    LBM_EDEVICE = -3,  /* a HIP runtime call or kernel launch failed */
    LBM_ENODEV = -4,   /* no usable GPU */
    LBM_ESTATE = -5,   /* call not valid in the current state (e.g. step before init) */
    LBM_ENUMERIC = -6  /* non-finite or non-positive density found by lbm_totals */
} lbm_status;

/* Collision operators (lbm_set_collision). */
typedef enum {
    LBM_COLLISION_FILTERED = 0,  /* eq. post-1 with the truncated eq. hermite-coll (the default) */
    LBM_COLLISION_BGK = 1        /* eq. BGK, f' = f - (f - f^eq)/tau, with the same truncated f^eq */
} lbm_collision;

/* Step-kernel variants for a single box (lbm_set_kernel). */
typedef enum {
    LBM_KERNEL_AUTO = 0,      /* the scalar step unless a tuned choice was set */
    LBM_KERNEL_SCALAR = 1,    /* one site per thread, 4/8-byte accesses */
    LBM_KERNEL_ROW_WAVE = 2,  /* V sites per lane, 8/16-byte accesses, x-neighbours by lane shuffle */
    LBM_KERNEL_IN_PLACE = 3,  /* one site per thread on one buffer: each step reads and writes the same
                                 elements, alternating between two layouts of the state (bit-identical
                                 results, half the memory) */
    LBM_KERNEL_TWO_ROW = 4,   /* two sites per thread (rows 2j and 2j+1, ny even): the second site's loads
                                 are in flight while the first collides (bit-identical results) */
    LBM_KERNEL_TWIST = 5,     /* in place on one buffer with the twisted layouts: every step reads and
                                 writes each element once, only at the cells x + b (b the positive part
                                 of a velocity), so it touches fewer row tiles (bit-identical results,
                                 half the memory) */
    LBM_KERNEL_TWO_STEP = 6   /* two steps per launch (D3Q15, D3Q19): a block walks a column of the box
                                 in z, takes the first step on the column and a one-site ring around it
                                 and keeps that state in LDS for the second, so the state is read and
                                 written once per two steps (bit-identical results) */
} lbm_kernel;

typedef struct {
    int32_t lattice, dtype;
    int32_t D, Q, two_n, K;      /* dimension, velocities, isotropy order, Hermite truncation */
    double T0;                   /* lattice temperature c_s^2 */
    int32_t nbox;                /* 1 for a single box */
    int64_t dims[3];             /* box 0 (nx, ny, nz) */
    int64_t nsites;              /* total sites over all boxes */
    int64_t t;                   /* steps taken since lbm_init */
    int64_t bytes_per_site_update; /* 2 * Q * sizeof(storage): one read + one write per population */
    uint64_t state_bytes;        /* bytes of one population buffer (see lbm_state_bytes) */
    int32_t block, grid;         /* launch shape in use (threads per block; batched grid size, 0 = one wave per
                                    tile; for LBM_KERNEL_TWO_STEP its number of blocks) */
    int32_t graph_chunk;         /* steps per captured graph */
    int32_t kernel;              /* step kernel in use (lbm_kernel, never AUTO) */
    int32_t collision;           /* lbm_collision in use */
    double theta;                /* weight of the energy-flux term (0: none) */
} lbm_info;

/* Create a single periodic box (eq. lbe on an nx*ny*nz torus).
 * dims = {nx, ny, nz}, each >= 1; D2Q9 requires nz == 1.  ny and nz at most
 * 65535 with ny * nz below 2^31; one population row (nx times the storage
 * bytes) below 2 GiB; at most 2^36 sites in total (memory is the practical
 * limit: a D3Q19 FP16 box of 2^32 sites takes 163 GB with the in-place
 * step); in a batch every box holds less than 2 GiB of populations and has nx
 * at most 2^21.
 * tau: relaxation time, finite and > 1/2 (viscosity T0 (tau - 1/2)).  No
 * device memory for the populations is allocated until lbm_init /
 * lbm_set_state, unless bound with lbm_bind_state.  Errors: LBM_EINVAL,
 * LBM_ENODEV, LBM_EDEVICE, LBM_ENOMEM. */
lbm_status lbm_create(lbm_t* out, int32_t lattice, const int64_t dims[3], double tau, int32_t dtype);

/* Create nbox independent periodic boxes advanced together by one launch per
 * step.  dims: nbox * 3 int64 (nx, ny, nz per box); tau: nbox doubles.  Same
 * rules per box as lbm_create.  Boxes are stored back to back, in order. */
lbm_status lbm_create_batch(lbm_t* out, int32_t lattice, int32_t nbox, const int64_t* dims,
                            const double* tau, int32_t dtype);

/* Hermite truncation order K of both expansions, 2 <= K <= 2N - 1 (the
 * truncation rule after eq. hermite-coll).  K = 2 is the zero-velocity filter
 * eq. filter-Pi with the second-order equilibrium.  With BGK, K is the order
 * of the equilibrium.  K = 2 is rejected while an energy-flux weight theta != 0
 * is set.  Only before lbm_init. */
lbm_status lbm_set_hermite_order(lbm_t h, int32_t K);

/* Collision operator and the weight theta of the energy-flux term (eq. pq,
 * Discussion section).  collision: LBM_COLLISION_FILTERED (default) or
 * LBM_COLLISION_BGK.  theta != 0 adds theta times the energy-flux part to the
 * filtered non-equilibrium part: the compact form eq. filter-Q, with f^eq / rho
 * so that it reduces to the theta term of eq. filter2 at u = 0, expanded in
 * Hermite tensors and truncated at the same order K, built on the relative
 * non-equilibrium energy flux eq. Q_def.  It needs the filtered operator and
 * K >= 3 (its series starts at the third order).  theta must be finite.
 * Errors: LBM_EINVAL (unknown collision, theta not finite, theta != 0 with BGK
 * or with K = 2), LBM_ESTATE after lbm_init. */
lbm_status lbm_set_collision(lbm_t h, int32_t collision, double theta);

/* Run device work on `hip_stream` (a hipStream_t; NULL = the null stream).
 * The caller keeps ownership of the stream; it must outlive the handle's use. */
lbm_status lbm_set_stream(lbm_t h, void* hip_stream);

/* Bytes needed for one population buffer: Q * nstored stored values, rounded
 * up to a multiple of 256.  Layout (blocked structure of arrays): the local
 * sites l = (z * ny + y) * nx + x of a box are cut into blocks of w
 * consecutive sites, and block l / w holds Q runs of w values, population i of
 * site l at element l / w * Q * w + m(i) * w + l % w from the box's first
 * element, where the tile row m(i) is the rank of c_i in the order of
 * increasing (c_z, c_y, c_x) and i the order of lbm_lattice_table.
 *   - A single box: w = nx (each x-row is one block, "row tiles"), and
 *     nstored = nx * ny * nz.
 *   - A batch: w = 64, and each box is padded to a whole number of blocks
 *     (n_b rounded up to a multiple of 64); box b starts at element Q P_b,
 *     P_b the padded site count of the boxes before it.  The padding is zero
 *     after lbm_init and lbm_set_state and never read or written by a step. */
lbm_status lbm_state_bytes(lbm_t h, size_t* bytes_each);

/* Use caller-owned device memory (e.g. two torch tensors) for the two
 * population buffers instead of library allocations.  Each must hold at least
 * lbm_state_bytes() bytes, be 256-byte aligned, live on the handle's device and
 * outlive the handle.  Only before lbm_init / lbm_set_state. */
lbm_status lbm_bind_state(lbm_t h, void* buf_a, void* buf_b, size_t bytes_each);

/* f := f^eq_K(rho, u) at every site (eq. hermite), t := 0.  rho and u are
 * float64 in the field layout above; on_device != 0 means they are device
 * pointers, else host pointers (copied, then released).  Borrowed for the
 * call only; synchronises the stream. */
lbm_status lbm_init(lbm_t h, const double* rho, const double* u, int32_t on_device);

/* Advance n >= 0 steps of eq. lbe-reg: per site pull f_i from x - c_i
 * (periodic), collide, store.  Asynchronous on the handle's stream; long runs
 * are issued as captured graphs of graph_chunk steps.  LBM_ESTATE before init. */
lbm_status lbm_step(lbm_t h, int64_t n);

/* Build (or rebuild) the captured step graphs now, so that a later lbm_step
 * does not pay for graph instantiation.  Optional. */
lbm_status lbm_prepare(lbm_t h);

/* Steps per captured graph, 1 to 4096 (default 32; else LBM_EINVAL).  Takes
 * effect at the next lbm_step / lbm_prepare. */
lbm_status lbm_set_graph_chunk(lbm_t h, int32_t steps);

/* Launch shape: threads per block (64, 128 or 256; 0 = default) and,
 * for batches, the number of blocks of the persistent step kernel (0 = enough
 * blocks for every tile to get its own wave; a batch tile is one wave's work:
 * one 64-site block of a box's layout).  For a single box the grid is the
 * number of blocks of LBM_KERNEL_TWO_STEP (0 = one per compute unit; its
 * blocks have a fixed size).  Only before lbm_init. */
lbm_status lbm_set_launch(lbm_t h, int32_t block, int32_t grid);

/* Choose the single-box step kernel.  All variants compute the same bits.
 * LBM_KERNEL_ROW_WAVE needs nx to be a multiple of the sites per lane V (4 for
 * FP32/FP16/BF16, 2 for FP64) with nx / V <= 64, and V above the largest
 * velocity component (so FP64 D3Q39 has none); else LBM_EINVAL.
 * LBM_KERNEL_IN_PLACE steps the state inside one buffer: with library-owned
 * memory only one population buffer is allocated, so a box of twice the size
 * fits.  After an odd number of its steps the state is kept in a swapped
 * layout (population i of site x at site x + c_i, tile row m(opp(i))); the
 * moments, totals and residual read it as it is, and lbm_get_state returns the
 * natural layout (rearranged on the host).  Switching kernels later (lbm_tune)
 * allocates the second buffer.  Batches always use the batched kernel (one
 * wave per 64-site block); for them LBM_KERNEL_AUTO and LBM_KERNEL_SCALAR are
 * accepted and the other variants are LBM_EINVAL.
 * LBM_KERNEL_TWIST (single box) also steps inside one buffer.  The state is
 * kept in twisted layouts: population i of site x sits at site x + b_i, b_i
 * the positive part of c_i component by component, in tile row m(i) after an
 * even number of its steps and m(opp(i)) after an odd number.  lbm_init and
 * lbm_set_state write that layout; the readers and lbm_get_state handle it as
 * they handle the swapped one.
 * LBM_KERNEL_TWO_ROW needs a single box with ny even (else LBM_EINVAL).
 * LBM_KERNEL_TWO_STEP needs a single D3Q15 or D3Q19 box with nx a multiple of
 * 64, ny a multiple of 8 (4 for FP64 storage) and one z-plane of populations
 * (Q nx ny values) below 2 GiB, else LBM_EINVAL.  An odd step count ends with
 * one step of the scalar kernel; the state stays in the natural layout.
 * May be called at any time: on an initialised handle the state is first
 * brought to the natural layout and then into the new kernel's starting
 * layout (which may allocate the second buffer), and the run continues bit
 * for bit. */
lbm_status lbm_set_kernel(lbm_t h, int32_t kernel);

/* Autotune the step's launch: time every candidate over `steps` steps with HIP
 * events, in three interleaved rounds, and keep the candidate with the fastest
 * round.  Single box: the scalar step at 64/128/256 threads per block, the
 * in-place, twist and two-row (ny even) steps at 256, the scalar, in-place
 * and twist steps at one whole x-row per block when nx rounds up to 192 lanes,
 * the row-wave step where it applies, and the two-step kernel (where it
 * applies) at one and at two blocks per compute unit.  Batch: 64/128/256 threads per block, with
 * one wave per 64-site block of the layout or 1024/2048/4096 persistent
 * blocks.  The state is saved before and restored after, so t and the
 * populations are unchanged (all candidates compute the same bits).  Choices are appended to the text file `cache_path` (NULL: the
 * path in the environment variable LBM_TUNE_CACHE, or no cache); a later call
 * with the same lattice, dtype, K, collision kind and geometry reuses the
 * cached choice without timing.  Needs an initialised handle (LBM_ESTATE
 * otherwise); allocates one state-sized scratch buffer while timing. */
lbm_status lbm_tune(lbm_t h, int32_t steps, const char* cache_path);

/* rho and u (eq. mme) of the current state, in float64, in the field layout
 * above.  on_device: as for lbm_init.  Synchronises. */
lbm_status lbm_moments(lbm_t h, double* rho, double* u, int32_t on_device);

/* Global totals per box, float64, computed on the GPU with a fixed reduction
 * order: out[4*b + 0] = sum rho, out[4*b + 1 + a] = sum rho u_a (a < 3; 0 for
 * a >= D).  out has 4 * nbox doubles on the host.  Returns LBM_ENUMERIC when a
 * total is not finite or a box's mass is not positive.  Synchronises. */
lbm_status lbm_totals(lbm_t h, double* out);

/* Error residuals of the current state against reference fields (same layout
 * as lbm_moments), in float64 on the GPU: out = {max |du|, sqrt(sum |du|^2),
 * max |drho|, sqrt(sum drho^2)} over all sites and components.
 * on_device: as for lbm_init.  Synchronises. */
lbm_status lbm_residual(lbm_t h, const double* rho_ref, const double* u_ref, int32_t on_device,
                        double out[4]);

/* lbm_residual for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * calls no hipMalloc, hipFree or other allocating routine and does not
 * synchronise: the two residual kernels are enqueued on the handle's stream.
 * rho_ref and u_ref are device pointers (layout as for lbm_moments); out is a
 * device pointer to 4 doubles that receives {max |du|, sqrt(sum |du|^2),
 * max |drho|, sqrt(sum drho^2)}, the values lbm_residual returns (the square
 * roots taken on the GPU), valid once the stream reaches that point.
 * The per-chunk partial sums live in a 2 MiB array that the library holds on
 * each GPU until the process ends, so a handle of at most 65536 reduction
 * chunks of 4096 sites is accepted (2^28 sites in one box); larger handles get
 * LBM_EINVAL.  All calls on one GPU share that array: calls that overlap on
 * one GPU (two streams, two threads) race and give wrong results. */
lbm_status lbm_residual_noalloc(lbm_t h, const double* rho_ref, const double* u_ref, double* out);

/* Checkpoint: bytes needed by lbm_get_state (a header plus the raw stored
 * populations, Q * nstored values, padding included). */
lbm_status lbm_checkpoint_bytes(lbm_t h, size_t* bytes);

/* Copy the state to host memory `buf` of at least lbm_checkpoint_bytes(): a
 * 64-byte header (lattice, dtype, K, geometry hash, t) followed by the stored
 * values S (f_i - w_i) in the layout described at lbm_state_bytes (S = 36 for
 * D2Q9 and D3Q19, 72 for D3Q15, 6480 for D3Q39). */
lbm_status lbm_get_state(lbm_t h, void* buf, size_t bytes);

/* Restore a state written by lbm_get_state on a handle of the same lattice,
 * dtype, K and geometry.  The next steps reproduce the original run bit for
 * bit when the handle also has the same collision operator and theta (these
 * are not recorded: the populations are valid input to any operator). */
lbm_status lbm_set_state(lbm_t h, const void* buf, size_t bytes);

/* Describe the handle. */
lbm_status lbm_get_info(lbm_t h, lbm_info* info);

/* Wait for all work issued on the handle's stream. */
lbm_status lbm_sync(lbm_t h);

/* Free the handle and every library-owned allocation; caller-bound buffers are
 * left alone.  NULL is accepted. */
lbm_status lbm_destroy(lbm_t h);

/* Thread-local message for the last failed call on this thread ("" if none). */
const char* lbm_last_error(void);

/* The library's copy of a lattice: D, Q, T0, 2N, c (Q*3 int32, z = 0 in 2-D)
 * and w (Q doubles).  Any output pointer may be NULL.  Host only. */
lbm_status lbm_lattice_table(int32_t lattice, int32_t* D, int32_t* Q, double* T0, int32_t* two_n,
                             int32_t* c, double* w);

/* Measurement aid: stream `bytes` (a multiple of 16) from device buffer src to
 * device buffer dst `reps` times with a plain vectorised copy kernel on
 * `hip_stream`, and return the mean milliseconds per copy from HIP events.
 * Used to calibrate traffic counters and the attainable HBM bandwidth. */
lbm_status lbm_copy_probe(void* dst, const void* src, size_t bytes, int32_t reps, void* hip_stream,
                          double* ms_per_copy);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
