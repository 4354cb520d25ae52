/*
 * tof.h -- C ABI of the MI355X (gfx950) gradient engine for finite-difference
 * topology optimization of permanent magnets (Abert et al. 2017).
 *
 * One gradient evaluation takes a density field rho on a regular cuboid-cell
 * grid to
 *   M = chi rho^p M0                       (Sec. Methodology, penalized magnetization)
 *   H = -N (*) M                           (Sec. Discretization, eq. (convolution);
 *                                           N the positive Newell tensor, eq. (demag_tensor))
 *   J(H), g = dJ/dH                        (eq. (objective_function))
 *   A = -N (*) g                           (the same operator, Sec. Methodology: the
 *                                           adjoint problem is a stray-field problem)
 *   dJ/drho = chi p rho^(p-1) M0 . A       (eqs. (dj_drho), (adjoint1); the paper
 *                                           prints a minus sign, the discrete chain
 *                                           rule gives this plus sign)
 * The convolution runs as a zero-padded FFT convolution (padded lengths
 * L >= 2n - 1 per axis, default 2n), as Sec. Discretization prescribes.
 *
 * Conventions for every entry point:
 *  - Arrays are C order [nz][ny][nx] (x fastest); vector fields are
 *    component-major [3][nz][ny][nx] (or [c][...] with c listed components).
 *  - Pointers named *_host are host memory; every other array pointer is
 *    device memory owned by the caller, of the context's dtype (float for
 *    TOF_F32, double for TOF_F64) unless stated otherwise.  J is always a
 *    device double.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Hot
 *    calls only enqueue work on it and return without synchronizing, and
 *    allocate nothing; results are valid once the stream has reached them.
 *  - Every call validates its arguments before any launch and returns a
 *    tof_status; TOF_OK is 0.  On failure tof_last_error(ctx) describes it
 *    (a thread-local message for calls that have no context).  No exception
 *    crosses the ABI.
 *  - A context is not thread-safe; calls that overlap on one context race.
 *    Use one context per stream.
 */
#ifndef TOF_H
#define TOF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tof_ctx tof_ctx;

typedef enum {
    TOF_OK = 0,
    TOF_ERR_INVALID = -1,      /* bad argument (null pointer, bad box, size) */
    TOF_ERR_UNSUPPORTED = -2,  /* valid but not implemented (e.g. padded length with a prime > 7) */
    TOF_ERR_OOM = -3,          /* device allocation failed */
    TOF_ERR_HIP = -4,          /* a HIP runtime call failed */
    TOF_ERR_NUMERIC = -5,      /* a setup self-check failed */
    TOF_ERR_STATE = -6         /* call order: design/objective not set */
} tof_status;

typedef enum { TOF_F32 = 1, TOF_F64 = 2 } tof_dtype;

/* Objective kinds (S = number of sensor cells, t = target, lam = weight). */
typedef enum {
    TOF_J_MEAN_SQ_HZ = 1,        /* J = (1/S) sum_s (Hz_s - t)^2 */
    TOF_J_MEAN_SQ_HZ_GRADXY = 2, /* J = (1/S) sum_s (Hz_s - t)^2 + lam (1/S) sum_s (DxHz_s^2 + DyHz_s^2),
                                    central differences with the cell sizes; the sensor needs
                                    in-grid x and y neighbours */
    TOF_J_MEAN_SQ_H_TARGET = 3,  /* J = (1/S) sum_s |H_s - H*_s|^2, H* given per sensor cell */
    TOF_J_NEG_HALF_HZ2 = 4,      /* J = -1/2 V_cell sum_s Hz_s^2 (the paper's benchmark objective,
                                    Sec. "Validation and Benchmarks") */
    TOF_J_FIELD_GRADIENT = 5     /* J = -1/2 V_cell [sum_s Hz_s^2 + lam sum_q (D_n Hz_q)^2] (the paper's
                                    field and gradient design): s over the sensor (the field
                                    region), q over a one-cell strip outside it on its -x, +x and
                                    -y sides, D_n the forward difference along q's outward
                                    normal, (Hz(q + n) - Hz(q)) / h_n; the strip and its outer
                                    neighbours must be in the grid */
} tof_objective_kind;

/* Grid flags (tof_grid.flags). */
#define TOF_GRID_SELFTEST_PERTURB 1  /* test hook: setup adds 1e-9 to the self term of N_xx before
                                        its trace self-check, which must then fail (TOF_ERR_NUMERIC) */

/* Grid: the FFT box of nx*ny*nz cells of size dx*dy*dz (the regular cuboid
 * grid of Sec. Discretization).  Lx, Ly, Lz are the padded FFT lengths; 0
 * selects 2n, or, when 2n has a prime factor above 7, the smallest even
 * 7-smooth length above 2n.  Explicit lengths must be even, 7-smooth,
 * >= 2n - 1 and <= 1024 (so n <= 512 per axis).
 * validate = 1: every hot call first checks its input arrays for NaN and
 * infinite values on the device, waits for that check and returns
 * TOF_ERR_INVALID (launching nothing else) when it finds one; such calls
 * synchronize their stream, so they cannot be captured into a graph.
 * validate = 0 (the fast path): no check, non-finite inputs propagate. */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    int32_t Lx, Ly, Lz;
    int32_t dtype;          /* tof_dtype */
    int32_t validate;       /* 0 or 1 */
    int32_t flags;          /* TOF_GRID_* bits, normally 0 */
} tof_grid;

/* Half-open cell index box [x0,x1) x [y0,y1) x [z0,z1). */
typedef struct {
    int32_t x0, x1, y0, y1, z0, z1;
} tof_box;

typedef struct {
    int32_t kind;               /* tof_objective_kind */
    tof_box sensor;             /* sensor cells */
    double target;              /* t (kinds 1, 2) */
    double lambda_grad;         /* lam (kinds 2, 5) */
    const double *h_target_host;/* kind 3: H* as [3][sensor cells], C order over the sensor box, host memory */
    const double *h_target_dev; /* kind 3: the same in device memory; give exactly one of the two (else both NULL) */
} tof_objective;

/*
 * tof_create -- validate the grid, pick FFT plans, allocate the workspaces
 * and compute the tensor spectra (setup; allowed to allocate and to block).
 * The demagnetization tensor of Sec. Discretization, eq. (demag_tensor) (a
 * function of the index difference only), is evaluated on the GPU from
 * Newell's closed form in double-double arithmetic, wrapped onto the padded
 * box and transformed in FP64 (the FFT acceleration of the text after that
 * equation); the spectra are stored in the grid's dtype.  Self-checks before
 * the context is returned: the real-space trace, max |tr N(k) - delta_k0| <
 * 1e-12 over all offsets, and spectra that are real to 1e-9 relative.
 * On success *out owns all device memory of the context (tof_ctx_bytes);
 * setup also holds temporaries (about 30 bytes per padded cell) until it
 * returns.  Blocks until setup is done.
 * Errors: TOF_ERR_INVALID (null/empty/oversized grid, non-positive cell,
 * bad validate/flags), TOF_ERR_UNSUPPORTED (explicit L not 7-smooth or too
 * small), TOF_ERR_OOM, TOF_ERR_HIP, TOF_ERR_NUMERIC (a self-check failed).
 */
tof_status tof_create(const tof_grid *grid, void *stream, tof_ctx **out);

/* Release everything the context owns.  NULL is a no-op. */
void tof_destroy(tof_ctx *ctx);

/*
 * tof_set_design -- the design region chi and magnetization M = chi rho^p M0
 * (Sec. Methodology: the penalized magnetization M(rho) = rho^p M0 with M0
 * constant or spatially varying; chi the characteristic function of the
 * design region).
 *  design:   index box of design cells (NULL = whole grid).
 *  mask:     optional device uint8 [nz][ny][nx]; chi = box && mask != 0.
 *  m0_host:  uniform M0 (3 doubles); ignored when m0_field is given.
 *  m0_field: optional device [3][nz][ny][nx] of the dtype: spatially varying M0.
 *  p:        penalization exponent, 1 <= p <= 16 (integer; rho^p by multiplication).
 * Pointers are borrowed: mask and m0_field must stay valid while used.
 * Errors: TOF_ERR_INVALID.
 */
tof_status tof_set_design(tof_ctx *ctx, const tof_box *design, const uint8_t *mask,
                          const double m0_host[3], const void *m0_field, int32_t p);

/*
 * tof_set_objective -- the objective J(H) of Sec. Methodology,
 * eq. (objective_function), one of the kinds above, and its sensor cells.
 * Copies H* (kind 3) into the context (synchronously).  The context keeps no
 * pointer of `obj`.  Errors: TOF_ERR_INVALID (box outside the grid, missing
 * x/y neighbours for kinds 2 and 5, not exactly one H* for kind 3; the
 * previous objective stays), TOF_ERR_OOM / TOF_ERR_HIP (the context is then
 * left without an objective: hot calls that need one return TOF_ERR_STATE).
 */
tof_status tof_set_objective(tof_ctx *ctx, const tof_objective *obj);

/*
 * tof_field -- H = -N (*) (chi rho^p M0) on the whole grid: the discrete
 * convolution of Sec. Discretization, eq. (convolution), with the tensor of
 * eq. (demag_tensor), computed as a zero-padded FFT convolution (the text
 * after eq. (demag_tensor)); the stray-field operator D of Sec. Methodology.
 *  rho:        device [nz][ny][nx].
 *  H:          device [c][nz][ny][nx], c = number of bits in comps_mask
 *              (bit 0 = Hx, bit 1 = Hy, bit 2 = Hz), in component order.
 * Errors: TOF_ERR_INVALID, TOF_ERR_STATE (no design), TOF_ERR_HIP.
 */
tof_status tof_field(tof_ctx *ctx, const void *rho, void *H, int32_t comps_mask, void *stream);

/*
 * tof_objective_and_grad -- one gradient evaluation of Sec. Methodology:
 * J^(rho) = J(H(rho), rho) (eq. (objective_function)) and its derivative
 * through the adjoint problem (eqs. (dj_drho), (adjoint1), (adjoint2)),
 * solved with the same stray-field operator as the forward problem:
 * forward field on the cells J reads, J (FP64, fixed-order reduction),
 * g = dJ/dH, the adjoint field A = -N (*) g on the design cells,
 * dJ/drho = chi p rho^(p-1) M0 . A.
 *  rho:  device [nz][ny][nx].
 *  J:    device double[1] (may be NULL).
 *  grad: device [nz][ny][nx]; zero outside the design region.
 * Errors: TOF_ERR_INVALID, TOF_ERR_STATE, TOF_ERR_HIP.
 */
tof_status tof_objective_and_grad(tof_ctx *ctx, const void *rho, double *J, void *grad,
                                  void *stream);

/*
 * tof_adjoint -- vector-Jacobian product of tof_field (the adjoint solve of
 * Sec. Methodology with a given dL/dH in place of dJ/dH): given any gH =
 * dL/dH as device [3][nz][ny][nx], writes dL/drho = chi p rho^(p-1) M0 .
 * (-N (*) gH) to grad [nz][ny][nx] (zero outside the design region).
 * Errors: TOF_ERR_INVALID, TOF_ERR_STATE, TOF_ERR_HIP.
 */
tof_status tof_adjoint(tof_ctx *ctx, const void *rho, const void *gH, void *grad, void *stream);

/*
 * tof_project_step -- one projected-gradient update that keeps rho in the
 * bounds 0 <= rho <= 1 of Sec. Methodology (the paper minimizes with a
 * bound-constrained quasi-Newton method, Sec. Discretization; this is the
 * simplest such step): on the design cells chi (box and mask),
 * rho <- clamp(rho - alpha grad / G, 0, 1), G = max over chi of |grad|;
 * other cells are left unchanged; G = 0 leaves rho unchanged.
 * rho (updated in place), grad: device [nz][ny][nx]; alpha >= 0.
 * Errors: TOF_ERR_INVALID, TOF_ERR_STATE, TOF_ERR_HIP.
 */
tof_status tof_project_step(tof_ctx *ctx, void *rho, const void *grad, double alpha, void *stream);

/*
 * tof_project_step_static -- tof_project_step without a context, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): it allocates nothing and
 * launches the same two kernels.  Their scratch (the partial maxima of the
 * first launch, at most 2048 doubles = 16 KiB) is a static device array of
 * the library, one per GPU, held until the process ends; every entry the
 * second launch reads is written by the first, so nothing needs clearing.
 * All calls on one GPU share that array: calls that overlap on one GPU (other
 * streams, other threads) race; serialize them.
 *  grid:   only nx, ny, nz (each in [1, 512]) and dtype are read.
 *  design: index box of design cells (NULL = whole grid); mask: optional
 *          device uint8 [nz][ny][nx], chi = box && mask != 0.
 *  rho (updated in place), grad: device [nz][ny][nx] of the dtype; alpha >= 0.
 * Same update as tof_project_step.  Errors: TOF_ERR_INVALID (null pointers,
 * sizes beyond 512 per axis, bad box or alpha), TOF_ERR_HIP.  The message is
 * the thread's (tof_last_error(NULL)).
 */
tof_status tof_project_step_static(const tof_grid *grid, const tof_box *design, const uint8_t *mask, void *rho,
                                   const void *grad, double alpha, void *stream);

/*
 * tof_tensor -- the real-space tensor as computed on the GPU (for checks):
 * N_c(k) for offsets 0 <= k_a < n_a, device double [6][nz][ny][nx],
 * components xx, yy, zz, xy, xz, yz; other offsets follow by parity (the
 * diagonal is even in every axis, xy odd in x and y, xz odd in x and z, yz odd
 * in y and z).  Allocates temporaries (setup-class call) and synchronizes.
 * Errors: TOF_ERR_INVALID, TOF_ERR_OOM, TOF_ERR_HIP.
 */
tof_status tof_tensor(tof_ctx *ctx, double *N, void *stream);

/*
 * tof_tensor_full -- the same tensor at every signed offset, device double
 * [6][2nz-1][2ny-1][2nx-1], entry (kz + nz - 1, ky + ny - 1, kx + nx - 1) for
 * offset (kx, ky, kz), |k_a| < n_a: the octant of tof_tensor with the parity
 * signs applied (the discrete tensor of eq. (demag_tensor) for every pair of
 * cells of the grid).  Allocates temporaries and synchronizes.
 * Errors: TOF_ERR_INVALID, TOF_ERR_OOM, TOF_ERR_HIP.
 */
tof_status tof_tensor_full(tof_ctx *ctx, double *N, void *stream);

/*
 * Per-launch timing (a measurement aid).  While enabled, every hot call
 * times its kernel launches on their stream with HIP events: each launch
 * carries a stop event that takes the kernel's completion timestamp
 * (hipExtLaunchKernelGGL, no packet added to the stream).  A launch that
 * directly follows a timed launch on the same stream (no other launch of the
 * library in between) is timed from that launch's completion to its own,
 * which is the launch's share of a back-to-back sequence; the first launch
 * of such a chain is timed from an event recorded just before it, which adds
 * that event's latency, and a slot reports those only when it has no chained
 * launch.  A pass of several kernels is timed to an event recorded after its
 * last one.  Slots:
 * 0-4 the passes of the forward convolution (x, y, z with the tensor product,
 * inverse y, inverse x with its epilogue), 5 the objective (with
 * TOF_OPT_FUSE_OBJECTIVE also the adjoint's x pass, slot 6 then unused), 6-10
 * the passes of the adjoint convolution (the last one also zeroes the
 * gradient outside the design region), 11 the sum of the objective's block
 * terms into J when the fused objective is not followed by the fused
 * adjoint y / z-sum kernel (which otherwise forms J).  With the fused y /
 * z-sum kernels (TOF_OPT_FUSE_YZ) slot 2 (8 in the adjoint) holds the fused
 * kernel, which also does the inverse y transform, and slots 1 and 3 (7 and
 * 9) are unused.  At most 1024 calls are recorded between reads; later ones
 * are not timed.  Errors: TOF_ERR_INVALID, TOF_ERR_HIP.
 */
#define TOF_PROFILE_SLOTS 12
tof_status tof_profile_enable(tof_ctx *ctx, int32_t enable);

/*
 * Synchronizes the recorded events, then per slot writes the summed
 * milliseconds, the number of timed launches and the algorithmic bytes of one
 * launch (the arrays the pass must read and write: its input and output, the
 * density it reads, the tensor spectrum octant it reads), then clears the
 * record.  Host arrays of TOF_PROFILE_SLOTS entries.  Errors: TOF_ERR_INVALID,
 * TOF_ERR_HIP.
 */
tof_status tof_profile_read(tof_ctx *ctx, double ms_host[], int64_t count_host[], double bytes_host[]);

/*
 * Bursts (a measurement aid that adds nothing to a launch): with timing
 * enabled, tof_profile_burst arms every slot whose bit is set in slot_mask;
 * the next call that runs the slot's pass launches that pass `repeats` more
 * times back to back right after its own launch, between two events on its
 * stream, and disarms the slot.  Every repeated pass writes only its
 * outputs, from inputs it leaves unchanged, so the call's results are those
 * of a call without the burst; the z passes of the unfused paths work in
 * place and are not repeated (their slots report 0).
 * tof_profile_burst_read synchronizes and writes per slot the mean
 * milliseconds per launch of its last burst (0 where none ran), then clears
 * them.  repeats in [1, TOF_PROFILE_MAX_BURST].
 * Errors: TOF_ERR_INVALID (timing off, repeats or mask out of range, null
 * argument), TOF_ERR_HIP.
 */
#define TOF_PROFILE_MAX_BURST 4096
tof_status tof_profile_burst(tof_ctx *ctx, uint32_t slot_mask, int32_t repeats);
tof_status tof_profile_burst_read(tof_ctx *ctx, double ms_host[]);

/*
 * Name of the kernel last timed in a slot (e.g. "k_yzsum_gather"), "" if
 * none; valid until the next timed call on the context.  *work_items (if not
 * NULL) receives that launch's grid size times block size (the work-item
 * count profilers report), 0 if none.
 */
const char *tof_profile_kernel(const tof_ctx *ctx, int32_t slot, int64_t *work_items);

/*
 * Pass choices (options 1-3), each 0 or 1 (default 1); the result is the
 * same convolution either way, up to rounding order.
 *   TOF_OPT_ZSUM     when the source or the target spans at most 4 z rows,
 *                    the z pass is a direct sum against the tensor
 *                    transformed along x and y, instead of FFTs along z.
 *   TOF_OPT_FUSE_YZ  that direct sum runs fused with the y transforms
 *                    (power-of-two Ly from 32 to 512), so the y spectra of
 *                    the many-row side never go through device memory.
 *   TOF_OPT_FUSE_OBJECTIVE  tof_objective_and_grad evaluates J and dJ/dH in
 *                    the kernel that starts the adjoint (its FFT along x;
 *                    power-of-two Lx from 32 to 512), which also transforms
 *                    the field rows it reads back along x, so neither the
 *                    field nor dJ/dH is stored; the per-block J terms are
 *                    added, in block order, by the adjoint's next kernel.
 *                    The J reduction order differs from the separate
 *                    objective kernel's (rounding only).
 * Errors: TOF_ERR_INVALID.
 */
#define TOF_OPT_ZSUM 1
#define TOF_OPT_FUSE_YZ 2
#define TOF_OPT_FUSE_OBJECTIVE 3
/*
 * Tile choices (options 4-6), the same result bit for bit, only the work
 * split changes (for a schedule tuner):
 *   TOF_OPT_X_TILE  tile of the x passes with power-of-two Lx: 0 (default)
 *                   picks one row pair a block when the full tiles would
 *                   give fewer than 512 blocks; 1 always the full tile (the
 *                   length's compiled row pairs per block); 2 always one
 *                   row pair a block.
 *   TOF_OPT_GATHER_GROUPS, TOF_OPT_SCATTER_GROUPS  row groups of the fused
 *                   y / z-sum kernels (blocks = groups x (Lx/2+1)), 1 to
 *                   64, or 0 for the default (3 and 8, at most the rows).
 *                   The gather's groups are added in group order, so its
 *                   group count changes the rounding of the sum.
 */
#define TOF_OPT_X_TILE 4
#define TOF_OPT_GATHER_GROUPS 5
#define TOF_OPT_SCATTER_GROUPS 6
tof_status tof_set_option(tof_ctx *ctx, int32_t option, int32_t value);

/* Padded lengths chosen for the context: out[0..2] = Lx, Ly, Lz. */
tof_status tof_padded_lengths(const tof_ctx *ctx, int32_t out[3]);

/*
 * Device bytes a context for `grid` holds once tof_create has returned
 * (spectra, workspaces, twiddle tables, small buffers), computed on the host
 * without creating anything: a caller can size memory first.  Setup needs
 * its temporaries on top (see tof_create), and tof_set_objective adds the
 * objective's buffers (a few words per sensor cell).  0 for an invalid grid
 * (tof_last_error(NULL) says why).
 */
size_t tof_workspace_bytes(const tof_grid *grid);

/* Device bytes a context holds now (workspaces, spectra, objective buffers). */
size_t tof_ctx_bytes(const tof_ctx *ctx);

/* Last error message of the context (or of this thread when ctx is NULL). */
const char *tof_last_error(const tof_ctx *ctx);

/*
 * The batched form: one gradient evaluation (tof_objective_and_grad) of many
 * independent designs, each with its own context, with one launch per pass
 * and kernel instantiation for all of them instead of five launches per
 * design.  tof_batch_create records every design's launches (their
 * arguments: the context, rho[i], J[i], grad[i], as for
 * tof_objective_and_grad) and groups them per pass; designs whose padded
 * lengths and pass choices select the same kernels share a launch, over a
 * device table of their arguments.  Setup-class call (allocates the table).
 * The contexts and buffers are borrowed: they must stay valid, and their
 * design, objective and options unchanged, while the batch is used.
 * tof_batch_run enqueues one evaluation of every design on `stream` (no
 * allocation, no synchronization: capturable into a graph), its launches
 * one after another on `stream`; results are those of
 * tof_objective_and_grad on each context (the same kernels).
 * Runs of one batch must not overlap.
 * Requires the fused passes (TOF_OPT_ZSUM, TOF_OPT_FUSE_YZ and
 * TOF_OPT_FUSE_OBJECTIVE on, power-of-two Lx and Ly from 32 to 512, an
 * objective on one or a few z layers) and no validation or timing.
 * Errors: TOF_ERR_INVALID, TOF_ERR_STATE, TOF_ERR_UNSUPPORTED (a design
 * launches a kernel with no batched form), TOF_ERR_OOM, TOF_ERR_HIP; the
 * message is the thread's (tof_last_error(NULL)).
 */
typedef struct tof_batch tof_batch;
tof_status tof_batch_create(tof_ctx *const *ctxs, const void *const *rho, double *const *J, void *const *grad,
                            int32_t n, tof_batch **out);
tof_status tof_batch_run(tof_batch *batch, void *stream);
/* Kernel launches one tof_batch_run makes. */
int32_t tof_batch_launches(const tof_batch *batch);
/* Waits for the device, then frees the batch.  NULL is a no-op. */
void tof_batch_destroy(tof_batch *batch);

/*
 * tof_dd_newell_host -- the double-double Newell evaluation the GPU setup
 * uses, run on the host (same source), for CPU-side checks: the tensor entry
 * of component c (0..5 as above) at offset (kx, ky, kz) >= 0 for cell size
 * (dx, dy, dz), rounded to double.  Returns NaN for bad arguments.
 */
double tof_dd_newell_host(int32_t c, int32_t kx, int32_t ky, int32_t kz,
                          double dx, double dy, double dz);

#ifdef __cplusplus
}
#endif

#endif /* TOF_H */
