/*
 * pic.h -- C ABI of the MI355X (gfx950) library for the explicit, energy-conserving
 * particle-in-cell step of Ricketson & Hu, "An explicit, energy-conserving
 * particle-in-cell scheme".
 *
 * Problem (section 2.1, eq. (vlasov), (maxwell)): dimensionless Vlasov equation for one
 * mobile species with charge-to-mass ratio +1 on a uniform neutralising background
 * (Gauss: div E = rho - 1), time in 1/omega_p, length in Debye lengths, velocity in
 * thermal speeds, c = speed of light / thermal speed.  Here space is one-dimensional
 * and periodic, x in [0, L), with velocities of 1 or 3 components ("1D-1V", "1D-3V").
 *
 * Discretisation (section 2.2): particles (x_p, v_p, w_p); nodes x_i = i h, h = L/N_g;
 * cardinal B-spline shapes of degree 1 (tent, S(z) = max(0, 1 - |z|/h)) or 2; current
 * deposit j_i = (1/h) sum_p w_p v_p S(x_i - x_p); gather E_p = sum_i E_i S(x_p - x_i).
 * Electric field components live on the nodes; in the electromagnetic scheme B_y, B_z
 * live on the half nodes (i + 1/2) h (a one-dimensional Yee lattice, section 2.2.2).
 *
 * Schemes (section 5 names them):
 *   PIC_ESEC2   eq. (good_translation): predictor deposit j^{n,*} at x* with v^n, predictor
 *               field E*, half-step velocity v*, centred deposit j^{*,n+1/2} at
 *               x^{n+1/2} with v*, Ampere update, provisional v-dagger, and the
 *               energy-restoring factor Gamma of eq. (opt_solution).
 *   PIC_ESEC1   eq. (naivetranslation) + eq. (PICmodification): as ESEC2 without the
 *               predictor deposit (v* uses E^n).  Its one grid-wide dependency per step
 *               lets one launch finish step n and deposit step n+1's centred current,
 *               so the state is read and written once per step.
 *   PIC_EMEC_LI eq. (EMbasic): ESEC2's particle update with the Crank-Nicolson
 *               (linearly implicit) Maxwell update; requires nv == 3.
 *   PIC_EMEC_PSATD eq. (EM_PSATD), section 4.2: as PIC_EMEC_LI with the Maxwell update
 *               integrated exactly in time for each Fourier mode with the current held
 *               fixed over the step (eq. (PSATDformula)): (E*, B*) = PSATD(E^n, B^n,
 *               j^{n,*}, dt/2) for v*, (E^{n+1}, B^{n+1}) = PSATD(E^n, B^n, j^{*,n+1/2},
 *               dt), and v-dagger gathers the exact time average of E over the step and
 *               B^{n+1/2} = (B^n + B^{n+1})/2.  The curls are spectral on the same
 *               staggered grid (d/dx from nodes to half nodes multiplies mode k by
 *               i k e^{i k h/2}, back by i k e^{-i k h/2}); E_x has no curl term.  Each
 *               field update is a fixed-order real-space convolution with rows computed
 *               once at initialisation.  Requires nv == 3.
 *   PIC_EMEC_LF eq. (EMleapfrog), section 4.1: the Yee leapfrog.  B lives at half steps:
 *               the caller's B is B^{-1/2} at initialisation, and after m steps E holds
 *               E^m and B holds B^{m-1/2}.  Each step: B^{n+1/2} = B^{n-1/2} - dt curl E^n,
 *               E* = E^n + dt/2 (c^2 curl B^{n+1/2} - j^{n,*}), v* gathers E* and
 *               B^{n+1/2} at x*, E^{n+1} = E^n + dt (c^2 curl B^{n+1/2} - j^{*,n+1/2}),
 *               v-dagger gathers (E^n + E^{n+1})/2 and B^{n+1/2} at x^{n+1/2}.  The record
 *               of step n reports the magnetic energy of that section,
 *               W_B^n = c^2/2 h sum B^{n+1/2} . B^{n-1/2}.  Requires nv == 3 and
 *               c dt <= h (the leapfrog's stability limit).
 *   PIC_STANDARD the comparison scheme of section 5 (not energy-conserving): Vlasov-Poisson
 *               with the leapfrog/Boris push in its symmetric form, eq. (symm_Boris):
 *               x* = x^n + dt/2 v^n, E^{n+1/2} the Gauss field (spectral, as the initial
 *               field) of the charge density at the x*, v^{n+1} = v^n + dt (E^{n+1/2}(x*)
 *               + v^{n+1/2} x b_ext), x^{n+1} = x* + dt/2 v^{n+1}.  Needs
 *               PIC_F_INIT_GAUSS; electrostatic only.  Its fields live at half steps:
 *               after step n the caller's E holds E^{n-1/2}, and the record of step
 *               n >= 1 is TE at (n - 1/2) dt, the mean of the kinetic energies of steps
 *               n - 1 and n plus the field energy of E^{n-1/2}.
 * Electrostatic Ampere form (eq. (ampere), 1D): E^{n+1} = E^n - dt (j - mean(j)); the
 * mean is removed because E = -d(phi)/dx has zero mean in a periodic domain.
 * Correction (eq. (opt_solution)): r = 1 + 2 (v* - (v-dagger + v^n)/2).(v-dagger - v^n)
 * / |v-dagger|^2; Gamma = sqrt(r) if r >= 0 and finite, else Gamma = 1 and the particle is
 * counted as a fallback (section 3.2: an imaginary root is replaced by 1).
 * Energy (section 5.1): TE = 1/2 sum_p w_p |v_p|^2 + 1/2 h sum_i |E_i|^2
 *                            + c^2/2 h sum_{i+1/2} |B_{i+1/2}|^2 (EM only).
 *
 * Memory: every pointer in pic_buffers is a DEVICE pointer owned by the caller and must
 * stay valid until pic_destroy.  The library allocates no device memory: all scratch
 * space is carved from the caller's workspace.  All work is enqueued on the caller's HIP
 * stream; only pic_diagnostics (and the state/checkpoint calls) synchronise it.
 * Errors: every call returns a pic_status; nothing aborts.  PIC_EINVAL leaves every
 * argument untouched.  After PIC_EDEVICE the context is poisoned and later calls on it
 * return PIC_ESTATE.  A context is bound to one stream and is not thread-safe.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 1

enum pic_status {
    PIC_OK = 0,
    PIC_EINVAL = -1,         /* invalid parameter, pointer, size or alignment          */
    PIC_ENOMEM = -2,         /* workspace smaller than pic_workspace_size()            */
    PIC_EDEVICE = -3,        /* a HIP call failed; the context is poisoned             */
    PIC_ESTATE = -4,         /* call on a poisoned or destroyed context                */
    PIC_ENONFINITE = -5,     /* a particle or field value became NaN/Inf (diagnostics) */
    PIC_EUNSUPPORTED = -6    /* valid but outside what this library handles            */
};

enum pic_scheme { PIC_ESEC2 = 0, PIC_ESEC1 = 1, PIC_EMEC_LI = 2, PIC_STANDARD = 3,
                  PIC_EMEC_PSATD = 4, PIC_EMEC_LF = 5 };

enum pic_flag {
    PIC_F_INIT_GAUSS = 1u,   /* set E_x^0 from the particles: dE/dx = rho - 1 solved
                                spectrally on the nodes (mean and Nyquist modes zero);
                                otherwise the caller's E (and B) are E^0 (B^0)          */
    PIC_F_TRACK_IDS = 2u,    /* permute the caller's id array with the particles        */
    PIC_F_INTERLEAVE = 4u,   /* deal particle batches to the workgroups round-robin
                                instead of in contiguous chunks (faster once the state
                                streams from HBM); chosen by itself when the state is
                                larger than 192 MB.  Not with rebin_every > 0           */
    PIC_F_FILTER_RHO = 16u,  /* PIC_STANDARD: one pass of the binomial filter (1/4, 1/2,
                                1/4) on the charge density before each field solve
                                (section 5 filters the standard scheme's density)       */
    PIC_F_CHARGE_CONSERVING = 32u, /* exact charge conservation (section 3.5, eq. (discCont),
                                eq. (detbal)) for PIC_ESEC2 with tent shapes
                                (shape_order 1), electrostatic: E_x and the current live on
                                the half nodes (i + 1/2) h; the centred current is
                                deposited, and v-dagger's field gathered, through the pieces
                                of each particle's path x^n -> x^{n+1} between the half
                                nodes, each piece carrying its fraction of the path at its
                                midpoint.  Then D-(E) = rho - mean(rho) holds at every step
                                (if it holds at the start), with rho_i = (1/h) sum_p w_p
                                S2(x_i - x_p) on the nodes, S2 the quadratic B-spline, and
                                D-(E)_i = (E_{i+1/2} - E_{i-1/2}) / h.  PIC_F_INIT_GAUSS
                                then solves that law (running sum, mean of E zero).  Needs
                                rebin_every == 0 and the LDS_ATOMIC or LDS_F64 deposit    */
    PIC_F_DETERMINISTIC = 8u /* bit-for-bit reproducible runs (and continuations through
                                pic_save_state / pic_load_state with the same launch
                                shape): each workgroup's deposit is summed exactly in
                                fixed point and the workgroups' sums are added in
                                workgroup order (an extra small launch per deposit);
                                wavefronts take their particles in a fixed order.  Needs
                                rebin_every == 0 and the LDS_ATOMIC deposit.  Results
                                differ from the default mode only by rounding           */
};

/* Deposit strategies for the per-workgroup LDS current tiles (section 2.2 deposit).  All
 * give the same sums up to floating-point summation order. */
enum pic_deposit_mode {
    PIC_DEPOSIT_AUTO = 0,         /* WINDOW when rebin_every > 0, else LDS_ATOMIC         */
    PIC_DEPOSIT_LDS_ATOMIC = 1,   /* every particle adds its stencil with 64-bit integer
                                     LDS atomics on a fixed-point tile (scale chosen per
                                     run so no entry overflows; out-of-range contributions
                                     go to an FP64 side tile); workgroup sums are exact     */
    PIC_DEPOSIT_WINDOW = 2,       /* each thread sums its particles' stencils in registers
                                     over a few nodes and adds them when the window moves;
                                     pays off when particles are cell-sorted             */
    PIC_DEPOSIT_WAVE = 3,         /* each lane sums its stencils in registers over a window
                                     shared by the wavefront (anchored at its first
                                     particle); the window is summed across the wavefront
                                     (DPP) before one LDS add; for cell-sorted particles   */
    PIC_DEPOSIT_LDS_F64 = 4       /* every particle adds its stencil with FP64 LDS atomics */
};

typedef struct {
    int32_t abi_version;   /* must equal PIC_ABI_VERSION                                 */
    int32_t nv;            /* velocity components per particle: 1 or 3                   */
    int32_t scheme;        /* enum pic_scheme; the EM schemes require nv == 3            */
    int32_t shape_order;   /* B-spline degree: 1 (tent) or 2 (quadratic)                 */
    int64_t n_particles;   /* N_p >= 1                                                   */
    int32_t n_cells;       /* N_g >= 2 * shape_order + 1                                 */
    int32_t rebin_every;   /* counting-sort the particles by (cell, sign of v_x) before
                              steps 0, K, 2K, ...; 0: never.  Particle order is then
                              unspecified: track identities with PIC_F_TRACK_IDS          */
    double  length;        /* L > 0                                                      */
    double  dt;            /* time step > 0                                              */
    double  c;             /* speed of light (EM schemes), > 0                           */
    double  b_ext[3];      /* uniform imposed magnetic field added to every gathered B
                              (section 3.2 starts from an externally imposed B); used
                              only when nv == 3                                           */
    uint32_t flags;        /* enum pic_flag bits                                         */
    int32_t block_threads; /* threads per workgroup of the particle passes: 0 = default
                              (1024, halved down to 64 while N_p < 512 block_threads,
                              i.e. two particles per thread of 256 workgroups), else a
                              multiple of 64 in [64, 1024]                                */
    int32_t grid_blocks;   /* workgroups of the particle passes: 0 = default,
                              min(256, ceil(N_p / (2 block_threads))), one per CU.
                              Each workgroup takes a chunk of
                              ceil(N_p / grid) particles rounded up to a multiple of 64,
                              so the grid launched may be smaller than asked             */
    int32_t deposit_mode;  /* enum pic_deposit_mode                                      */
    int32_t record_capacity; /* per-step diagnostic records kept on the device: 0 = 4096 */
    int32_t reserved;      /* must be 0                                                  */
} pic_params;

typedef struct {
    double  *x;            /* [N_p] positions, in/out; wrapped into [0, L) at init       */
    double  *v;            /* [nv][N_p] velocities (structure of arrays), in/out         */
    const double *w;       /* [N_p] weights, or NULL for uniform w_p = L / N_p           */
    int64_t *id;           /* [N_p] particle ids permuted with the particles (needed with
                              PIC_F_TRACK_IDS), may be NULL otherwise                     */
    double  *E;            /* [3][N_g] node field (E_x, E_y, E_z), in/out; the
                              electrostatic schemes use and update E_x only               */
    double  *B;            /* [2][N_g] half-node field (B_y, B_z), in/out; EM schemes
                              (PIC_EMEC_LI, PIC_EMEC_PSATD, PIC_EMEC_LF) only, NULL
                              otherwise                                                   */
    void    *workspace;    /* >= pic_workspace_size(params) bytes, 256-byte aligned,
                              caller-owned scratch the library carves up                  */
    size_t   workspace_bytes;
} pic_buffers;

/* One record per step; pic_diagnostics returns them in step order. */
typedef struct {
    int64_t step;          /* n (0 = initial state)                                      */
    double  time;          /* n * dt                                                     */
    double  kinetic;       /* 1/2 sum_p w_p |v_p^n|^2                                    */
    double  field_e;       /* 1/2 h sum_i |E_i^n|^2                                      */
    double  field_b;       /* c^2/2 h sum |B^n|^2 (EM), else 0                           */
    double  total;         /* kinetic + field_e + field_b                                */
    double  rel_energy_err;/* |TE^n - TE^0| / TE^0                                       */
    double  max_gamma_dev; /* max_p |Gamma_p - 1| over the particles of this step        */
    int64_t fallbacks;     /* particles whose radicand was negative or not finite        */
    int64_t fallbacks_total; /* cumulative since init                                    */
    int32_t nonfinite;     /* 1 if a NaN/Inf appeared in this step's state               */
    int32_t pad;
} pic_diag;

typedef struct pic_ctx pic_ctx;

/* Bytes of workspace the library needs for these parameters (0 if they are invalid). */
size_t pic_workspace_size(const pic_params *p);

/* Host-only check of the parameters (no GPU needed).  PIC_OK, PIC_EINVAL or
 * PIC_EUNSUPPORTED; pic_last_error(NULL) then describes the problem. */
int pic_validate_params(const pic_params *p);

/* Host-only check of a run's inputs before they are copied to the device (no GPU needed):
 * the parameters as pic_validate_params, then every value of the HOST arrays x [N_p],
 * v [nv][N_p], w [N_p] (may be NULL), E [3][N_g] and B [2][N_g] (EM schemes; may be NULL
 * otherwise) must be finite.  PIC_ENONFINITE names the first non-finite value (array and
 * index) in pic_last_error(NULL) and stores its index within that array in *bad_index (may
 * be NULL; -1 when nothing is wrong); PIC_EINVAL for NULL x, v, E (or B in EM).  Nothing is
 * modified.  The device-side counterpart is the non-finite flag of the records. */
int pic_check_inputs(const pic_params *p, const double *x, const double *v, const double *w,
                     const double *E, const double *B, int64_t *bad_index);

/* Bind a context to the caller's buffers and HIP stream (hipStream_t, may be NULL for
 * the null stream) and enqueue the initial work: wrap x into [0, L); optionally the
 * Gauss solve for E_x^0; the energy record of step 0; for ESEC2 and the EM schemes the
 * predictor deposit j^{0,*} (eq. (good_translation), (EMbasic), (EM_PSATD)); for
 * PIC_EMEC_PSATD also the rows of its field-update convolutions.
 * On success *out receives the context.  The first init on a device (of any form) also
 * checks, with two one-workgroup launches and a wait on the stream, that the runtime
 * passes the workgroup size where the kernels read it; PIC_EUNSUPPORTED if not. */
int pic_init(const pic_params *p, const pic_buffers *b, void *hip_stream, pic_ctx **out);

/* Enqueue n_steps steps (eq. (good_translation) / (naivetranslation)+(PICmodification) /
 * (EMbasic) / (EM_PSATD) / (EMleapfrog) / (symm_Boris)), each recording a pic_diag.  Asynchronous: returns after enqueueing. */
int pic_step(pic_ctx *ctx, int64_t n_steps);

/* Synchronise the stream and copy out the records written since the previous call (the
 * first call also returns step 0), oldest first, at most max_records of them; records
 * older than the device ring's capacity are lost.  *n_written receives the count.
 * Returns PIC_ENONFINITE if any returned record has nonfinite set. */
int pic_diagnostics(pic_ctx *ctx, pic_diag *out, int64_t max_records, int64_t *n_written);

/* Synchronise and make the caller's x, v (and id) arrays hold the current particle
 * state (after a rebin the current state may sit in the workspace). */
int pic_sync_state(pic_ctx *ctx);

/* ----------------------------------------------------------- checkpoint / resume
 * The complete state of a run between two steps: positions, velocities, ids (with
 * PIC_F_TRACK_IDS), the library's permuted weights (rebins with non-uniform weights),
 * E^n and B^n, the predictor current j^{n,*} that ESEC2 and the EM schemes carry from one step
 * to the next (eq. (good_translation) with (doublestardef); for ESEC1 the centred current
 * j^{n+1/2} its previous launch deposited), the step number n, the
 * initial total energy, the fallback total, the deposit's fixed-point scales and the
 * record of step n.  The saved state is a self-describing block of HOST memory in the
 * library's own format (native byte order; not a portable file format). */

/* Bytes pic_save_state writes for this context; 0 for a NULL or poisoned context. */
size_t pic_state_size(const pic_ctx *ctx);

/* Synchronise the stream and write the state into dst (HOST memory of at least
 * pic_state_size(ctx) bytes; PIC_EINVAL if smaller or NULL). */
int pic_save_state(pic_ctx *ctx, void *dst, size_t bytes);

/* Synchronise and replace the context's state by a saved one (HOST memory): the caller's
 * x, v (id) and E (B) arrays receive the saved values, and the next pic_step continues
 * from step n exactly as the saving context would have (in PIC_F_DETERMINISTIC with the
 * same launch shape, bit for bit; otherwise up to the order of the current sums).  The
 * next pic_diagnostics returns the record of step n first.  The context must have been
 * initialised with the same nv, scheme, shape order, N_p, N_g, L, dt, c, b_ext and the
 * same PIC_F_DETERMINISTIC and PIC_F_TRACK_IDS bits (and non-uniform weights with rebins
 * if the saver had them); otherwise, or for a damaged block, PIC_EINVAL with nothing
 * modified.  The number of current replicas may differ (their sum is then restored). */
int pic_load_state(pic_ctx *ctx, const void *src, size_t bytes);

/* Kernel classes timed by the optional event profiler. */
enum pic_kernel_class {
    PIC_K_PASS_A = 0,      /* (PIC_STANDARD: the field solve of each step)
                              gather at x*, v*, centred deposit; its last workgroup does
                              the Ampere / Crank-Nicolson field update                 */
    PIC_K_PASS_B = 1,      /* gather at x^{n+1/2}, Gamma, state write, predictor deposit
                              (ESEC1: the one launch per step, which ends with the next
                              step's centred deposit);
                              its last workgroup writes the step record and E* (B*)    */
    PIC_K_REBIN = 2,       /* counting-sort rebin (all of its kernels)                 */
    PIC_K_COUNT = 3
};

/* Enable (on != 0) or disable HIP-event timing of every kernel pic_step enqueues: a
 * hipEvent is recorded on the context's stream right before and right after each
 * launch.  Timing adds a few microseconds per launch; use it on a separate run. */
int pic_profile_enable(pic_ctx *ctx, int on);

/* The launch shape the context resolved (threads per workgroup, workgroups and particles
 * per workgroup of the particle passes).  Any output pointer may be NULL. */
int pic_launch_shape(const pic_ctx *ctx, int32_t *block_threads, int32_t *grid_blocks,
                     int64_t *chunk);

/* Synchronise and return, per pic_kernel_class, the summed milliseconds and the launch
 * count since profiling was enabled (arrays of PIC_K_COUNT entries); resets them. */
int pic_profile_read(pic_ctx *ctx, double *ms, int64_t *launches);

/* Release the context (host memory only; caller buffers are untouched). */
int pic_destroy(pic_ctx *ctx);

const char *pic_strerror(int status);

/* ------------------------------------------------ allocation-free single run
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.
 *
 * Does what pic_init(p, b, hip_stream) followed by pic_step(n_steps) does, in one call
 * and without a context, with the workspace taken from a static device array of the
 * library (PIC_STATIC_SCRATCH_BYTES per device, held by every device the library runs
 * on until the process ends) instead of the caller's: b->workspace must be NULL and
 * b->workspace_bytes 0; every other field of b is as for pic_init (caller-owned device
 * arrays, updated in place).  When diag_out (a DEVICE pointer to one pic_diag) is not
 * NULL, the record of the newest step is written there.  Asynchronous: everything is
 * enqueued on hip_stream.  No device or pinned memory is allocated and nothing is freed.
 * Errors: PIC_ENOMEM when pic_workspace_size(p) exceeds PIC_STATIC_SCRATCH_BYTES (for
 * example with rebins of many particles or a large record_capacity); otherwise as
 * pic_init and pic_step, with messages from pic_last_error(NULL).
 * Every call on one device shares that device's array, which keeps the previous call's
 * contents (the call clears what must start at zero): calls that overlap on one device
 * (other streams, other threads) race and give wrong results.  The first call on a
 * device of any entry point waits once on the stream for the library's check of the
 * kernels' launch layout, so make one call outside graph capture first. */
#define PIC_STATIC_SCRATCH_BYTES ((size_t)16 << 20)

int pic_run_static(const pic_params *p, const pic_buffers *b, void *hip_stream,
                   int64_t n_steps, pic_diag *diag_out);

/* ------------------------------------------------------------ batched ensemble form
 * Many independent runs of one scheme advanced together: each run has its own particle
 * count, cell count and length; all share the scheme, shape order, nv, dt, c and b_ext.
 * Schemes: ESEC2, ESEC1 and EMEC(LI).
 * Every pass of every step is one persistent launch over a table of work items (chunks of
 * one run's particles), and steps can be replayed from a captured hipGraph.  Each run
 * computes exactly what pic_step computes for it alone (same records, same parity). */
enum pic_batch_flag {
    PIC_BF_INIT_GAUSS = 1u       /* as PIC_F_INIT_GAUSS, for every run                     */
};

typedef struct {
    int32_t abi_version;         /* PIC_ABI_VERSION                                       */
    int32_t n_runs;              /* >= 1                                                  */
    int32_t nv, scheme, shape_order;
    uint32_t flags;              /* enum pic_batch_flag                                   */
    double  dt, c;
    double  b_ext[3];
    const int64_t *n_particles;  /* HOST array [n_runs]: N_p of each run (>= 1)           */
    const int32_t *n_cells;      /* HOST array [n_runs]: N_g of each run                  */
    const double  *length;       /* HOST array [n_runs]: L of each run                    */
    int32_t block_threads;       /* 0 = default (256), else a multiple of 64 in [64, 512] */
    int32_t chunk;               /* particles per work item, 0 = default; a multiple of
                                    block_threads                                         */
    int32_t grid_blocks;         /* persistent grid, 0 = default                          */
    int32_t graph_steps;         /* > 0: pic_batch_step replays a captured hipGraph of this
                                    many steps (needs a non-null stream); 0: plain launches */
    int32_t record_capacity;     /* per-run record ring, 0 = 1024                         */
    int32_t reserved;            /* 0                                                     */
} pic_batch_params;

typedef struct {                 /* DEVICE pointers, caller-owned, packed by run          */
    double  *x;                  /* [N] with N = sum_r N_p,r; run r starts at
                                    P_r = sum_{s<r} N_p,s                                  */
    double  *v;                  /* [nv][N]: component c of run r at c N + P_r            */
    const double *w;             /* [N] weights or NULL (uniform L_r / N_p,r per run)     */
    double  *E;                  /* [3 G] with G = sum_r N_g,r: run r's [3][N_g,r] block
                                    starts at 3 sum_{s<r} N_g,s                             */
    double  *B;                  /* [2 G] likewise (EMEC(LI) only), else NULL             */
    void    *workspace;          /* >= pic_batch_workspace_size bytes, 256-byte aligned   */
    size_t   workspace_bytes;
} pic_batch_buffers;

typedef struct pic_batch pic_batch;

/* Workspace bytes for these parameters, 0 if invalid (pic_last_error(NULL) says why). */
size_t pic_batch_workspace_size(const pic_batch_params *p);

/* Bind and initialise every run (as pic_init does for one run). */
int pic_batch_init(const pic_batch_params *p, const pic_batch_buffers *b, void *hip_stream,
                   pic_batch **out);

/* Enqueue n_steps steps of every run; asynchronous. */
int pic_batch_step(pic_batch *ctx, int64_t n_steps);

/* Synchronise and copy out run `run`'s records written since the previous call for that
 * run (the first call also returns step 0), as pic_diagnostics does. */
int pic_batch_diagnostics(pic_batch *ctx, int32_t run, pic_diag *out, int64_t max_records,
                          int64_t *n_written);

int pic_batch_destroy(pic_batch *ctx);

/* ----------------------------------------------------------------- adjoint form
 * Reverse-mode derivative of an ESEC2 run (1D-1V electrostatic, started from the Gauss
 * solve) with respect to the parameters of its initial condition, for the loss
 *     J = loss_weight * sum_{n=1..N} W_E^n,   W_E = (h/2) sum_i E_i^2  (section 5.1).
 * The initial condition is the one of the paper's Landau / two-stream problems
 * (section 5): positions from the density 1 + sum_m alpha_m cos(k_m x) by inverse-CDF
 * sampling of given uniforms u_p (Newton to 1e-15 L), velocities v_b s_p + v_s g_p for
 * given factors s_p (beam signs) and draws g_p.  The gradient is taken with respect to
 * (alpha_1 .. alpha_M, v_b, v_s); the sampling is differentiated implicitly,
 * dx_p/dalpha_m = -sin(k_m x_p) / (k_m (1 + sum_j alpha_j cos(k_j x_p))).
 *
 * pic_adj_forward samples, initialises and runs N steps exactly as pic_init + pic_step,
 * storing the particle state (x, v) every checkpoint_every steps and every step's grids
 * and fields (E^n, the two currents, E*, E-bar and E^{n+1}: 6 N_g values);
 * pic_adj_backward recomputes each segment's states from its checkpoint and those grids
 * (one gather-only launch per step) and runs the reverse of the steps, of the Gauss solve
 * and of the sampling.  The fallback Gamma := 1 (section 3.2) is a constant in the
 * derivative.
 * Streams: the context enqueues on the caller's stream.  The backward sweep recomputes the
 * next segment's states on a side stream of its own (created by pic_adj_init on the
 * caller's stream's device, default priority, destroyed by pic_adj_destroy) while the
 * caller's stream reverses the current segment; events order the two, and the sweep's
 * last launch on the caller's stream waits for the side stream, so work enqueued after
 * pic_adj_backward on the caller's stream sees all of it.  pic_adj_init fails with
 * PIC_EDEVICE if the stream or its events cannot be created. */
#define PIC_ADJ_MAX_MODES 16

typedef struct {
    int32_t abi_version;         /* PIC_ABI_VERSION                                       */
    int32_t shape_order;         /* 1 or 2                                                */
    int64_t n_particles;         /* >= 1                                                  */
    int32_t n_cells;             /* as pic_params                                         */
    int32_t n_steps;             /* N >= 1                                                */
    int32_t checkpoint_every;    /* K >= 1: stored states at steps 0, K, 2K, ...          */
    int32_t n_modes;             /* M in [0, PIC_ADJ_MAX_MODES]                           */
    double  length, dt;
    double  loss_weight;         /* usually dt (time integral of W_E)                     */
    double  k[PIC_ADJ_MAX_MODES];/* mode wavenumbers, each a multiple of 2 pi / L         */
    int32_t block_threads;       /* as pic_params; both 0: 512 threads x 512 workgroups   */
    int32_t grid_blocks;         /* (two per CU) from N_p >= 524288, else pic_params' own */
                                 /* defaults                                              */
    int32_t reserved[2];         /* 0                                                     */
} pic_adj_params;

typedef struct {                 /* DEVICE pointers, caller-owned, [N_p] unless stated    */
    const double *u;             /* uniforms in (0, 1)                                    */
    const double *s;             /* beam factors s_p                                      */
    const double *g;             /* spread draws g_p                                      */
    double *x, *v;               /* state: x^N, v^N after pic_adj_forward                 */
    double *E;                   /* [3][N_g]: E^N after pic_adj_forward (E_x used)        */
    double *loss;                /* [1]: J, written by pic_adj_forward                    */
    double *grad;                /* [M + 2]: dJ/d(alpha_1..alpha_M, v_b, v_s) times
                                    loss_bar, written by pic_adj_backward                  */
    void    *workspace;          /* >= pic_adj_workspace_size bytes, 256-byte aligned     */
    size_t   workspace_bytes;
} pic_adj_buffers;

typedef struct pic_adj pic_adj;

/* Workspace bytes (0 if the parameters are invalid; pic_last_error(NULL) says why).
 * About (2 ceil(N / K) + 4 K - 2) * 8 N_p + 48 N N_g bytes: checkpoints, two segments of
 * states, the adjoint state and every step's grids and fields. */
size_t pic_adj_workspace_size(const pic_adj_params *p);

int pic_adj_init(const pic_adj_params *p, const pic_adj_buffers *b, void *hip_stream,
                 pic_adj **out);

/* Enqueue the forward run for these parameter values (host arrays/values). */
int pic_adj_forward(pic_adj *ctx, const double *alpha, double v_beam, double v_spread);

/* Enqueue the reverse sweep for the last forward run; loss_bar scales the gradient. */
int pic_adj_backward(pic_adj *ctx, double loss_bar);

/* Synchronise and copy the records (as pic_diag, steps 0..N) of the last forward run. */
int pic_adj_records(pic_adj *ctx, pic_diag *out, int64_t max_records, int64_t *n_written);

int pic_adj_destroy(pic_adj *ctx);

/* Last error message of a context, or of the calling thread's last failed
 * validation/init when ctx is NULL. */
const char *pic_last_error(const pic_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
