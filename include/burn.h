/*
 * burn.h -- C ABI of the MI355X per-cell reaction-network burn (libburn.so).
 *
 * The operation: every cell is an independent zone at fixed density rho that
 * evolves its molar abundances Y_1..Y_N and temperature T over a time dt
 * (the single-zone burn with self-heating of the paper, Sec. 2, where the
 * generated network RHS and Jacobian are integrated with a VODE-class stiff
 * integrator; Sec. 3 applies it zone by zone inside the hydrodynamics).
 *
 *   dY_i/dt = sum_r nu_ir R_r,          dT/dt = (1/c_v) sum_r q_r R_r,
 *   R_r     = e^{p_r} lambda_r(T) rho^{n_r-1} prod_j Y_j^{m_jr} / prod_j m_jr!,
 *   lambda_r(T) = exp(a0 + a1/T + a2 T^-1/3 + a3 T^1/3 + a4 T + a5 T^5/3 + a6 ln T)
 *
 * (the seven-parameter ReacLib rate form; the rate collections themselves are
 * cited in Sec. 2).  nu_ir = products minus reactants multiplicity, m_jr =
 * reactant multiplicity, n_r = number of reactant slots, p_r = log-rate
 * multiplier (the sensitivity knob of Sec. 1).  The integrator is a
 * variable-order (1..5) BDF in backward differences with modified Newton and
 * a dense partially pivoted LU of (I - c J), all in FP64.
 *
 * Conventions for every entry point:
 *  - Arrays marked DEVICE are device pointers (memory owned by the caller,
 *    e.g. PyTorch); arrays marked HOST are host pointers.
 *  - Cell arrays are structure-of-arrays: element (i, c) of a [K][n_cells]
 *    array is at i * n_cells + c, so consecutive cells are consecutive.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *    asynchronously; outputs are valid after the stream is synchronized.
 *  - A negative return value means nothing was enqueued; bn_last_error()
 *    then describes why.  Per-cell outcomes go to status[] (BN_CELL_*).
 *  - The library keeps no pointer to caller memory after the enqueued work
 *    finishes.  A network handle owns a small device copy of its tables.
 */
#ifndef MI355X_BURN_H
#define MI355X_BURN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Call-level return codes. */
#define BN_SUCCESS 0
#define BN_EINVAL (-1)       /* null pointer, bad size, rtol <= 0, atol < 0, dt <= 0, ... */
#define BN_EHIP (-2)         /* a HIP runtime call failed */
#define BN_ENOMEM (-3)       /* device allocation failed */
#define BN_EUNSUPPORTED (-4) /* network larger than the kernels support */

/* Per-cell outcomes written to status[]. */
#define BN_CELL_OK 0             /* reached dt */
#define BN_CELL_MAX_STEPS 1      /* step budget exhausted */
#define BN_CELL_STEP_UNDERFLOW 2 /* step fell below 10 ulp(t) */
#define BN_CELL_NONFINITE 3      /* rates / RHS / Jacobian not finite at the initial state */
#define BN_CELL_BAD_INPUT 4      /* rho <= 0, T <= 0, or a non-finite input */

/* Per-cell counters written to counters[BN_N_COUNTERS][n_cells]. */
#define BN_N_COUNTERS 8
#define BN_CNT_STEPS 0       /* accepted steps */
#define BN_CNT_REJ_ERR 1     /* error-test rejections */
#define BN_CNT_NEWTON_FAIL 2 /* failed Newton attempts */
#define BN_CNT_RHS 3         /* right-hand-side evaluations */
#define BN_CNT_JAC 4         /* Jacobian evaluations */
#define BN_CNT_LU 5          /* LU factorizations of I - cJ */
#define BN_CNT_SOLVE 6       /* forward/back substitution pairs */
#define BN_CNT_ORDER 7       /* BDF order at the end */

/* Largest supported system: species + temperature. */
#define BN_MAX_SYSTEM 64
#define BN_MAX_REACTIONS 1024

typedef struct bn_network bn_network; /* opaque; tables immutable after create */

/* Network description (all HOST pointers, read during bn_network_create). */
typedef struct {
  int32_t n_species;        /* N >= 1, N + 1 <= BN_MAX_SYSTEM */
  int32_t n_reactions;      /* R >= 1, R <= BN_MAX_REACTIONS */
  const int32_t *mass;      /* [N] mass numbers A_i >= 1 */
  const int32_t *reactants; /* [R][3] species index per slot, -1 = empty;
                               a repeated index is a multiplicity (2B = B,B,-1);
                               at least one slot in use */
  const int32_t *products;  /* [R][3] same convention (may be all -1) */
  const double *coef;       /* [R][7] a0..a6 of the rate fit */
  const double *q;          /* [R] heat released per reaction event */
  double c_v;               /* specific heat, > 0 */
  const double *screen;     /* [R] or NULL: strengths h_r of a synthetic
                               screening factor, the rate of reaction r being
                               multiplied by exp(h_r G) with
                               G = sqrt(rho (1 + sum_j A_j^2 Y_j)) T^(-3/2)
                               (the paper's network code screens its rates,
                               Sec. 2; this stands in for it).  A screened
                               network burns through burn_batch / burn_batch_ex
                               only (the persistent, source, adjoint and
                               autotune entry points return BN_EUNSUPPORTED) */
} bn_network_desc;

/* Validate `desc` (indices in range, every reaction conserves mass number,
 * finite coefficients, c_v > 0), build the device tables and return a handle
 * in *out.  Returns BN_SUCCESS, BN_EINVAL, BN_EUNSUPPORTED, BN_ENOMEM or
 * BN_EHIP.  The handle is bound to the device current at creation.
 * An unscreened network of more than 16 components also gets the areas in
 * which its persistent launches (burn_batch_multi, _noalloc) keep every
 * cell's Jacobian between refreshes (shapes that factor in LDS): 16 n^2
 * doubles per compute unit for n <= 32, else 8 n^2 (16 MB for n = 22, 43 MB
 * for n = 51 on 256 units), held until bn_network_destroy; if that
 * allocation fails the launches assemble the Jacobian at every
 * factorization instead (same results).  Two persistent launches of such a
 * network must not be in flight at once (they share its areas). */
int bn_network_create(const bn_network_desc *desc, bn_network **out);

/* Free the handle and its device tables (NULL is a no-op).  The caller must
 * make sure no enqueued burn still uses it. */
void bn_network_destroy(bn_network *net);

/* Number of species / reactions of a handle (-1 for NULL). */
int bn_network_n_species(const bn_network *net);
int bn_network_n_reactions(const bn_network *net);

/* Burn n_cells independent cells from t = 0 to t = dt.
 *   state    DEVICE [N][n_cells]  molar abundances Y, in/out
 *   rho      DEVICE [n_cells]     density (> 0)
 *   T        DEVICE [n_cells]     temperature (> 0), in/out
 *   dt > 0, rtol > 0, atol >= 0   end time and tolerances (atol applies to
 *                                 every component, temperature included)
 *   log_mult DEVICE [R] or NULL   p_r: lambda_r is multiplied by exp(p_r)
 *   status   DEVICE [n_cells] or NULL              BN_CELL_* per cell
 *   counters DEVICE [BN_N_COUNTERS][n_cells] or NULL
 *   stream   hipStream_t or NULL
 * A cell that fails keeps its last accepted (Y, T); a BAD_INPUT or
 * NONFINITE cell is left unchanged.  n_cells == 0 is a no-op.
 * Returns BN_SUCCESS or a negative code (nothing enqueued). */
int burn_batch(const bn_network *net, int64_t n_cells, double *state, const double *rho,
               double *T, double dt, double rtol, double atol, const double *log_mult,
               int32_t *status, int32_t *counters, void *stream);

/* Optional knobs for burn_batch_ex (zero-initialise, then set fields). */
typedef struct {
  int32_t max_steps;      /* accepted-step budget per cell; <= 0 means 100000 */
  int32_t lanes_per_cell; /* 0 = the network's launch choice (tuned or default);
                             otherwise 4, 8, 16, 32 or 64 */
  int32_t block_waves;    /* 0 = automatic; waves per workgroup (tuning) */
  int32_t order_cells;    /* burn_batch_multi only: 1 = hand each network's
                             cells out costliest first (see there), 0 = in
                             index order; ignored by the other calls */
} bn_burn_opts;

/* burn_batch with knobs (opts may be NULL: defaults). */
int burn_batch_ex(const bn_network *net, int64_t n_cells, double *state, const double *rho,
                  double *T, double dt, double rtol, double atol, const double *log_mult,
                  int32_t *status, int32_t *counters, const bn_burn_opts *opts, void *stream);

/* burn_batch_ex with a constant per-cell source added to the right-hand
 * side, dy/dt = f(y) + A_adv: the advective forcing a simplified-SDC coupling
 * hands to each zone's reaction integration (Sec. 2 of the paper: the
 * network couples to the hydrodynamics through such integration schemes).
 *   source  DEVICE [N+1][n_cells]  constant rates for the abundances (rows
 *                                  0..N-1) and the temperature (row N)
 * The source does not enter the Jacobian.  A non-finite source entry makes
 * the cell BN_CELL_BAD_INPUT.  opts as for burn_batch_ex (its lanes_per_cell
 * must select one of 4, 16, 32 or 64 lanes, or be 0). */
int burn_batch_sdc(const bn_network *net, int64_t n_cells, double *state, const double *rho,
                   double *T, double dt, double rtol, double atol, const double *log_mult,
                   const double *source, int32_t *status, int32_t *counters,
                   const bn_burn_opts *opts, void *stream);

/* ---- Persistent multi-network burn ------------------------------------ */

/* One network's batch of cells inside a multi-network launch.  The arrays
 * follow the conventions of burn_batch. */
typedef struct {
  const bn_network *net;
  int64_t n_cells;
  double *state;          /* DEVICE [N][n_cells], in/out */
  const double *rho;      /* DEVICE [n_cells] */
  double *T;              /* DEVICE [n_cells], in/out */
  const double *log_mult; /* DEVICE [R] or NULL */
  int32_t *status;        /* DEVICE [n_cells] or NULL */
  int32_t *counters;      /* DEVICE [BN_N_COUNTERS][n_cells] or NULL */
} bn_batch_item;

#define BN_MAX_ITEMS 8

/* Device workspace burn_batch_multi needs for n_items items (one 8-byte
 * queue counter per item, rounded up to 256 bytes). */
size_t burn_batch_multi_workspace_bytes(int32_t n_items);

/* Device workspace of burn_batch_multi with opts->order_cells = 1: the bytes
 * above plus, per item with cells, 256 four-byte bucket counters, 8 queue
 * counters of 8 bytes and 8 (N + 8) bytes per cell (the probe's step size, the cell's position, and
 * position-ordered copies of its state, T, rho, status and counters), each
 * region on a 256-byte boundary.  items is HOST [n_items]; NULL gives the
 * unordered size. */
size_t burn_batch_multi_order_workspace_bytes(int32_t n_items, const bn_batch_item *items);

/* Burn the cells of up to BN_MAX_ITEMS networks (same dt and tolerances) in
 * ONE persistent kernel launch with a device work queue (one per
 * waves-per-SIMD class of the networks' persistent choices, see
 * bn_network_set_persistent_launch): the grid is sized to
 * the GPU, and each lane group that finishes a cell takes the next unstarted
 * cell of the current network, so cells of uneven stiffness and networks of
 * different sizes share the machine without per-batch tails.  Per-cell
 * results are bitwise identical to burn_batch with the same launch shape (a
 * cell's arithmetic depends on the shape, never on where or when it runs).
 *   items      HOST [n_items]   the batches (networks on the current device)
 *   opts       HOST or NULL     max_steps and block_waves are honoured;
 *                               lanes_per_cell must be 0 (each network uses its
 *                               launch choice, see bn_network_autotune);
 *                               order_cells 0 or 1 (else BN_EINVAL)
 *   workspace  DEVICE           >= burn_batch_multi_workspace_bytes(n_items)
 *                               bytes (with order_cells = 1:
 *                               burn_batch_multi_order_workspace_bytes), 8-byte
 *                               aligned, caller-owned; it must not be used by
 *                               another launch in flight
 * A network of more than 16 components keeps its cells' Jacobians between
 * refreshes in areas of its own (bn_network_create); two launches of one
 * such network must not be in flight at once.
 * With order_cells = 1 each network's queue hands out its cells in order of
 * increasing initial step size h0 (the integrator's first-step estimate
 * 0.01 ||y0|| / ||f(y0)||, the same weighted norms as in the burn), so the
 * stiffest cells start first and the launch ends on short ones; a probe
 * kernel evaluates one right-hand side per cell, a counting sort over 128
 * buckets of log2 h0 (two per octave) builds the order, the cells' arrays
 * are copied into the workspace in that order before the burn (so cells
 * that run at nearby times share memory lines) and copied back after it.
 * The order is dealt round-robin into 8 parts, one per XCD of the MI355X:
 * a workgroup takes the cells of its own XCD's part first (they then share
 * that XCD's L2) and those of the other parts when its own is exhausted.
 * Only the order of work changes, not any cell's result.
 * The call enqueues small counter-reset kernels, the order kernels when
 * asked, and the burn kernel on `stream` and nothing else (no allocation, no
 * memset, no synchronization), so a sequence of calls can be captured into a
 * HIP graph and replayed.
 * Returns BN_SUCCESS or a negative code (nothing enqueued). */
int burn_batch_multi(int32_t n_items, const bn_batch_item *items, double dt, double rtol,
                     double atol, const bn_burn_opts *opts, void *workspace,
                     size_t workspace_bytes, void *stream);

/* Bytes of device scratch burn_batch_multi_noalloc has on each device. */
#define BN_NOALLOC_SCRATCH_BYTES (64u << 20)

/* burn_batch_multi for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments and results as burn_batch_multi, without the workspace:
 * the queue counters and (order_cells = 1) the order and staging arrays live
 * in a static device array of BN_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on every device it runs on until the process ends.  The call itself
 * allocates nothing (no hipMalloc, no library allocation); its counters are
 * cleared by kernels at the start of every call.  Calls on one device share
 * that array: two calls in flight on the same device at once (on different
 * streams, or from different threads without ordering) race and their results
 * are undefined.  A launch that needs more scratch than the array holds
 * (burn_batch_multi_order_workspace_bytes, or burn_batch_multi_workspace_bytes
 * without ordering) is rejected with BN_EINVAL and a message naming both
 * sizes; nothing is enqueued.  Returns BN_SUCCESS or a negative code. */
int burn_batch_multi_noalloc(int32_t n_items, const bn_batch_item *items, double dt,
                             double rtol, double atol, const bn_burn_opts *opts, void *stream);

/* ---- Generated per-network kernels ------------------------------------- */

/* The paper generates the right-hand side and analytic Jacobian of each
 * network as code (Sec. 2, "Arbitrary Network Generation").  These calls do
 * the same for the burn: the library writes a HIP source in which the rates,
 * the right-hand side and the Jacobian of one network are straight-line code
 * (stoichiometry, rate coefficients and sparsity as compile-time constants;
 * every sum in ascending reaction order, as in the definitions), compiles it
 * for gfx950 at run time (hiprtc) together with the integrator, and launches
 * it in place of the table-driven kernels.  The integrator, its decisions,
 * statuses and counters are those of burn_batch.
 *
 * Layout of the generated body: a cell is owned by one lane (systems of up
 * to 8 components) or a pair of lanes (up to 16): each lane keeps its rows of
 * the LU factors in registers, with the fill pattern of I - cJ under diagonal
 * pivots fixed at compile time, and checks at every column that partial
 * pivoting chooses the diagonal; a cell whose factorization would pivot
 * elsewhere finishes it with row interchanges in a per-lane scratch area
 * (the pivots are always those of partial pivoting, first largest magnitude).
 * One workgroup of four waves per compute unit; the cells come from a device
 * queue as in burn_batch_multi. */
#define BN_BODY_TABLE 0     /* the table-driven kernels (any network) */
#define BN_BODY_GENERATED 1 /* the network's generated kernel */

/* The generated source for a network (host only; no device needed).
 *   lanes_per_cell  0 = automatic (1 up to 8 components, else 2 up to 16),
 *                   or 1 or 2
 * Writes at most cap bytes (NUL-terminated) into buf (may be NULL) and the
 * full size including the NUL into *len (may be NULL).  BN_EUNSUPPORTED for
 * screened networks and systems above 16 components. */
int bn_codegen_source(const bn_network_desc *desc, int32_t lanes_per_cell, char *buf, size_t cap,
                      size_t *len);

/* Compile a network's generated kernel into the cache directory cache_dir
 * (host only; no device needed), so that bn_network_generate finds it there.
 * The cache file is named by a hash of the source, the integrator body, the
 * compiler options and the compiler version.  BN_EHIP with the compiler log
 * in bn_last_error if compilation fails. */
int bn_codegen_prebuild(const bn_network_desc *desc, int32_t lanes_per_cell,
                        const char *cache_dir);

/* Generate, compile (or take from cache_dir, which may be NULL for no cache;
 * a compiled kernel is written there when the directory is writable) and
 * load the network's kernel on the network's device, allocate its
 * workspaces (per lane of the launch grid: the Jacobian's nonzero rows and a
 * pivoting scratch area of n^2 + 4n doubles; they belong to the network and
 * are freed by bn_network_destroy) and select BN_BODY_GENERATED.  The
 * device must be gfx950.  From then on burn_batch, burn_batch_ex (with
 * lanes_per_cell 0) and burn_batch_multi use the generated kernel for this
 * network; the sensitivity, source-term and screened calls keep the
 * table-driven kernels.  Two launches of one generated network must not be
 * in flight at once (they share its workspaces).  Compilation takes seconds;
 * the call is synchronous. */
int bn_network_generate(bn_network *net, int32_t lanes_per_cell, const char *cache_dir);

/* Select the body a network's burns use: BN_BODY_TABLE, or
 * BN_BODY_GENERATED (after bn_network_generate; else BN_EINVAL). */
int bn_network_set_body(bn_network *net, int32_t body);

/* The selected body, and the lanes per cell of the generated kernel (0 if
 * there is none).  Either pointer may be NULL. */
int bn_network_get_body(const bn_network *net, int32_t *body, int32_t *lanes_per_cell);

/* ---- Launch-shape autotuner -------------------------------------------- */

typedef struct {
  int32_t lanes_per_cell; /* L: lanes that own one cell */
  int32_t slots_per_lane; /* S: system components per lane (n <= L*S) */
  int32_t block_waves;    /* waves per workgroup */
  int32_t status;         /* 0 measured, else the launch error (skipped) */
  double ms;              /* kernel time on the sample */
} bn_tune_result;

/* Time every launch shape that fits this network on a sample of cells (the
 * caller's arrays are only read: the sample is burned in library-allocated
 * scratch copies) and make the fastest the network's launch choice, used by
 * burn_batch (lanes_per_cell = 0) and burn_batch_multi.  Each shape runs
 * once to warm up, then is timed once, or three times (the fastest counts)
 * when a run takes under 10 ms.  Synchronizes
 * `stream`; allocates device memory; not for use under graph capture.
 *   state, rho, T  DEVICE sample in the burn_batch layout (n_cells >= 1)
 *   results        HOST [max_results] or NULL; *n_results = entries written
 * Returns BN_SUCCESS or a negative code. */
int bn_network_autotune(bn_network *net, int64_t n_cells, const double *state,
                        const double *rho, const double *T, double dt, double rtol,
                        double atol, const double *log_mult, int32_t max_steps,
                        bn_tune_result *results, int32_t max_results, int32_t *n_results,
                        void *stream);

/* Set / read the network's launch choice directly (e.g. from a cached
 * tuning).  Setting validates the shape against the system size. */
int bn_network_set_launch(bn_network *net, int32_t lanes_per_cell, int32_t slots_per_lane,
                          int32_t block_waves);
int bn_network_get_launch(const bn_network *net, int32_t *lanes_per_cell,
                          int32_t *slots_per_lane, int32_t *block_waves);

/* The persistent kernel's launch choice for a network: lanes per cell,
 * slots per lane, the waves per SIMD its instance is compiled for (2: shapes
 * (8,1) (16,1) (32,1) (64,1); 1: (4,4) (16,2) (32,1) (64,1)) and the waves per
 * workgroup.  burn_batch_multi runs each network with its choice and gives
 * the networks of each waves-per-SIMD class a launch of their own (one
 * launch per class, in a call that has both). */
typedef struct {
  int32_t lanes_per_cell;
  int32_t slots_per_lane;
  int32_t waves_per_simd; /* 2 or 1 */
  int32_t block_waves;    /* waves per workgroup, 1..4 */
  int32_t status;         /* 0 measured, else the error of that candidate (skipped) */
  double ms;              /* time of an ordered persistent launch of the sample */
} bn_persistent_tune_result;

/* Time every persistent launch choice that fits this network (shapes with
 * L*S >= n and not mostly padding, both waves-per-SIMD classes, 1, 2 and 4
 * waves per workgroup) on a sample of cells, each as an ordered
 * burn_batch_multi launch of the sample alone, and make the fastest the
 * network's persistent choice (and its time per cell the network's cost
 * estimate), unless it beats the choice derived without tuning by less than
 * 3 % (then that one is kept: a sample's tail weighs more than a full
 * batch's).  The candidates are the table-driven kernel's: a network whose
 * generated kernel is selected is timed with the table body and keeps its
 * selection.  The caller's arrays are only read.  Synchronizes `stream`;
 * allocates device memory; not for use under graph capture.
 *   state, rho, T  DEVICE sample in the burn_batch layout (n_cells >= 1)
 *   results        HOST [max_results] or NULL; *n_results = entries written
 * Returns BN_SUCCESS or a negative code (the previous choice is kept). */
int bn_network_autotune_persistent(bn_network *net, int64_t n_cells, const double *state,
                                   const double *rho, const double *T, double dt, double rtol,
                                   double atol, const double *log_mult, int32_t max_steps,
                                   bn_persistent_tune_result *results, int32_t max_results,
                                   int32_t *n_results, void *stream);

/* Set the persistent choice directly (e.g. from a cached tuning);
 * lanes_per_cell = 0 clears it.  ms_per_cell > 0 also sets the network's
 * cost estimate (the order in which a multi-network launch takes its
 * networks).  Get reports the choice a launch would use now (the tuned one,
 * or the one derived from the plain choice and the LDS footprint). */
int bn_network_set_persistent_launch(bn_network *net, int32_t lanes_per_cell,
                                     int32_t slots_per_lane, int32_t waves_per_simd,
                                     int32_t block_waves, double ms_per_cell);
int bn_network_get_persistent_launch(const bn_network *net, int32_t *lanes_per_cell,
                                     int32_t *slots_per_lane, int32_t *waves_per_simd,
                                     int32_t *block_waves);

/* ---- Sensitivities: discrete adjoint in the log-rate multipliers ------- */

/* The paper asks how a burn responds to the individual reaction rates
 * (Sec. 1).  These calls differentiate, cell by cell, the end state
 * (Y, T)(dt) and the released energy E = c_v (T(dt) - T0) with respect to the
 * network's log-rate multipliers p_r (lambda_r -> e^{p_r} lambda_r).  The
 * differentiated map is the burn replayed on its own frozen schedule: a
 * recording run (the same integrator as burn_batch) fixes every accepted
 * step's order, step size and history rescale ratio, and the replay solves
 * every corrector exactly (full Newton to a weighted increment <= 1e-10).
 * The replay's end state is what the forward call returns; it agrees with
 * burn_batch's to the integrator's Newton tolerance.  The reverse sweep needs
 * the corrected state of every replayed step: from a pool in the workspace
 * where the replay kept them, or else recomputed segment by segment from a
 * checkpoint of the history taken every 16 accepted steps (the same doubles
 * either way, so the gradients do not depend on the pool's size).
 *
 * Workspace: caller-provided DEVICE memory of
 * burn_batch_adjoint_workspace_bytes(net, n_cells, max_steps) bytes, 8-byte
 * aligned, holding per cell the schedule (20 bytes per step of max_steps),
 * a checkpoint of 7 (N + 1) doubles every 16 steps, the corrected states of
 * one 16-step segment for the reverse sweep, and the order in which the
 * replay and the reverse sweep take the cells (most recorded steps first,
 * so that the cells sharing a wave have similar step counts; 12 bytes per
 * cell, and 8 bytes per cell for the pool offsets), and the recording run's
 * queue counter (the recording run takes cells from a device queue on a
 * grid sized to the GPU, as burn_batch_multi does); the forward call fills
 * it, the backward call reads it (same net, cells, dt, tolerances, log_mult,
 * max_steps and workspace_bytes), and it must not be shared by calls in
 * flight.  Bytes beyond that minimum are the pool of corrected states: the
 * replay keeps the states of the cells that fit there (in cell index order,
 * 8 (N + 1) bytes per accepted step) and the reverse sweep then skips their
 * recomputation.  burn_batch_adjoint_states_bytes(net, S) is the pool that
 * holds S accepted steps; the accepted steps of a batch are the sum over its
 * OK cells of counter 0 of a previous forward call.
 * max_steps (1 .. 1,000,000) bounds the accepted steps of a cell; a cell that
 * needs more ends with BN_CELL_MAX_STEPS and a zero gradient.
 * Networks with more than BN_ADJOINT_MAX_REACTIONS reactions are not
 * supported (BN_EUNSUPPORTED). */
#define BN_ADJOINT_MAX_REACTIONS 256

size_t burn_batch_adjoint_workspace_bytes(const bn_network *net, int64_t n_cells,
                                          int32_t max_steps);

/* Bytes of a pool of corrected states for total_steps accepted steps
 * (8 (N + 1) total_steps), to append to the minimum workspace. */
size_t burn_batch_adjoint_states_bytes(const bn_network *net, int64_t total_steps);

/* Forward: recording run plus replay.
 *   state0, T0  DEVICE [N][n_cells], [n_cells]  initial state (read only)
 *   rho         DEVICE [n_cells]
 *   log_mult    DEVICE [R] or NULL
 *   state_out   DEVICE [N][n_cells]  replayed end abundances
 *   T_out       DEVICE [n_cells]     replayed end temperature
 *   E_out       DEVICE [n_cells]     c_v (T_out - T0)
 *   status      DEVICE [n_cells]     BN_CELL_* (required: the backward call
 *                                    reads it)
 *   counters    DEVICE [BN_N_COUNTERS][n_cells] or NULL (recording run)
 *   replay_iters DEVICE [2][n_cells] or NULL  per cell, the replay's Newton
 *                                    iterations (row 0) and Newton-matrix
 *                                    factorizations (row 1)
 * A cell that fails keeps the recording run's last accepted state. */
int burn_batch_adjoint_forward(const bn_network *net, int64_t n_cells, const double *state0,
                               const double *rho, const double *T0, double dt, double rtol,
                               double atol, const double *log_mult, int32_t max_steps,
                               double *state_out, double *T_out, double *E_out,
                               int32_t *status, int32_t *counters, int32_t *replay_iters,
                               void *workspace, size_t workspace_bytes, void *stream);

/* Backward: per-cell vector-Jacobian product.
 *   gY    DEVICE [N][n_cells]   cotangent of the end abundances
 *   gE    DEVICE [n_cells]      cotangent of E
 *   grad  DEVICE [R][n_cells]   out: sum_i gY_i dY_i/dp_r + gE dE/dp_r per
 *                               cell (zero for a cell whose status is not OK)
 *   status DEVICE [n_cells]     as written by the forward call */
int burn_batch_adjoint_backward(const bn_network *net, int64_t n_cells, const double *state0,
                                const double *rho, const double *T0, double dt, double rtol,
                                double atol, const double *log_mult, int32_t max_steps,
                                const double *gY, const double *gE, double *grad,
                                const int32_t *status, void *workspace, size_t workspace_bytes,
                                void *stream);

/* Forward and backward in one call. */
int burn_batch_adjoint(const bn_network *net, int64_t n_cells, const double *state0,
                       const double *rho, const double *T0, double dt, double rtol, double atol,
                       const double *log_mult, int32_t max_steps, const double *gY,
                       const double *gE, double *state_out, double *T_out, double *E_out,
                       double *grad, int32_t *status, int32_t *counters,
                       int32_t *replay_iters, void *workspace, size_t workspace_bytes,
                       void *stream);

/* Thread-local description of the last failed call on this thread ("" if
 * none); valid until the next call from the same thread. */
const char *bn_last_error(void);

/* Library version string. */
const char *bn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MI355X_BURN_H */
