/*
 * ssqa.h -- C ABI of the MI355X (gfx950) stochastic simulated quantum annealing library.
 *
 * The library anneals a fully connected integer Ising model
 *     H(sigma) = - sum_i h_i sigma_i - sum_{i<j} J_ij sigma_i sigma_j          (paper, Eq. 1)
 * with R Trotter replicas per trial coupled in a ring (Section 3.1, Eq. 4-5, Fig. 2) using the
 * SSQA spin update (Section 3.2, Eq. 6a-c), on T independent trials at once.
 *
 * Integer model.  Every quantity is an integer at one scale S chosen by the caller: h, J, the noise
 * amplitude n_rnd, J_perp(t), I_0(t) and alpha.  For a graph-isomorphism problem (Section 4) the
 * coefficients are quarter-integers and J_perp moves in sixths, so S = 12 makes all of them exact;
 * ssqa_gi_to_ising builds such a model.  All arithmetic is exact: a run is a deterministic function
 * of (problem, parameters, seed).
 *
 * Random stream.  Philox4x32-10 (Salmon et al., SC'11) with key (low, high 32 bits of seed) and
 * counter (tag, i >> 7, k, b): tag 0 gives the initial spins, tag t+1 the noise r(t) of the update
 * t -> t+1; spin i uses bit (i & 31) of output word (i & 127) >> 5, and bit 1 means +1.  The result
 * therefore does not depend on how the work is tiled or launched.
 *
 * Initial state: sigma(0) from tag 0, Is(0) = 0 where sigma = +1 and -alpha where sigma = -1, and
 * sigma(t - d) = sigma(0) for t < d.
 *
 * Memory and streams.  Host arrays passed to ssqa_create_problem and the schedules are copied before
 * the call returns; the caller keeps ownership.  Output arrays of ssqa_anneal and ssqa_energy are
 * caller-owned DEVICE pointers on the problem's device.  ssqa_anneal and ssqa_energy are
 * asynchronous with respect to the host on the given HIP stream (NULL = the default stream).
 *
 * Errors.  Every call returns an ssqa_status; nothing throws across the ABI.  On failure no output
 * is written, and ssqa_last_error() returns a message for the calling thread.
 */
#ifndef SSQA_H
#define SSQA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ssqa_status {
    SSQA_OK = 0,
    SSQA_EINVAL = -1,  /* invalid argument: null pointer, size or parameter out of range, J not symmetric */
    SSQA_ENOMEM = -2,  /* device or host allocation failed */
    SSQA_ERANGE = -3,  /* an int32 intermediate (field, counter sum, energy) could overflow */
    SSQA_EDEVICE = -4, /* HIP runtime error: no device, launch or copy failure */
    SSQA_ENOTSUP = -5  /* valid request outside what this build supports (e.g. R > 64) */
} ssqa_status;

/* Human-readable name of a status code (static storage). */
const char* ssqa_status_string(ssqa_status s);

/* Message describing the last failure on the calling thread ("" if none). */
const char* ssqa_last_error(void);

/* ------------------------------------------------------------------------------------------- */
/* Problem: the integer Ising model, resident on one device.                                   */
/* ------------------------------------------------------------------------------------------- */

typedef struct ssqa_problem* ssqa_problem_t;

/*
 * Copy an integer Ising model (paper, Eq. 1) to device `device` and prepare it for the sweep.
 *   n_spins : N >= 1, at most 16384.
 *   h       : host int32 [N], the spin biases h_i.
 *   J       : host int32 [N * N] row-major, the couplings J_ij; must be symmetric with a zero
 *             diagonal (only i != j pairs couple, Eq. 1 sums over i < j).
 *   out     : receives the handle.
 * J is stored as P signed int8 planes with J = sum_p 256^p J_p (P = 1 when every |J_ij| <= 127),
 * zero-padded to a multiple of 128 rows and columns, and additionally as fp4 (e2m1) when every J_ij is
 * one of 0, +-1, +-2, +-3, +-4, +-6 and B + 128 < 2^22, where B = max_i (|h_i| + 2 sum_j |J_ij|).  An
 * anneal uses the fp4 copy only while B + n_rnd + (1 + mode) max_t |J_perp(t)| + 128 < 2^22: every
 * partial sum of its fp32 accumulation is then an integer inside [2^23, 2^24), so the field product is
 * exact (Eq. 6a-b need the field exactly).
 * Fails with SSQA_EINVAL for a bad size, pointer or non-symmetric J, and with SSQA_ERANGE when
 * 2 * sum_i |h_i| + sum_ij |J_ij| >= 2^30 (energies and fields must stay inside int32).
 */
ssqa_status ssqa_create_problem(int32_t n_spins, const int32_t* h, const int32_t* J, int32_t device,
                                ssqa_problem_t* out);

/* Release the problem's device memory.  NULL is ignored.  No call may still be using it. */
void ssqa_destroy_problem(ssqa_problem_t problem);

/* N, the number of int8 planes P, the padded size of the device layout, and 1 when the fp4 copy of
 * J exists (operand_format 2 is then available to anneals whose noise and coupling keep the bound above,
 * and is what operand_format 0 picks for them), else 0.  A NULL handle gives 0. */
int32_t ssqa_problem_spins(ssqa_problem_t problem);
int32_t ssqa_problem_planes(ssqa_problem_t problem);
int32_t ssqa_problem_padded(ssqa_problem_t problem);
int32_t ssqa_problem_fp4_exact(ssqa_problem_t problem);

/* ------------------------------------------------------------------------------------------- */
/* Annealing.                                                                                  */
/* ------------------------------------------------------------------------------------------- */

#define SSQA_NO_TARGET INT64_MIN

/*
 * State of an anneal after t cycles, in a layout that does not depend on how the library tiles the
 * work (caller-owned DEVICE buffers on the problem's device):
 *   counters : int8 [T * R * N], Is(t) of spin i of replica k of trial b at (b * R + k) * N + i;
 *   history  : uint32 [T * R * d * W] with W = ceil(N / 32), sigma(t - s) for s = 1 .. d at
 *              ((b * R + k) * d + (s - 1)) * W + (i >> 5), bit i & 31, bit 1 meaning +1; unused
 *              (may be NULL) when d = 0.
 * sigma(t) itself is the sign of the counters (Eq. 6c).  The random stream is keyed by the absolute
 * cycle, so an anneal resumed from a checkpoint at cycle t continues bit for bit as if uninterrupted.
 */
typedef struct ssqa_anneal_state {
    int8_t* counters;
    uint32_t* history;
} ssqa_anneal_state;

typedef struct ssqa_anneal_params {
    int32_t replicas;          /* R >= 1 (Eq. 4); replica k couples to replica (k+1) mod R      */
    int32_t trials;            /* T >= 1 independent trials                                     */
    int32_t cycles;            /* SC >= 0 annealing cycles (updates of all N*R spins, Sec. 3.2) */
    int32_t delay;             /* d in [0, 6]: the coupling reads sigma(t - d) (Eq. 6a)         */
    int32_t alpha;             /* alpha >= 1: counter top is I_0 - alpha (Eq. 6b)               */
    int32_t noise_amp;         /* n_rnd >= 0 at the integer scale (Eq. 6a)                      */
    int32_t coupling_mode;     /* 0: J_perp(t) sigma_{i,k+1}(t-d) as printed in Eq. 6a;
                                  1: J_perp(t) (sigma_{i,k-1}(t-d) + sigma_{i,k+1}(t-d))          */
    int32_t cycles_per_launch; /* 0: all cycles in one persistent launch; k > 0: a host loop of
                                  launches of at most k cycles (state kept in device memory)     */
    const int32_t* jperp;      /* host int32 [cycles]: J_perp(t) at the integer scale           */
    const int32_t* i0;         /* host int32 [cycles]: I_0(t), 1 <= alpha <= I_0(t) <= 127     */
    uint64_t seed;             /* Philox key                                                    */
    int64_t target_energy;     /* E* for first_hit, or SSQA_NO_TARGET                           */
    int32_t block_columns;     /* columns (whole trials) per workgroup: 0 = automatic (a tiling the
                                  autotuner recorded for this shape, else: 64 when R <= 64 and the
                                  bit planes fit in LDS, else 32; 128 when the operands are fp4 or J
                                  fits one int8 plane, R divides 128, the problem pads to at least
                                  1024 rows (1536 for ssqa_anneal, which also needs at least two
                                  128-column blocks per CU) and the planes fit in LDS), or
                                  32 / 64 / 128 (128 with int8 operands needs every |J_ij| <= 127,
                                  else SSQA_ENOTSUP).  A tiling choice only: results do not depend
                                  on it                                                            */
    int32_t operand_format;    /* field-product operands: 0 = automatic (fp4 when the problem has an
                                  fp4 copy and B + n_rnd + (1 + mode) max_t |J_perp(t)| + 128 < 2^22,
                                  see ssqa_create_problem, else int8 planes); 1 = int8 planes; 2 = fp4
                                  (e2m1, fp32 accumulation, exact under the same conditions;
                                  SSQA_ENOTSUP otherwise).  Results do not depend on it            */
    int32_t start_cycle;       /* 0 for a fresh anneal; t0 in (0, cycles]: continue from the state
                                  `resume` holds after t0 cycles (best_energy and first_hit are then
                                  read as well as written: they must hold that run's values)      */
    int32_t stop_cycle;        /* 0 or cycles: run to the end (including the energy of sigma(SC));
                                  t1 in (start_cycle, cycles): stop after cycle t1 - 1            */
    const ssqa_anneal_state* resume;   /* required when start_cycle > 0, else ignored            */
    int32_t split_rows;        /* ssqa_anneal only: the row-split form (each trial's rows spread over
                                  row groups of workgroups, one launch per cycle; Sec. 3.2's update of
                                  all N R spins per cycle is unchanged): 0 = automatic (taken from 1280
                                  padded rows when the trials fill at most 16 column blocks of 32 or 64
                                  columns, from 2048 when they fill at most 64), -1 = never, k > 0 =
                                  from k padded rows on.  Only for fresh runs to the end (start_cycle
                                  = 0, stop_cycle = 0 or cycles, no checkpoint) on blocks of at most
                                  64 columns (block_columns 0, 32 or 64); other runs,
                                  ssqa_anneal_noalloc, batches and served requests ignore it.  The
                                  split form enqueues one launch per cycle, so the call returns once
                                  they are all queued (a few microseconds of host time per cycle).
                                  A scheduling choice only: results do not depend on it          */
} ssqa_anneal_params;

typedef struct ssqa_anneal_outputs {
    int64_t* best_energy;      /* device int64 [T]: min over replicas and t in [0, SC] of H_p    */
    int32_t* first_hit;        /* device int32 [T]: first t whose best replica has H_p == target,
                                  -1 if never (or no target)                                    */
    int32_t* energy_trace;     /* device int32 [(SC + 1) * T * R] or NULL: H_p of replica k of
                                  trial b at cycle t at index (t * T + b) * R + k                */
    int8_t* final_is;          /* device int8 [T * R * N] or NULL: Is(SC) at (b * R + k) * N + i */
    const ssqa_anneal_state* checkpoint;   /* or NULL: receives the state after the last cycle run
                                  (cycle stop_cycle, or SC)                                        */
} ssqa_anneal_outputs;

/*
 * Run SSQA (paper, Section 3.2, Eq. 6a-c) for `cycles` cycles on `trials` independent trials of
 * `replicas` coupled replicas, all N * R spins of a trial updated synchronously every cycle:
 *   I  = h_i + sum_j J_ij sigma_{j,k}(t) + n_rnd r_{i,k}(t) + coupling
 *   Is = I_0(t) - alpha if Is + I >= I_0(t);  -I_0(t) if Is + I < -I_0(t);  Is + I otherwise
 *   sigma_{i,k}(t+1) = +1 if Is >= 0 else -1
 * The problem Hamiltonian H_p (Eq. 5) of every replica is evaluated at t = 0 .. SC (one extra field
 * pass after the last update) for best_energy, first_hit and the optional trace.
 * Asynchronous on `stream`; the host schedules are copied before return.  Requires
 * |J_perp(t)| <= 2^20 and n_rnd <= 2^20.  Returns SSQA_ENOTSUP when R exceeds the columns per
 * workgroup (64, or 32 for N above about 6500 with d = 1) or the bit planes do not fit in LDS.
 */
ssqa_status ssqa_anneal(ssqa_problem_t problem, const ssqa_anneal_params* params,
                        const ssqa_anneal_outputs* outputs, void* hip_stream);

/*
 * ssqa_anneal for callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, checks and results, bit for bit, but the anneal's device state (counters,
 * bit-plane history and schedules, in the layout ssqa_anneal would choose) lives in a fixed 64 MiB array
 * that the library holds on each device it runs this call on until the process ends.  Nothing is allocated:
 * no hipMalloc, no stream-ordered pool, no pinned staging.  The caller still passes the problem and the
 * output buffers.
 *   - An anneal whose state exceeds 64 MiB (about T * R * N bytes of counters, plus 1/8 of that per unit
 *     of delay d, plus 8 * SC bytes of schedules) fails with SSQA_ENOTSUP before any device work.
 *   - The host waits for the copy of the schedules into the array before returning (so the caller may
 *     free them); the anneal itself runs asynchronously on `hip_stream`.
 *   - Every call on a device shares that device's array and leaves its contents behind (nothing in it has
 *     to start at zero).  Calls on one stream are ordered; calls that overlap on one device (several
 *     streams or host threads) race on the array and must be serialised by the caller.
 */
ssqa_status ssqa_anneal_noalloc(ssqa_problem_t problem, const ssqa_anneal_params* params,
                                const ssqa_anneal_outputs* outputs, void* hip_stream);

/* ------------------------------------------------------------------------------------------- */
/* Autotuner: the tiling of the field product (Section 3.2's parallel update of all N * R spins) */
/* chosen by timing the legal candidates on the device.                                        */
/* ------------------------------------------------------------------------------------------- */

/* One tiling of an anneal: whole trials per workgroup of `block_columns` columns, and the operands of the
 * field product.  A tiling changes only speed, never results. */
typedef struct ssqa_tile {
    int32_t block_columns;     /* 32, 64 or 128 columns (trial-replica pairs) per workgroup          */
    int32_t trials_per_block;  /* 1 .. block_columns / R trials per workgroup                        */
    int32_t operand_format;    /* 1 = int8 planes, 2 = fp4 (as ssqa_anneal_params.operand_format)     */
    int32_t blocks;            /* workgroups of the launch: ceil(T / trials_per_block)               */
    double ms_per_cycle;       /* measured device time per cycle (0 when not measured)               */
} ssqa_tile;

/*
 * Time every legal tiling of the anneal `params` describes (block_columns and operand_format must be 0:
 * the tuner chooses them) on its first min(cycles, probe_cycles) cycles, on `hip_stream`, and record the
 * fastest in the process-wide cache under (device name, architecture and compute units; kernel build;
 * padded N, planes, R, T, d, coupling mode, epilogue variant, whether fp4 is exact).  Candidates: 32, 64
 * and 128 columns (128 with int8 operands for single-plane J only) where the replicas and the LDS allow,
 * whole-block packing and spreading the trials over 1, 2 or 4 workgroups per CU, fp4 (when exact) and int8
 * operands.  Up to
 * `capacity` timed candidates are written to `candidates` (host array), their number to `count` (may be
 * NULL), the chosen one to `chosen`.  Synchronises the stream; allocates and frees its own device memory.
 * Afterwards ssqa_anneal and ssqa_anneal_noalloc take the recorded tiling for requests of this shape with
 * block_columns = 0 and operand_format = 0.  Errors as for ssqa_anneal.
 */
ssqa_status ssqa_tune_anneal(ssqa_problem_t problem, const ssqa_anneal_params* params, int32_t probe_cycles,
                             void* hip_stream, ssqa_tile* candidates, int32_t capacity, int32_t* count,
                             ssqa_tile* chosen);

/*
 * Time the batched form of these anneals (arguments as for ssqa_batch_create, without outputs) on their first
 * min(cycles, probe_cycles) cycles for every padded size from which automatic blocks could take 128
 * columns (each distinct padded N of an anneal that could, and never), and record the fastest floor in the
 * cache under (device, kernel build, the batch's shape).  `wide_rows` receives it (0 = never); ms_per_cycle
 * (may be NULL) its time per cycle.  ssqa_batch_create then uses it for a batch of the same shape.
 */
ssqa_status ssqa_tune_batch(int32_t count, const ssqa_problem_t* problems, const ssqa_anneal_params* params,
                            int32_t probe_cycles, void* hip_stream, int32_t* wide_rows, double* ms_per_cycle);

/* The tiling ssqa_anneal would use for `params` (a recorded one for automatic requests, else the built-in
 * rules); `tuned` (may be NULL) receives 1 when it came from the cache.  No device work. */
ssqa_status ssqa_tune_lookup(ssqa_problem_t problem, const ssqa_anneal_params* params, ssqa_tile* tile,
                             int32_t* tuned);

/* Record `tile` for the shape of `params` (block_columns = operand_format = 0) without timing it;
 * SSQA_ENOTSUP when the tile cannot run that anneal. */
ssqa_status ssqa_tune_set(ssqa_problem_t problem, const ssqa_anneal_params* params, const ssqa_tile* tile);

/* Write every cached entry to a JSON file {"format": "ssqa-tune-1", "entries": [...]} (SSQA_EINVAL when it
 * cannot be written).  Entries of other devices and kernel builds are kept and written too. */
ssqa_status ssqa_tune_save(const char* path);

/* Merge the entries of a file written by ssqa_tune_save into the cache (an entry replaces one of the same
 * key); `loaded` (may be NULL) receives their number.  A file that does not parse, or any entry with a
 * missing or out-of-range field, fails with SSQA_EINVAL and leaves the cache unchanged.  Entries apply only
 * on the device and kernel build they name. */
ssqa_status ssqa_tune_load(const char* path, int32_t* loaded);

/* Number of cached entries; clearing the cache restores the built-in rules. */
int32_t ssqa_tune_entries(void);
void ssqa_tune_clear(void);

/* ------------------------------------------------------------------------------------------- */
/* Batched form: many anneals of uneven size in one persistent launch, replayed from a HIP graph.*/
/* ------------------------------------------------------------------------------------------- */

typedef struct ssqa_batch* ssqa_batch_t;

/*
 * Prepare `count` anneals to run together: anneal i applies params[i] to problems[i] and writes
 * outputs[i], with exactly the results ssqa_anneal would give for it alone (the random stream depends
 * only on the seed and the spin, replica, trial and cycle indices).  All problems must live on one
 * device; params[i].cycles_per_launch must be 0.  The library splits every anneal into blocks of whole
 * trials, orders all blocks by decreasing cost (N padded squared times cycles) and records one persistent
 * launch over that work list (one per distinct (alpha == 1, coupling mode) pair present) plus the optional
 * final-counter copies in a HIP graph.  Schedules are copied; problems, params' host arrays and the
 * output device buffers must stay valid until ssqa_batch_destroy.  Device state for all anneals is
 * allocated here.  Errors as for ssqa_anneal (the first failing anneal is named in ssqa_last_error()).
 */
ssqa_status ssqa_batch_create(int32_t count, const ssqa_problem_t* problems, const ssqa_anneal_params* params,
                              const ssqa_anneal_outputs* outputs, ssqa_batch_t* out);

/* Run the prepared anneals (a graph launch, asynchronous on `stream`).  May be called repeatedly; each
 * run starts every anneal from cycle 0 and overwrites its outputs.  Runs of one batch must not overlap. */
ssqa_status ssqa_batch_run(ssqa_batch_t batch, void* hip_stream);

/* Number of workgroups (column blocks) in the batch's work list. */
int32_t ssqa_batch_blocks(ssqa_batch_t batch);

/* Free the batch's graph and device state.  NULL is ignored.  No run may still be in flight. */
void ssqa_batch_destroy(ssqa_batch_t batch);

/* ------------------------------------------------------------------------------------------- */
/* Serving: continuous batching of anneal requests with memory-based admission.                */
/* ------------------------------------------------------------------------------------------- */

typedef struct ssqa_server* ssqa_server_t;

typedef struct ssqa_server_config {
    int32_t device;            /* device every request runs on                                   */
    int32_t cycles_per_step;   /* K >= 1: cycles every active request advances per step          */
    int32_t max_active;        /* at most this many requests on the device at once (1..65535)    */
    int64_t memory_budget;     /* bytes of device memory admitted requests may hold together     */
    int32_t split_rows;        /* a request whose N pads to at least this many rows (and whose block
                                  is narrower than 128 columns) spreads each trial's rows over row
                                  groups of workgroups, one launch per cycle (Section 3.2's parallel
                                  update of all N R spins over more of the chip); 0 = 4096, -1 = never */
} ssqa_server_config;

typedef struct ssqa_request {
    int32_t n_spins;           /* N, as for ssqa_create_problem                                   */
    const int32_t* h;          /* host int32 [N], copied at submit                                */
    const int32_t* J;          /* host int32 [N * N], symmetric, zero diagonal, copied at submit  */
    ssqa_anneal_params params; /* as for ssqa_anneal; cycles = the most cycles the request may run;
                                  schedules copied at submit; cycles_per_launch must be 0          */
    int32_t early_exit;        /* 1: retire at the first step boundary where some trial's best
                                  energy equals params.target_energy; 0: run all cycles           */
} ssqa_request;

typedef enum ssqa_request_state {
    SSQA_REQ_QUEUED = 0,
    SSQA_REQ_RUNNING = 1,
    SSQA_REQ_DONE = 2,
    SSQA_REQ_CANCELLED = 3,
    SSQA_REQ_FAILED = 4        /* e.g. SSQA_ENOMEM: the request alone exceeds the memory budget   */
} ssqa_request_state;

typedef struct ssqa_request_info {
    int32_t state;             /* ssqa_request_state                                              */
    int32_t status;            /* ssqa_status of a failed request                                 */
    int32_t cycles_done;       /* cycles the request has run                                      */
    int32_t trials;
    double submit_s, admit_s, done_s;  /* seconds since server creation (-1: not yet)            */
    int64_t memory_bytes;      /* device memory charged to the request while it runs              */
} ssqa_request_info;

typedef struct ssqa_server_stats_t {
    int32_t queued, active;
    int64_t memory_in_use;
    double spin_updates;       /* spin updates executed so far                                     */
    double elapsed_s;          /* seconds since server creation                                    */
} ssqa_server_stats_t;

/*
 * Create a request server (no device work until the first step).  The server is single-threaded:
 * calls on one server must not overlap.
 */
ssqa_status ssqa_server_create(const ssqa_server_config* config, ssqa_server_t* out);

/* Queue a request (first come, first served); `id` receives its handle. */
ssqa_status ssqa_server_submit(ssqa_server_t server, const ssqa_request* request, int64_t* id);

/*
 * One serving step on `stream`: admit queued requests in order while the slot limit and the memory
 * budget allow (a request that alone exceeds the budget fails with SSQA_ENOMEM), run K more cycles of
 * every active request in one launch (each continues from its own cycle; counters, delayed spins and
 * best energies stay on the device), read back the per-trial best energies and retire requests that
 * finished their cycles or, with early_exit, reached their target.  Synchronises `stream`.
 * `active` (may be NULL) receives the number of requests still running.  A request's results are the
 * same alone or among others: best and first hit per trial equal those of ssqa_anneal with the same
 * parameters (with early exit, best is the target for the trials that reached it by the retiring step).
 */
ssqa_status ssqa_server_step(ssqa_server_t server, void* hip_stream, int32_t* active);

/* State and timings of a request; with `best` (host int64 [T]) and `first_hit` (host int32 [T]) non-NULL,
 * also its per-trial results so far. */
ssqa_status ssqa_server_poll(ssqa_server_t server, int64_t id, ssqa_request_info* info, int64_t* best,
                             int32_t* first_hit);

/* Cancel a queued or running request (a running one is released at the next step). */
ssqa_status ssqa_server_cancel(ssqa_server_t server, int64_t id);

/* Queue length, active requests, memory in use and work done so far. */
ssqa_status ssqa_server_stats(ssqa_server_t server, ssqa_server_stats_t* stats);

/* Release every request's device memory and the server.  NULL is ignored. */
void ssqa_server_destroy(ssqa_server_t server);

/*
 * Problem Hamiltonian (Eq. 1 / Eq. 5) of `cols` spin configurations, exactly:
 *   spins    : device int8 [cols * N], configuration c at c * N + i, entries +1 or -1.
 *   energies : device int64 [cols].
 * Asynchronous on `stream`.
 */
ssqa_status ssqa_energy(ssqa_problem_t problem, const int8_t* spins, int32_t cols, int64_t* energies,
                        void* hip_stream);

/*
 * QMC Hamiltonian (Eq. 4) of `trials` trials of `replicas` replicas from their counters, exactly:
 *   H_c = sum_k H_p(sigma_k) - J_perp sum_k sum_i sigma_{i,k} sigma_{i,(k+1) mod R},
 * with sigma = +1 where the counter is >= 0 (Eq. 6c).
 *   counters : device int8 [trials * replicas * N] in the layout of ssqa_anneal's final_is.
 *   jperp    : J_perp at the integer scale.
 *   energies : device int64 [trials].
 * Asynchronous on `stream`.
 */
ssqa_status ssqa_qmc_energy(ssqa_problem_t problem, const int8_t* counters, int32_t trials, int32_t replicas,
                            int32_t jperp, int64_t* energies, void* hip_stream);

/* ------------------------------------------------------------------------------------------- */
/* Traditional simulated annealing: the SA baseline of Section 4.4 and Table 4.                  */
/* ------------------------------------------------------------------------------------------- */

/*
 * Serial single-spin Metropolis annealing of `trials` independent chains of the problem (one wave
 * of 64 lanes per chain).  Cycle t picks one spin i uniformly at random, computes the energy change
 * of flipping it, dE = 2 sigma_i (h_i + sum_j J_ij sigma_j) (H of Eq. 1), and accepts the flip if
 * dE <= 0, else with probability exp(-dE beta(t)).  beta is the inverse temperature at the integer
 * scale of the problem (ssqa_sa_schedule builds Section 4.4's schedule).
 * Random stream (Philox4x32-10, key = seed halves): the initial spins use counter
 * (i >> 7, 0xFFFFFFFE, 0, b), spin i taking bit (i & 31) of word (i & 127) >> 5 (bit 1 = +1); cycle
 * t uses counter (t, 0xFFFFFFFF, 0, b): i = (w0 * N) >> 32, and the flip is accepted iff
 * w1 < ssqa_sa_accept_threshold(dE, beta(t)).
 */
typedef struct ssqa_sa_params {
    int32_t trials;            /* T >= 1, at most 2^24                                             */
    int32_t cycles;            /* attempted flips per chain, >= 0                                  */
    const double* beta;        /* host double [cycles]: finite, >= 0                               */
    uint64_t seed;
    int64_t target_energy;     /* E* (for first_hit), or SSQA_NO_TARGET                            */
} ssqa_sa_params;

typedef struct ssqa_sa_outputs {
    int64_t* best_energy;      /* device int64 [T]: minimum energy over t in [0, cycles]           */
    int32_t* first_hit;        /* device int32 [T]: first t in [0, cycles] whose state (after t
                                  cycles) has energy E*, else -1                                   */
    int64_t* final_energy;     /* device int64 [T], or NULL                                        */
    int8_t* final_spins;       /* device int8 [T][N] (+-1), or NULL                                */
    int64_t* energy_trace;     /* device int64 [cycles + 1][T]: energy after t cycles, or NULL     */
} ssqa_sa_outputs;

/* Asynchronous on hip_stream.  SSQA_EINVAL for bad sizes, NULL required pointers or a beta that is
 * negative or not finite; SSQA_ENOTSUP when N exceeds 32768 (the chain's fields live in LDS). */
ssqa_status ssqa_sa_anneal(ssqa_problem_t problem, const ssqa_sa_params* params, const ssqa_sa_outputs* outputs,
                           void* hip_stream);

/* beta(t) = 1/(scale t_start) + t Delta, Delta = (1/(scale t_end) - 1/(scale t_start)) / (cycles - 1):
 * 1/T grows by the same amount every cycle (Section 4.4), from t_start at t = 0 to t_end at the last
 * cycle, at the integer scale `scale` (energies there are scale times the paper's).  Host output
 * double [cycles].  SSQA_EINVAL unless cycles >= 1, scale >= 1 and 0 < t_end, t_start. */
ssqa_status ssqa_sa_schedule(int32_t cycles, double t_start, double t_end, int32_t scale, double* beta);

/* 2^32 exp(-de beta) (de >= 0, beta >= 0), evaluated by the fixed sequence of correctly rounded double
 * operations the GPU chain uses: n = floor(x / ln 2 + 1/2) with x = de beta, r = n ln 2 - x, the degree-13
 * Taylor polynomial of exp(r) in Horner form, scaled by 2^(32 - n); 0 when x > 700. */
double ssqa_sa_accept_threshold(int64_t de, double beta);

/* ------------------------------------------------------------------------------------------- */
/* Host helpers: schedules and the graph-isomorphism mapping (no device work).                 */
/* ------------------------------------------------------------------------------------------- */

/*
 * J_perp schedule of Section 4.2 / Table 2, at the integer scale:
 *   each iteration lasts tau * (beta + 1) cycles; J_perp starts it at jmin and rises by
 *   (jmax - jmin) / beta every tau cycles, resetting to jmin when the next iteration starts.
 * jmin = jmin_num / den and jmax = jmax_num / den in paper units; out[t] = scale * J_perp(t)
 * must be an integer for every level (else SSQA_EINVAL).  out: host int32 [cycles].
 */
ssqa_status ssqa_jperp_schedule(int32_t cycles, int32_t tau, int32_t beta, int32_t jmin_num,
                                int32_t jmax_num, int32_t den, int32_t scale, int32_t* out);

/*
 * I_0 schedule of SSA (Section 4.4): I_0 starts at i0_min, is multiplied by `growth` (= 1 / beta)
 * every tau cycles up to i0_max, stays there for tau cycles and restarts at i0_min.
 * out[t] = scale * I_0(t).  out: host int32 [cycles].
 */
ssqa_status ssqa_ssa_i0_schedule(int32_t cycles, int32_t tau, int32_t growth, int32_t i0_min,
                                 int32_t i0_max, int32_t scale, int32_t* out);

/*
 * Graph isomorphism as an integer Ising model (Section 4.1, Eq. 8; mapping of Section 4.2).
 *   a1, a2 : host uint8 [n * n] adjacency matrices (symmetric, zero diagonal) of graphs 1 and 2.
 *   Spin p = u * n + i is x_{u,i} = 1 ("vertex u of graph 2 maps to vertex i of graph 1").
 *   QUBO: Q_pp = -2 c1; for p < q: 2 c1 when exactly one of u == v, i == j holds; c2 when u != v,
 *   i != j and a1[i][j] != a2[u][v] (each such unordered spin pair penalised once); else 0.
 *   Ising at scale S (a multiple of 4): J_pq = -(S/4) Q_pq, h_p = -(S/2) Q_pp - (S/4) sum_q Q_pq.
 *   h      : host int32 [n*n];  J : host int32 [n^4] row-major.
 *   e_star : receives the scaled ground energy, reached exactly when x encodes an isomorphism.
 */
ssqa_status ssqa_gi_to_ising(int32_t n, const uint8_t* a1, const uint8_t* a2, int32_t c1, int32_t c2,
                             int32_t scale, int32_t* h, int32_t* J, int64_t* e_star);

/*
 * The Philox4x32-10 block function used by the kernels, on the host, for verification:
 * out = Philox4x32-10(counter ctr[0..3], key key[0..1]).
 */
void ssqa_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#ifdef __cplusplus
}
#endif

#endif /* SSQA_H */
