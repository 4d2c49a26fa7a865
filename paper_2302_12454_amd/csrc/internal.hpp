// Internal interfaces between the C ABI (api.cpp) and the HIP kernels (sweep.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssqa {

// Rows per tile: one Philox output block covers 128 consecutive spins of one replica.
constexpr int kTileRows = 128;
// K extent of one int8 MFMA (v_mfma_i32_16x16x64_i8).
constexpr int kStepK = 64;
// Largest delay d supported (bit-plane ring of d + 2 planes in LDS).
constexpr int kMaxDelay = 6;

// Byte offset of J_ij inside one int8 plane of padded size np, in the fragment-tiled layout the sweep
// kernel reads: for row tile r (128 rows), K step s (64 columns) and fragment ai, one contiguous 1 KiB
// block holds the 16 x 64 operand of a v_mfma_i32_16x16x64_i8 in lane order (lane = 16 g + slot holds
// row slot -> tile row 32 (slot / 4) + 4 ai + slot % 4, columns 64 s + 16 g .. + 15).
__host__ __device__ inline size_t tiled_offset(int i, int j, int np) {
    const int nsteps = np / kStepK;
    const int r = i >> 7, o = i & 127;
    const int slot = 4 * (o >> 5) + (o & 3);
    const int ai = (o & 31) >> 2;
    const int s = j >> 6, gk = (j & 63) >> 4, byte = j & 15;
    const int lane = gk * 16 + slot;
    return ((size_t)(r * nsteps + s) * 8 + ai) * 1024 + (size_t)lane * 16 + byte;
}

// Byte offset and nibble of J_ij in the fp4 copy (K steps of 128 for v_mfma_scale_f32_16x16x128_f8f6f4).
// Block (row tile r, K step s, fragment ai) is 1 KiB; lane = 16 g + slot holds 32 values of row slot
// (tile row 32 (slot / 4) + 4 ai + slot % 4) for K = 128 s + 32 g + o, o < 32.  Value o = 16 h + 4 d + m
// sits in byte 4 d + m, nibble h, so that operand dword d holds the K offsets whose bit-plane positions
// are congruent to d modulo 4 (see the sweep kernel).
__host__ __device__ inline size_t tiled_offset_fp4(int i, int j, int kp4, int* nibble) {
    const int nsteps = kp4 / 128;
    const int r = i >> 7, orow = i & 127;
    const int slot = 4 * (orow >> 5) + (orow & 3);
    const int ai = (orow & 31) >> 2;
    const int s = j >> 7, g = (j & 127) >> 5, o = j & 31;
    const int h = o >> 4, d = (o >> 2) & 3, m = o & 3;
    *nibble = h;
    return ((size_t)(r * nsteps + s) * 8 + ai) * 1024 + (size_t)(g * 16 + slot) * 16 + 4 * d + m;
}

// K extent of the fp4 copy of J: np rounded up to a multiple of 256, and at least 512, so that the sweep's
// K loop always has four or more steps of 128 (its software pipeline has one shape for every size).
inline int fp4_k_extent(int np) {
    const int k = (np + 255) / 256 * 256;
    return k < 512 ? 512 : k;
}

// Device-side description of one problem.
struct DeviceProblem {
    int32_t n;          // spins N
    int32_t np;         // N padded to a multiple of kTileRows (rows and columns of every plane)
    int32_t planes;     // P int8 planes, J = sum_p 256^p J_p
    const int8_t* J;    // [P][np * np] in the fragment-tiled layout of tiled_offset, zero padded
    const uint8_t* J4;  // fp4 (e2m1) copy of J in the layout of tiled_offset_fp4 when every J_ij is exactly
                        // representable (0, +-1, +-2, +-3, +-4, +-6), else nullptr
    int32_t kp4;        // K extent of the fp4 copy (fp4_k_extent)
    const int32_t* h;   // [np], zero padded
    const int32_t* hr;  // [np]: h_i - sum_j J_ij   (field offset for x = (sigma + 1) / 2)
    const int32_t* er;  // [np]: 2 h_i - sum_j J_ij (energy offset)
};

// Arguments of one launch of the persistent sweep kernel.
struct SweepArgs {
    DeviceProblem prob;
    int32_t nb;             // columns per workgroup: 32, 64 or 128 (fp4 operands only)
    int32_t fp4;            // 1: the field product runs on the fp4 copy of J
    int32_t fast;           // 1: alpha = 1 and max I0 + 2 noise_amp + 2 max |jperp| (1 + mode) <= 128
    int32_t R;              // replicas
    int32_t T;              // trials
    int32_t tpw;            // trials per workgroup
    int32_t cols_wg;        // tpw * R <= columns per workgroup
    int32_t t_begin;        // first cycle of this launch (absolute)
    int32_t t_end;          // cycles [t_begin, t_end) are updated in this launch
    int32_t final_pass;     // evaluate H_p at t_end as well (last launch of a run)
    int32_t save_hist;      // write sigma(t_end - s), s = 1..d, to hist_state at the end (for a resume)
    int32_t delay;
    int32_t alpha;
    int32_t noise_amp;
    int32_t mode;
    uint32_t key0, key1;
    int64_t target;         // INT64_MIN for none
    const int32_t* jperp;   // device [cycles] indexed by absolute t
    const int32_t* i0;      // device [cycles]
    int8_t* is_state;       // [n_wg * nb][np]: counters, column = wg * nb + local column
    uint32_t* hist_state;   // [n_wg][delay][nb][np / 32]: sigma(t_begin - s) bits, s = 1..d
    int64_t* best;          // [T]
    int32_t* first_hit;     // [T]
    int32_t* trace;         // [(SC + 1)][T * R] or nullptr; row t holds cycle t
    // Row-split form (sweep_split_kernel): one launch per cycle over n_cb column blocks (is_state as above, block
    // index in place of the workgroup) times n_groups row groups of group_tiles row tiles; sigma's bit-plane ring
    // and the per-column energy sums live in device memory between launches.
    int32_t n_groups;       // row groups per column block
    int32_t group_tiles;    // row tiles per group
    int32_t split_k;        // 4: groups of one tile of a 32-column block, whose K steps the workgroup's four waves
                            // share; else 0 or 1
    int32_t split_q, split_i0;   // J_perp(t) and I_0(t) of the launch's cycle (set by the kernel from its arguments)
    int32_t n_cb;           // column blocks
    uint32_t* ring;         // [d + 2][n_cb][nb][np / 32]: sigma(t) in ring slot t % (d + 2), spread bit order
    int32_t* e_sum;         // [2][n_cb * nb]: sum_i sigma_i (2 h_i + F_i) of cycle t in slot t & 1
};

// Row tiles per group of the row-split form (at most one per wave), and the groups of a block: enough to cover
// the tiles, rounded up to a multiple of the XCD count so that a row group's copies in every block share an XCD.
constexpr int kGroupTiles = 4;
constexpr int kGroupWords = 4 * kGroupTiles + 1;   // LDS words per column of a group's rows (one of padding)
inline int split_groups(int np, int xcds, int group_tiles = kGroupTiles) {
    const int g = (np / kTileRows + group_tiles - 1) / group_tiles;
    return (g + xcds - 1) / xcds * xcds;
}

// LDS of a row-split launch with split_k = 4 beyond sweep_lds_bytes: the partial sums the four waves pass
// each other, as much as three waves' accumulators (2 nb 32-bit words per lane each).
inline size_t split_k_lds_bytes(int nb) { return (size_t)3 * 64 * 2 * nb * 4; }

// Flags of one sweep_split_kernel launch at cycle t; its grid is n_cb x n_groups row-group workgroups (init,
// run), then n_cb closing workgroups (close).
constexpr int kSplitInit = 1;    // sigma(0) and Is(0) of the group's rows, best and first hit reset (t = 0)
constexpr int kSplitClose = 2;   // reduce cycle t - 1's energies to the trace, best and first hit
constexpr int kSplitRun = 4;     // the field product, energy and (with kSplitUpdate) the update of cycle t
constexpr int kSplitUpdate = 8;

// Launchers (sweep.hip).  Return hipSuccess or the launch error.
// rowvec receives [h | hr | er], three int32 vectors of np entries.
// J is device int32 [n * n] (elem = 4) or, for a single-plane problem, int8 (elem = 1).
hipError_t launch_prepare_planes(const void* J, int elem, const int32_t* h32, int32_t n, int32_t np, int32_t planes,
                                 int8_t* Jp, int32_t* rowvec, hipStream_t stream);
// fp4 copy of J (every entry must be one of 0, +-1, +-2, +-3, +-4, +-6): np rows by kp4 columns.
hipError_t launch_prepare_fp4(const void* J, int elem, int32_t n, int32_t np, int32_t kp4, uint8_t* J4,
                              hipStream_t stream);
// Sets the LDS limits of every sweep kernel variant once (before any launch or graph capture).
hipError_t configure_sweep_kernels();
// Dynamic LDS of one sweep workgroup for padded size np, delay d and nb columns.
size_t sweep_lds_bytes(int np, int delay, int nb);
// Dynamic LDS of a row-split launch (sweep_split_kernel): sigma(t) of the block, the group's rows of sigma(t - d)
// and sigma(t + 1) (kGroupWords words per column), and the rest as in sweep_lds_bytes.
size_t split_lds_bytes(int np, int nb);
// Kernel variant index of (alpha == 1, coupling mode, nb, fp4 operands); kSweepVariants in total.
constexpr int kSweepVariants = 24;
int sweep_variant(bool fast, int mode, int nb, bool fp4);
// Columns per workgroup of a variant.
int variant_columns(int variant);
hipError_t launch_sweep(const SweepArgs& args, int n_wg, hipStream_t stream);
// One launch of the row-split sweep (item: device copy of the anneal's arguments; grid n_cb * n_groups; kSplit*
// flags) for a variant with 32 or 64 columns per workgroup.
// The cycle's schedule entries come from the host copies jperp[t] and i0[t] (read with kSplitUpdate only) and
// travel as launch arguments, so that no launch waits on a device read of them.
hipError_t launch_sweep_split(const SweepArgs* item, const SweepArgs& host, int t, int flags, const int32_t* jperp,
                              const int32_t* i0, hipStream_t stream);
// items: device array of anneals; work: device list of (item << 16 | column block), n_work entries, all of
// one kernel variant; the LDS size is taken for the largest padded N and delay among them.
hipError_t launch_sweep_batch(const SweepArgs* items, const uint32_t* work, int n_work, int max_np, int max_delay,
                              int variant, hipStream_t stream);
// Public anneal state (ssqa_anneal_state) <-> the sweep's internal layout of one plain anneal.
hipError_t launch_import_state(const int8_t* counters, const uint32_t* history, int32_t n, int32_t np, int32_t R,
                               int32_t T, int32_t tpw, int32_t nb, int32_t delay, int8_t* is_state,
                               uint32_t* hist_state, hipStream_t stream);
hipError_t launch_export_history(const uint32_t* hist_state, int32_t n, int32_t np, int32_t R, int32_t T,
                                 int32_t tpw, int32_t nb, int32_t delay, uint32_t* history, hipStream_t stream);
hipError_t launch_copy_final_is(const int8_t* is_state, int32_t np, int32_t n, int32_t R, int32_t T,
                                int32_t tpw, int32_t nb, int8_t* out, hipStream_t stream);
hipError_t launch_energy(const DeviceProblem& prob, const int8_t* spins, int32_t cols, int64_t* energies,
                         hipStream_t stream);
hipError_t launch_qmc_energy(const DeviceProblem& prob, const int8_t* counters, int32_t trials, int32_t R,
                             int32_t jperp, int64_t* out, hipStream_t stream);
// Fixed device scratch of ssqa_anneal_noalloc (sweep.hip): kFixedScratchBytes on every device the library
// runs it on, held until the process ends.
constexpr size_t kFixedScratchBytes = size_t(64) << 20;
// Device address of the current device's copy of that scratch (`device` must be current).  Looked up once per
// device and kept.
hipError_t fixed_scratch(int device, void** ptr);


// Arguments of the simulated-annealing baseline kernel (sa.hip): one wave per chain.
struct SAArgs {
    DeviceProblem prob;
    int32_t T;              // chains (trials)
    int32_t cycles;         // attempted flips per chain
    const double* beta;     // device [cycles]: inverse temperature at the integer scale
    uint32_t key0, key1;
    int64_t target;         // INT64_MIN for none
    int64_t* best;          // [T]
    int32_t* first_hit;     // [T]
    int64_t* final_energy;  // [T] or nullptr
    int8_t* final_spins;    // [T][n] or nullptr
    int64_t* trace;         // [(cycles + 1)][T] or nullptr
};

// LDS words per chain: np int32 fields and np int8 spins.
__host__ __device__ inline int sa_lds_words(int np) { return np + np / 4; }
// Chains per workgroup that fit 160 KiB of LDS (at most 4); 0 when one does not.
int sa_waves_per_group(int np);
hipError_t launch_sa(const SAArgs& args, hipStream_t stream);
// 2^32 exp(-de beta) by a fixed sequence of rounded double operations (host and device alike).
__host__ __device__ double sa_exp_neg(double x);
__host__ __device__ double sa_accept_threshold(long long de, double beta);

}  // namespace ssqa

// ---------------------------------------------------------------------------------------------
// Host-side pieces shared by the C ABI translation units (api.cpp, server.cpp).
// ---------------------------------------------------------------------------------------------
#include <string>

#include "ssqa.h"

struct ssqa_problem {
    int32_t device;
    ssqa::DeviceProblem dev;
    int8_t* J_planes;
    uint8_t* J_fp4;    // fp4 copy of J, or nullptr
    int32_t* rowvec;   // [h | h - rowsum | 2h - rowsum], np each
    int64_t fp4_bound; // max_i (|h_i| + 2 sum_j |J_ij|): bounds the fp4 accumulator's partial sums
};

namespace ssqa {
namespace detail {

extern thread_local std::string g_last_error;
// Record a formatted message for ssqa_last_error() and return `s`.
ssqa_status fail(ssqa_status s, const char* fmt, ...);
ssqa_status hip_fail(hipError_t e, const char* what);

// Makes `device` current and restores the previous device on exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int device);
    ~DeviceGuard();
};

// Checks and statistics of a host coupling matrix J (int32 [n * n]) with biases h.
struct CouplingScan {
    long long first_asym = -1;   // first asymmetric pair in row order (i * n + j), or -1
    int first_diag = -1;         // first row with a non-zero diagonal entry, or -1
    long long total = 0;         // 2 sum_i |h_i| + sum_ij |J_ij|
    int planes = 1;              // balanced int8 planes J needs
    bool codes = true;           // every J_ij is one of 0, +-1, +-2, +-3, +-4, +-6 (fp4 codes)
    long long bound = 0;         // max_i (|h_i| + 2 sum_j |J_ij|)
};
// One pass over J, in 64 x 64 blocks and over host threads for large n; with J8 non-null it also writes J
// narrowed to int8 there (exact when planes == 1).
CouplingScan scan_couplings(int n, const int32_t* h, const int32_t* J, int8_t* J8);
// The failure a scan found (first asymmetric pair, first non-zero diagonal entry, then the int32 range).
ssqa_status check_couplings(const CouplingScan& scan, int n, const int32_t* J);
// ssqa_create_problem after a passed check: J on the host as int32, or (J8 non-null, planes == 1) as int8.
ssqa_status create_problem_impl(int32_t n, const int32_t* h, const int32_t* J, const int8_t* J8,
                                const CouplingScan& scan, int32_t device, ssqa_problem_t* out);
// Whether the fp4 field product of an anneal of `prob` with `pa` is exact (schedules already checked).
bool fp4_fits(const ssqa_problem* prob, const ssqa_anneal_params* pa);
// Whether the byte-parallel epilogue applies to `pa` over its whole schedule (alpha = 1 and small increments).
bool fast_epilogue(const ssqa_anneal_params* pa);
// Whether an anneal of `prob` with `pa` runs its field product on the fp4 copy of J.
bool use_fp4(const ssqa_problem* prob, const ssqa_anneal_params* pa);
// Columns per workgroup for an anneal of `prob` with `pa`: the requested 32, 64 or 128, else 64 or 32.
int block_columns(const ssqa_problem* prob, const ssqa_anneal_params* pa);
// The same from the padded size alone (no problem needed).
int block_columns_for(int np, const ssqa_anneal_params* pa);
// Full argument check of one anneal; records the reason on failure.
ssqa_status check_params(const ssqa_problem* prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out);
// Kernel arguments of one anneal (t_begin / t_end / final_pass left for the caller).  nb and tpw
// (columns and trials per workgroup) default to the packed layout of block_columns when 0; fp4 < 0 takes the
// operands use_fp4 picks, else 1 = fp4, 0 = int8 planes.
SweepArgs make_args(const ssqa_problem* prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out,
                    const int32_t* d_jperp, const int32_t* d_i0, int8_t* is_state, uint32_t* hist, int nb = 0,
                    int tpw = 0, int fp4 = -1);
// Workgroup layout of a plain anneal (ssqa_anneal): columns and trials per workgroup, workgroups, operands, and
// whether the autotuner's cache chose it.
struct PlainLayout {
    int nb, tpw, n_wg;
    bool fp4, tuned;
};
// The built-in rules, or, for an automatic request (block_columns = 0, operand_format = 0), the tile the
// autotuner recorded for this device, kernel build and shape when there is one.
PlainLayout plain_layout(const ssqa_problem* prob, const ssqa_anneal_params* pa);
// The built-in rules alone.
PlainLayout rule_layout(const ssqa_problem* prob, const ssqa_anneal_params* pa);
// Whether a tile (nb columns and tpw trials per workgroup, fp4 or int8 operands) can run `pa` on `prob`.
bool tile_legal(const ssqa_problem* prob, const ssqa_anneal_params* pa, int nb, int tpw, bool fp4);
// Whether an automatic block of a batch instance widens to 128 columns, with the padded-row floor `min_rows`
// (0: never).
bool batch_wide(const ssqa_problem* prob, const ssqa_anneal_params* pa, int min_rows);
// Built-in floor of the batched form (padded rows from which automatic blocks take 128 columns).
constexpr int kBatchWideRows = 1024;

// Autotuner cache (tune.cpp).  A tile recorded for (device, kernel build, padded N, planes, R, T, delay, mode,
// epilogue, fp4 availability); false when none applies.
struct TunedTile {
    int nb, tpw, fp4;
    double ms_per_cycle;
};
bool tuned_plain(const ssqa_problem* prob, const ssqa_anneal_params* pa, TunedTile* out);
// Identity of a batch's shape (padded N, planes, R, T, delay, mode, epilogue and fp4 availability of each
// anneal, in order) for the cache.
uint64_t batch_signature(int count, const ssqa_problem_t* problems, const ssqa_anneal_params* params);
// The 128-column floor recorded for a batch of this signature on this device and build, or -1.
int tuned_batch_rows(int device, uint64_t signature);
// ssqa_batch_create with the 128-column floor `wide_rows` (< 0: the recorded floor, else the built-in one).
ssqa_status batch_create_impl(int32_t count, const ssqa_problem_t* problems, const ssqa_anneal_params* params,
                              const ssqa_anneal_outputs* outputs, ssqa_batch_t* out, int wide_rows);
// Device state of one plain anneal: counters, bit-plane history and the two schedules ([jperp | i0]).
struct AnnealSizes {
    PlainLayout layout;
    size_t is_bytes, hist_bytes, sched_bytes;
};
AnnealSizes anneal_sizes(const ssqa_problem* prob, const ssqa_anneal_params* pa);
// Caller-provided device state of a plain anneal (at least the sizes anneal_sizes gives).
struct AnnealWorkspace {
    int8_t* is_state;
    uint32_t* hist;
    int32_t* sched;
};
// ssqa_anneal: with ws == nullptr the state is taken from the stream-ordered pool and the schedules are copied
// through pinned staging (no host wait); with a workspace nothing is allocated and the host waits for the
// schedule copy.  Checks the parameters first (anneal_sizes needs them valid).
ssqa_status anneal_impl(const ssqa_problem* prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out,
                        hipStream_t stream, const AnnealWorkspace* ws);
// Copies `count` host arrays back to back to device memory `dst` on `stream` through pinned staging owned by
// the library; returns without waiting for the copy.
hipError_t staged_upload(int device, void* dst, const void* const* srcs, const size_t* sizes, int count,
                         hipStream_t stream);
int device_cu_count(int device);
int device_xcd_count(int device);
// Keep freed stream-ordered allocations in the device pool.
void retain_pool_memory(int device);

}  // namespace detail
}  // namespace ssqa

#define SSQA_HIP(call, what)                                          \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return ssqa::detail::hip_fail(e_, what); \
    } while (0)
