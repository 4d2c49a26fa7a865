// C ABI of the SSQA library: argument checking, device memory, launches (see include/ssqa.h).
#include "ssqa.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "philox.hpp"
#include "work_order.hpp"

using namespace ssqa;

namespace ssqa {
namespace detail {

thread_local std::string g_last_error;

ssqa_status fail(ssqa_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

ssqa_status hip_fail(hipError_t e, const char* what) {
    return fail(SSQA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

DeviceGuard::DeviceGuard(int device) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(device) == hipSuccess;
}

DeviceGuard::~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
}

// Keep freed stream-ordered allocations in the device's default pool instead of returning them to the
// driver at every synchronisation, so repeated anneals reuse their state buffers.
void retain_pool_memory(int device) {
    static bool done[64] = {};
    if (device < 0 || device >= 64 || done[device]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t threshold = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
    }
    done[device] = true;
}

// Pinned host staging for the host arrays (schedules) that asynchronous calls copy to the device.  The call
// copies the caller's array into a slot and returns at once; a slot is reused only after the event recorded
// behind its copy has completed.  Slots are kept per device until the process ends.
namespace {
struct StageSlot {
    int device;
    size_t bytes;
    void* host;
    hipEvent_t done;
};
std::mutex g_stage_mutex;
std::vector<StageSlot> g_stage;
}  // namespace

hipError_t staged_upload(int device, void* dst, const void* const* srcs, const size_t* sizes, int count,
                         hipStream_t stream) {
    size_t total = 0;
    for (int i = 0; i < count; ++i) total += sizes[i];
    if (total == 0) return hipSuccess;
    std::lock_guard<std::mutex> lock(g_stage_mutex);
    StageSlot* slot = nullptr;
    for (StageSlot& s : g_stage)
        if (s.device == device && s.bytes >= total && hipEventQuery(s.done) == hipSuccess) {
            slot = &s;
            break;
        }
    if (!slot) {
        StageSlot s{device, std::max<size_t>(total, 64 * 1024), nullptr, nullptr};
        hipError_t e = hipHostMalloc(&s.host, s.bytes, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipHostFree(s.host);
            return e;
        }
        g_stage.push_back(s);
        slot = &g_stage.back();
    }
    char* h = static_cast<char*>(slot->host);
    for (int i = 0; i < count; ++i) {
        std::memcpy(h, srcs[i], sizes[i]);
        h += sizes[i];
    }
    hipError_t e = hipMemcpyAsync(dst, slot->host, total, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(slot->done, stream);
    return e;
}

int planes_needed(int32_t v) {
    int p = 0;
    do {
        const int8_t d = (int8_t)(v & 0xFF);
        v = (v - d) >> 8;
        ++p;
    } while (v != 0);
    return p;
}

// Whether every fp32 partial sum of the fp4 field product stays exact for this anneal.  The accumulator of
// row i starts at 1.5 * 2^23 plus v0 = h_i - sum_j J_ij + adj with |adj| <= n_rnd + (1 + mode) max_t |J_perp(t)|
// + 128, and each MFMA adds 2 J_ij x_j for some of the j: every partial sum is 1.5 * 2^23 plus an integer of
// magnitude at most |h_i| + 2 sum_j |J_ij| + |adj|.  While that stays below 2^22 the sum lies in [2^23, 2^24),
// where fp32 represents every integer, so no rounding occurs in any summation order and the bits read back are
// 0x4B400000 plus the integer (Eq. 6a-b need the field exactly).  Schedules must already be checked.
bool fp4_fits(const ssqa_problem* prob, const ssqa_anneal_params* pa) {
    long long q_max = 0;
    for (int t = 0; t < pa->cycles; ++t) q_max = std::max(q_max, std::llabs((long long)pa->jperp[t]));
    const long long bound = prob->fp4_bound + pa->noise_amp + (1LL + pa->coupling_mode) * q_max + 128;
    return bound < (1LL << 22);
}

bool use_fp4(const ssqa_problem* prob, const ssqa_anneal_params* pa) {
    if (pa->operand_format == 1 || prob->dev.J4 == nullptr) return false;
    return fp4_fits(prob, pa);
}

// The byte-parallel counter update applies when alpha = 1 and every counter plus 128 plus its noise and
// coupling increments stays below 256.  A counter holds at most max_t I0(t) - 1 (it may have been clamped
// in an earlier cycle with a larger I0), so the bound is taken over the whole schedule:
// max_t I0(t) + 2 noise_amp + 2 max_t |jperp(t)| (1 + mode) <= 128.
bool fast_epilogue(const ssqa_anneal_params* pa) {
    if (pa->alpha != 1) return false;
    long long i0_max = 1, q_max = 0;
    for (int t = 0; t < pa->cycles; ++t) {
        const long long q = pa->jperp[t] < 0 ? -(long long)pa->jperp[t] : pa->jperp[t];
        i0_max = std::max<long long>(i0_max, pa->i0[t]);
        q_max = std::max(q_max, q);
    }
    return i0_max + 2LL * pa->noise_amp + 2 * q_max * (1 + pa->coupling_mode) <= 128;
}

// Columns per workgroup: the requested width, or 64 when R <= 64 and the bit planes fit in LDS, else 32
// (plain_layout may widen an automatic 64 to 128).
int block_columns_for(int np, const ssqa_anneal_params* pa) {
    if (pa->block_columns == 32 || pa->block_columns == 64 || pa->block_columns == 128) return pa->block_columns;
    if (pa->replicas <= 64 && sweep_lds_bytes(np, pa->delay, 64) <= 160 * 1024) return 64;
    return 32;
}

int block_columns(const ssqa_problem* prob, const ssqa_anneal_params* pa) {
    return block_columns_for(prob->dev.np, pa);
}

int device_cu_count(int device) {
    // Cached per device; host threads may call the library concurrently, so the cache entries are atomic
    // (a repeated query by a second thread stores the same value).
    static std::atomic<int> counts[64] = {};
    if (device < 0 || device >= 64) return 256;
    int v = counts[device].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || v < 1) v = 256;
        counts[device].store(v, std::memory_order_relaxed);
    }
    return v;
}

int device_xcd_count(int device) {
    static std::atomic<int> counts[64] = {};
    if (device < 0 || device >= 64) return 1;
    int v = counts[device].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeNumberOfXccs, device) != hipSuccess || v < 1) v = 1;
        counts[device].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Whether an automatic 64-column block may widen to 128 columns: fp4 operands or J in one int8 plane, whole
// trials filling the block, bit planes that fit in LDS, and at least `min_rows` padded rows (0: never).  With fewer rows the K
// loop of a tile is short and two 64-column workgroups per CU hide its latency better than one of 128
// columns; a plain anneal, which has the chip to itself, gains from 1536 rows on, a batch, whose many
// matrices share each L2, already from 1024 (the halved J traffic per MFMA counts for more there).
static bool wide_blocks_pay(const ssqa_problem* prob, const ssqa_anneal_params* pa, int min_rows) {
    const int np = prob->dev.np;
    return min_rows > 0 && pa->block_columns == 0 && block_columns(prob, pa) == 64 &&
           (use_fp4(prob, pa) || prob->dev.planes == 1) && 128 % pa->replicas == 0 && np >= min_rows &&
           sweep_lds_bytes(np, pa->delay, 128) <= 160 * 1024;
}

bool batch_wide(const ssqa_problem* prob, const ssqa_anneal_params* pa, int min_rows) {
    return wide_blocks_pay(prob, pa, min_rows);
}

bool tile_legal(const ssqa_problem* prob, const ssqa_anneal_params* pa, int nb, int tpw, bool fp4) {
    if (nb != 32 && nb != 64 && nb != 128) return false;
    if (pa->replicas > nb || tpw < 1 || tpw > nb / pa->replicas) return false;
    if (fp4 && !use_fp4(prob, pa)) return false;
    if (nb == 128 && !fp4 && prob->dev.planes != 1) return false;
    return sweep_lds_bytes(prob->dev.np, pa->delay, nb) <= 160 * 1024;
}

// Layout of a plain anneal by the built-in rules.  Packing whole workgroups (as many trials as fit) gives
// the best J reuse once there are enough workgroups for every CU twice over; a smaller anneal is spread
// instead (the narrow block when the replicas fit it, and fewer trials per workgroup, leaving columns
// unused), so that its latency is not set by a handful of CUs.  Results do not depend on the layout.
PlainLayout rule_layout(const ssqa_problem* prob, const ssqa_anneal_params* pa) {
    const int R = pa->replicas, T = pa->trials;
    const int target = 2 * device_cu_count(prob->device);
    // A one-tile problem (128 padded rows) takes int8 operands when J is one plane: the fp4 copy's K extent is
    // at least 512 (four steps of 128, three of them padding), the plane's 128 (two steps of 64).  Measured
    // 8-10 % faster at N = 25 and 100; from 256 padded rows fp4 is as fast or faster.
    const bool fp4 = use_fp4(prob, pa) && !(pa->operand_format == 0 && prob->dev.np <= kTileRows && prob->dev.planes == 1);
    int nb = block_columns(prob, pa);
    // 128 columns per workgroup (one per CU, one wave per SIMD with 512 registers) feed each J fragment to twice
    // as many MFMAs; taken when wide blocks pay and still number two per CU.
    if (wide_blocks_pay(prob, pa, 1536) && (T + 128 / R - 1) / (128 / R) >= target)
        return PlainLayout{128, 128 / R, (T + 128 / R - 1) / (128 / R), fp4, false};
    if (pa->block_columns == 0 && nb == 64 && R <= 32 && (T + 64 / R - 1) / (64 / R) < target) nb = 32;
    const int full = nb / R;
    int tpw = full;
    if ((T + full - 1) / full < target) tpw = std::max(1, (T + target - 1) / target);
    return PlainLayout{nb, tpw, (T + tpw - 1) / tpw, fp4, false};
}

PlainLayout plain_layout(const ssqa_problem* prob, const ssqa_anneal_params* pa) {
    TunedTile t;
    if (pa->block_columns == 0 && pa->operand_format == 0 && tuned_plain(prob, pa, &t))
        return PlainLayout{t.nb, t.tpw, (pa->trials + t.tpw - 1) / t.tpw, t.fp4 != 0, true};
    return rule_layout(prob, pa);
}

ssqa_status check_params(const ssqa_problem* prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out) {
    const int R = pa->replicas, T = pa->trials, SC = pa->cycles;
    if (R < 1 || T < 1 || SC < 0) return fail(SSQA_EINVAL, "replicas, trials must be >= 1 and cycles >= 0");
    if (pa->block_columns != 0 && pa->block_columns != 32 && pa->block_columns != 64 && pa->block_columns != 128)
        return fail(SSQA_EINVAL, "block_columns must be 0, 32, 64 or 128");
    if (pa->operand_format < 0 || pa->operand_format > 2) return fail(SSQA_EINVAL, "operand_format must be 0, 1 or 2");
    if ((long long)T * R > (1LL << 28)) return fail(SSQA_EINVAL, "trials * replicas too large");
    if (pa->delay < 0 || pa->delay > kMaxDelay) return fail(SSQA_EINVAL, "delay %d outside [0, %d]", pa->delay, kMaxDelay);
    if (pa->alpha < 1) return fail(SSQA_EINVAL, "alpha must be >= 1");
    if (pa->noise_amp < 0 || pa->noise_amp > (1 << 20)) return fail(SSQA_EINVAL, "noise_amp outside [0, 2^20]");
    if (pa->coupling_mode != 0 && pa->coupling_mode != 1) return fail(SSQA_EINVAL, "coupling_mode must be 0 or 1");
    if (pa->cycles_per_launch < 0) return fail(SSQA_EINVAL, "cycles_per_launch must be >= 0");
    if (!out->best_energy || !out->first_hit) return fail(SSQA_EINVAL, "best_energy and first_hit are required");
    if (SC > 0 && (!pa->jperp || !pa->i0)) return fail(SSQA_EINVAL, "schedules are required");
    for (int t = 0; t < SC; ++t) {
        if (pa->i0[t] < pa->alpha || pa->i0[t] > 127)
            return fail(SSQA_EINVAL, "i0[%d] = %d outside [alpha, 127]", t, pa->i0[t]);
        if (pa->jperp[t] < -(1 << 20) || pa->jperp[t] > (1 << 20))
            return fail(SSQA_EINVAL, "jperp[%d] = %d outside [-2^20, 2^20]", t, pa->jperp[t]);
    }
    // operand format (the schedules are valid from here on)
    if (pa->operand_format == 2 && !prob->dev.J4)
        return fail(SSQA_ENOTSUP, "fp4 operands requested but J has entries outside {0, +-1, +-2, +-3, +-4, +-6} "
                                  "or max_i(|h_i| + 2 sum_j |J_ij|) + 128 >= 2^22");
    if (pa->operand_format == 2 && !fp4_fits(prob, pa))
        return fail(SSQA_ENOTSUP, "fp4 operands requested but max_i(|h_i| + 2 sum_j |J_ij|) + n_rnd + "
                                  "(1 + mode) max|jperp| + 128 >= 2^22: fp32 accumulation would not be exact");
    const int nb = block_columns(prob, pa);
    if (R > nb) return fail(SSQA_ENOTSUP, "replicas = %d exceeds %d columns per workgroup", R, nb);
    if (nb == 128 && !use_fp4(prob, pa) && prob->dev.planes != 1)
        return fail(SSQA_ENOTSUP, "128 columns per workgroup with int8 operands need every |J_ij| <= 127 "
                                  "(one int8 plane); this J needs %d", prob->dev.planes);
    if (sweep_lds_bytes(prob->dev.np, pa->delay, nb) > 160 * 1024)
        return fail(SSQA_ENOTSUP, "N = %d with delay %d needs %zu bytes of LDS per workgroup (> 160 KiB)",
                    prob->dev.n, pa->delay, sweep_lds_bytes(prob->dev.np, pa->delay, nb));
    return SSQA_OK;
}

SweepArgs make_args(const ssqa_problem* prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out,
                    const int32_t* d_jperp, const int32_t* d_i0, int8_t* is_state, uint32_t* hist, int nb, int tpw,
                    int fp4) {
    SweepArgs a{};
    if (nb == 0) nb = block_columns(prob, pa);
    if (tpw == 0) tpw = nb / pa->replicas;
    a.prob = prob->dev;
    a.nb = nb;
    a.fp4 = fp4 < 0 ? (use_fp4(prob, pa) ? 1 : 0) : (fp4 ? 1 : 0);
    a.fast = fast_epilogue(pa) ? 1 : 0;
    a.R = pa->replicas;
    a.T = pa->trials;
    a.tpw = tpw;
    a.cols_wg = tpw * pa->replicas;
    a.delay = pa->delay;
    a.alpha = pa->alpha;
    a.noise_amp = pa->noise_amp;
    a.mode = pa->coupling_mode;
    a.key0 = (uint32_t)(pa->seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(pa->seed >> 32);
    a.target = pa->target_energy;
    a.jperp = d_jperp;
    a.i0 = d_i0;
    a.is_state = is_state;
    a.hist_state = hist;
    a.best = out->best_energy;
    a.first_hit = out->first_hit;
    a.trace = out->energy_trace;
    return a;
}

// Sizes of the device state of a plain anneal (counters, bit-plane history, schedules) in its layout.
AnnealSizes anneal_sizes(const ssqa_problem* prob, const ssqa_anneal_params* pa) {
    const PlainLayout lay = plain_layout(prob, pa);
    const int np = prob->dev.np;
    AnnealSizes z;
    z.layout = lay;
    z.is_bytes = (size_t)lay.n_wg * lay.nb * np;
    z.hist_bytes = (size_t)lay.n_wg * std::max(pa->delay, 1) * lay.nb * (np / 32) * 4;
    z.sched_bytes = 2 * (size_t)std::max(pa->cycles, 1) * 4;
    return z;
}

// Automatic row-split form: from kSplitPlainRows padded rows for anneals of at most kSplitMaxBlocks column
// blocks, and from kSplitWideRows for at most kSplitWideBlocks.  The persistent form gives each workgroup whole
// trials, so every workgroup streams all of J through its CU once per cycle, whatever the number of
// workgroups; an anneal of few trials (SSA's R = 1, say) is then bound by one CU's load rate.  The row-split
// form spreads each trial's rows over row groups of workgroups at the price of one launch per cycle and
// sigma's exchange through device memory.  On one MI355X it was measured faster from N = 1225 (1280 padded
// rows) for 4 to 16 column blocks, slower at N = 625, and for 50 blocks of 64 columns slower at N = 1225 and
// faster from N = 2025 (2048 padded rows: 19.0 against 23.7 us per cycle, at N = 2500 24.2 against 36.4).
constexpr int kSplitPlainRows = 1280;
constexpr int kSplitMaxBlocks = 16;
constexpr int kSplitWideRows = 2048;
constexpr int kSplitWideBlocks = 64;

// Column-block width of the row-split form for a plain anneal (ssqa_anneal_params.split_rows), or 0 for the
// persistent form.  Blocks hold whole trials: 32 columns while that gives few enough blocks (a narrower block
// shortens each wave's work per cycle), else 64.
static int plain_split_columns(const ssqa_problem* prob, const ssqa_anneal_params* pa, int t0, int t1,
                               bool checkpoint, bool workspace) {
    if (pa->split_rows < 0 || workspace || checkpoint || t0 != 0 || t1 != pa->cycles) return 0;
    const int np = prob->dev.np, R = pa->replicas, T = pa->trials;
    auto fits = [&](int nb) { return R <= nb && split_lds_bytes(np, nb) <= 160 * 1024; };
    auto blocks = [&](int nb) { return (T + nb / R - 1) / (nb / R); };
    int nb = pa->block_columns;
    if (nb == 0) nb = fits(32) && (blocks(32) <= kSplitMaxBlocks || !fits(64)) ? 32 : 64;
    if (nb > 64 || !fits(nb)) return 0;
    // a forced split of very many trials keeps the persistent form rather than a grid past 2^30 workgroups
    if ((long long)blocks(nb) * (np / kTileRows + 16) > (1LL << 30)) return 0;
    if (pa->split_rows > 0) return np >= pa->split_rows ? nb : 0;
    const int n_cb = blocks(nb);
    const bool pays = (np >= kSplitPlainRows && n_cb <= kSplitMaxBlocks) || (np >= kSplitWideRows && n_cb <= kSplitWideBlocks);
    return pays ? nb : 0;
}

// The row-split form of a fresh anneal run to the end: whole trials per column block (nb / R each), the
// block's rows in row groups of 1, 2 or 4 tiles, one sweep_split_kernel launch per cycle (the launch boundary
// is the cycle's barrier), sigma's ring of d + 2 bit planes and the energy sums in device memory.
static hipError_t anneal_split(const ssqa_problem* prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out,
                               int nb, bool fp4, hipStream_t stream) {
    const int R = pa->replicas, T = pa->trials, SC = pa->cycles;
    const int np = prob->dev.np, tpw = nb / R;
    const int n_cb = (T + tpw - 1) / tpw;
    // The fewest row tiles per group (1, 2 or 4) that keep the row groups within two per CU: a group's
    // workgroup reads its tiles' J rows every cycle, so smaller groups shorten the cycle while CUs are idle.
    const int xcds = device_xcd_count(prob->device), cus = device_cu_count(prob->device);
    int group_tiles = 1;
    while (group_tiles < kGroupTiles && (long long)n_cb * split_groups(np, xcds, group_tiles) > 2LL * cus)
        group_tiles *= 2;
    const int n_groups = split_groups(np, xcds, group_tiles);
    // Groups of one tile leave three of a workgroup's four waves idle, and one wave alone streams the tile's J
    // rows at the rate its few loads in flight allow: with 32-column blocks the four waves then share the
    // tile's K steps (at least four each), when their partial sums fit in LDS beside the bit planes.
    const int k_steps = fp4 ? prob->dev.kp4 / 128 : np / kStepK;
    const bool split_k = group_tiles == 1 && nb == 32 && k_steps >= 16 &&
                         split_lds_bytes(np, nb) + split_k_lds_bytes(nb) <= 160 * 1024;
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t o_sched = 0;
    const size_t o_is = align((size_t)2 * std::max(SC, 1) * 4);
    const size_t o_ring = o_is + align((size_t)n_cb * nb * np);
    const size_t o_esum = o_ring + align((size_t)(pa->delay + 2) * n_cb * nb * (np / 32) * 4);
    const size_t esum_bytes = (size_t)2 * n_cb * nb * 4;
    const size_t o_item = o_esum + align(esum_bytes);
    const size_t total = o_item + sizeof(SweepArgs);
    retain_pool_memory(prob->device);
    void* mem = nullptr;
    hipError_t e = hipMallocAsync(&mem, total, stream);
    if (e != hipSuccess) return e;
    char* base = static_cast<char*>(mem);
    int32_t* d_sched = reinterpret_cast<int32_t*>(base + o_sched);
    SweepArgs a = make_args(prob, pa, out, d_sched, d_sched + std::max(SC, 1), reinterpret_cast<int8_t*>(base + o_is),
                            nullptr, nb, tpw, fp4 ? 1 : 0);
    a.n_cb = n_cb;
    a.n_groups = n_groups;
    a.group_tiles = group_tiles;
    a.split_k = split_k ? 4 : 1;
    a.ring = reinterpret_cast<uint32_t*>(base + o_ring);
    a.e_sum = reinterpret_cast<int32_t*>(base + o_esum);
    a.final_pass = 1;
    SweepArgs* d_args = reinterpret_cast<SweepArgs*>(base + o_item);
    {
        // schedules and arguments through pinned staging (no host wait); the init launch clears the energy slots
        const void* srcs[3] = {pa->jperp, pa->i0, &a};
        const size_t sizes[3] = {(size_t)SC * 4, (size_t)SC * 4, sizeof(SweepArgs)};
        if (SC > 0) e = staged_upload(prob->device, d_sched, srcs, sizes, 2, stream);
        if (e == hipSuccess) e = staged_upload(prob->device, d_args, srcs + 2, sizes + 2, 1, stream);
    }
    const int32_t *jp = pa->jperp, *ip = pa->i0;
    if (e == hipSuccess) e = launch_sweep_split(d_args, a, 0, kSplitInit, jp, ip, stream);
    for (int t = 0; e == hipSuccess && t < SC; ++t)
        e = launch_sweep_split(d_args, a, t, kSplitRun | kSplitUpdate | (t > 0 ? kSplitClose : 0), jp, ip, stream);
    // the energy of sigma(SC), then the close of its cycle
    if (e == hipSuccess) e = launch_sweep_split(d_args, a, SC, kSplitRun | (SC > 0 ? kSplitClose : 0), jp, ip, stream);
    if (e == hipSuccess) e = launch_sweep_split(d_args, a, SC + 1, kSplitClose, jp, ip, stream);
    if (e == hipSuccess && out->final_is)
        e = launch_copy_final_is(a.is_state, np, prob->dev.n, R, T, tpw, nb, out->final_is, stream);
    (void)hipFreeAsync(mem, stream);
    return e;
}

ssqa_status anneal_impl(const ssqa_problem* prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out,
                        hipStream_t stream, const AnnealWorkspace* ws) {
    if (!prob || !pa || !out) return fail(SSQA_EINVAL, "NULL problem, params or outputs");
    const ssqa_status st = check_params(prob, pa, out);
    if (st != SSQA_OK) return st;
    const int R = pa->replicas, T = pa->trials, SC = pa->cycles;
    const int t0 = pa->start_cycle;
    const int t1 = pa->stop_cycle == 0 ? SC : pa->stop_cycle;
    if (t0 < 0 || t0 > SC) return fail(SSQA_EINVAL, "start_cycle = %d outside [0, cycles = %d]", t0, SC);
    if (t1 < t0 || t1 > SC || (t1 == t0 && t1 != SC))
        return fail(SSQA_EINVAL, "stop_cycle = %d must lie in (start_cycle, cycles] (or be 0)", pa->stop_cycle);
    if (t0 > 0 && (!pa->resume || !pa->resume->counters || (pa->delay > 0 && !pa->resume->history)))
        return fail(SSQA_EINVAL, "start_cycle > 0 needs a resume state with counters (and history when d > 0)");
    const ssqa_anneal_state* ckpt = out->checkpoint;
    if (ckpt && (!ckpt->counters || (pa->delay > 0 && !ckpt->history)))
        return fail(SSQA_EINVAL, "checkpoint needs counters (and history when d > 0)");

    DeviceGuard guard(prob->device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice failed");
    const AnnealSizes z = anneal_sizes(prob, pa);
    const int nb = z.layout.nb, tpw = z.layout.tpw, n_wg = z.layout.n_wg;
    const int np = prob->dev.np;
    if (const int split_nb = plain_split_columns(prob, pa, t0, t1, ckpt != nullptr, ws != nullptr)) {
        const hipError_t se = anneal_split(prob, pa, out, split_nb, z.layout.fp4, stream);
        if (se != hipSuccess)
            return se == hipErrorOutOfMemory ? fail(SSQA_ENOMEM, "device allocation failed") : hip_fail(se, "anneal");
        return SSQA_OK;
    }

    int8_t* is_state = nullptr;
    uint32_t* hist = nullptr;
    int32_t* d_sched = nullptr;
    hipError_t e = hipSuccess;
    if (ws) {
        is_state = ws->is_state;
        hist = ws->hist;
        d_sched = ws->sched;
        // The caller's schedules go straight to the workspace; the host waits for the copy, so that no
        // staging memory is needed and the caller may free its arrays on return.
        if (SC > 0) e = hipMemcpyAsync(d_sched, pa->jperp, (size_t)SC * 4, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && SC > 0)
            e = hipMemcpyAsync(d_sched + SC, pa->i0, (size_t)SC * 4, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
    } else {
        retain_pool_memory(prob->device);
        e = hipMallocAsync(reinterpret_cast<void**>(&is_state), z.is_bytes, stream);
        if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&hist), z.hist_bytes, stream);
        if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&d_sched), z.sched_bytes, stream);
        if (e == hipSuccess && SC > 0) {
            // copied through pinned staging: the call returns without waiting for the device
            const void* srcs[2] = {pa->jperp, pa->i0};
            const size_t sizes[2] = {(size_t)SC * 4, (size_t)SC * 4};
            e = staged_upload(prob->device, d_sched, srcs, sizes, 2, stream);
        }
    }
    // [jperp | i0], SC entries each (one unused word each when SC = 0)
    const int32_t* d_jperp = d_sched;
    const int32_t* d_i0 = d_sched + std::max(SC, 1);

    if (e == hipSuccess && t0 > 0)
        e = launch_import_state(pa->resume->counters, pa->resume->history, prob->dev.n, np, R, T, tpw, nb, pa->delay,
                                is_state, hist, stream);
    if (e == hipSuccess) {
        SweepArgs a = make_args(prob, pa, out, d_jperp, d_i0, is_state, hist, nb, tpw, z.layout.fp4 ? 1 : 0);
        const int chunk = pa->cycles_per_launch > 0 ? pa->cycles_per_launch : std::max(t1 - t0, 1);
        int t = t0;
        do {
            a.t_begin = t;
            a.t_end = std::min(t1, t + chunk);
            a.final_pass = (a.t_end == SC) ? 1 : 0;
            a.save_hist = (!a.final_pass || ckpt) ? 1 : 0;
            e = launch_sweep(a, n_wg, stream);
            t = a.t_end;
        } while (e == hipSuccess && t < t1);
        if (e == hipSuccess && out->final_is)
            e = launch_copy_final_is(is_state, np, prob->dev.n, R, T, tpw, nb, out->final_is, stream);
        if (e == hipSuccess && ckpt) {
            e = launch_copy_final_is(is_state, np, prob->dev.n, R, T, tpw, nb, ckpt->counters, stream);
            if (e == hipSuccess && pa->delay > 0)
                e = launch_export_history(hist, prob->dev.n, np, R, T, tpw, nb, pa->delay, ckpt->history, stream);
        }
    }
    if (!ws) {
        if (is_state) (void)hipFreeAsync(is_state, stream);
        if (hist) (void)hipFreeAsync(hist, stream);
        if (d_sched) (void)hipFreeAsync(d_sched, stream);
    }
    if (e != hipSuccess) {
        return e == hipErrorOutOfMemory ? fail(SSQA_ENOMEM, "device allocation failed") : hip_fail(e, "anneal");
    }
    return SSQA_OK;
}

// Checks and statistics of J (scan_couplings).
CouplingScan scan_couplings(int n, const int32_t* h, const int32_t* J, int8_t* J8) {
    // Checks and statistics of J in one pass per row block, over host threads for large N (each pass streams
    // N^2 int32 values, 400 MB at N = 10^4):
    //   symmetry, 64 x 64 blocks against their mirrors (a column-order scan would miss the cache on every
    //   element), and per row the zero diagonal, sum |J_ij|, extremes and whether every entry has an fp4 code.
    // Failures are reported in a fixed order (first asymmetric pair in row order, then first non-zero diagonal
    // entry, then the range), whatever the thread count.
    constexpr int kB = 64;
    const int nblk = (n + kB - 1) / kB;
    auto scan = [&](int blk_lo, int blk_hi, CouplingScan& part) {
        for (int b = blk_lo; b < blk_hi; ++b) {
            const int bi = b * kB, ie = std::min(n, bi + kB);
            for (int bj = bi; bj < n; bj += kB) {
                const int je = std::min(n, bj + kB);
                for (int i = bi; i < ie; ++i)
                    for (int j = std::max(bj, i + 1); j < je; ++j)
                        if (J[(size_t)i * n + j] != J[(size_t)j * n + i]) {
                            const long long k = (long long)i * n + j;
                            if (part.first_asym < 0 || k < part.first_asym) part.first_asym = k;
                        }
            }
            for (int i = bi; i < ie; ++i) {
                const int32_t* row = J + (size_t)i * n;
                int8_t* row8 = J8 ? J8 + (size_t)i * n : nullptr;
                if (row[i] != 0 && part.first_diag < 0) part.first_diag = i;
                // The balanced base-256 digits a value needs grow with its distance from zero on either side,
                // so the row's extremes decide its plane count.
                long long row_abs = 0;
                int32_t vmin = 0, vmax = 0;
                int bad_codes = 0;
                for (int j = 0; j < n; ++j) {
                    const int32_t v = row[j];
                    const long long m = v < 0 ? -(long long)v : (long long)v;
                    row_abs += m;
                    vmin = std::min(vmin, v);
                    vmax = std::max(vmax, v);
                    bad_codes |= (m > 6) | (m == 5);
                }
                if (row8)
                    for (int j = 0; j < n; ++j) row8[j] = (int8_t)row[j];
                const long long ha = std::llabs((long long)h[i]);
                part.total += row_abs + 2 * ha;
                part.planes = std::max({part.planes, planes_needed(vmin), planes_needed(vmax)});
                if (bad_codes) part.codes = false;
                part.bound = std::max(part.bound, ha + 2 * row_abs);
            }
        }
    };
    const int threads = (long long)n * n >= (1LL << 22)
                            ? std::max(1, std::min({8, nblk, (int)std::thread::hardware_concurrency()}))
                            : 1;
    std::vector<CouplingScan> parts(threads);
    if (threads == 1) {
        scan(0, nblk, parts[0]);
    } else {
        // Row blocks dealt in an interleaved order, since the symmetry work of block b shrinks with b.
        std::vector<std::thread> pool;
        std::vector<std::vector<int>> mine(threads);
        for (int b = 0; b < nblk; ++b) mine[b % threads].push_back(b);
        for (int w = 0; w < threads; ++w)
            pool.emplace_back([&, w] {
                for (const int b : mine[w]) scan(b, b + 1, parts[w]);
            });
        for (std::thread& th : pool) th.join();
    }
    CouplingScan all;
    for (const CouplingScan& q : parts) {
        if (q.first_asym >= 0 && (all.first_asym < 0 || q.first_asym < all.first_asym)) all.first_asym = q.first_asym;
        if (q.first_diag >= 0 && (all.first_diag < 0 || q.first_diag < all.first_diag)) all.first_diag = q.first_diag;
        all.total += q.total;
        all.planes = std::max(all.planes, q.planes);
        all.codes = all.codes && q.codes;
        all.bound = std::max(all.bound, q.bound);
    }
    return all;
}

// The failure a scan found, in a fixed order: first asymmetric pair in row order, first non-zero diagonal
// entry, then the int32 range.
ssqa_status check_couplings(const CouplingScan& all, int n, const int32_t* J) {
    if (all.first_asym >= 0)
        return fail(SSQA_EINVAL, "J not symmetric at (%d, %d)", (int)(all.first_asym / n), (int)(all.first_asym % n));
    if (all.first_diag >= 0)
        return fail(SSQA_EINVAL, "J[%d][%d] = %d, diagonal must be zero", all.first_diag, all.first_diag,
                    J[(size_t)all.first_diag * n + all.first_diag]);
    if (all.total >= (1LL << 30)) return fail(SSQA_ERANGE, "2 sum|h| + sum|J| >= 2^30: int32 fields could overflow");
    return SSQA_OK;
}

ssqa_status create_problem_impl(int32_t n, const int32_t* h, const int32_t* J, const int8_t* J8,
                                const CouplingScan& sc, int32_t device, ssqa_problem_t* out) {
    const int planes = sc.planes;
    const bool fp4_codes = sc.codes;        // every J_ij in {0, +-1, +-2, +-3, +-4, +-6}
    const long long fp4_bound = sc.bound;   // max_i (|h_i| + 2 sum_j |J_ij|), see fp4_fits
    // The fp4 copy is built when J is representable and at least an anneal without noise and coupling keeps
    // the fp32 accumulation exact; each anneal checks its own bound (fp4_fits).
    const bool fp4_exact = fp4_codes && fp4_bound + 128 < (1LL << 22);
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count == 0)
        return fail(SSQA_EDEVICE, "no HIP device available");
    if (device < 0 || device >= dev_count) return fail(SSQA_EINVAL, "device %d outside [0, %d)", device, dev_count);
    DeviceGuard guard(device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice(%d) failed", device);

    const int np = (n + kTileRows - 1) / kTileRows * kTileRows;
    ssqa_problem* p = new (std::nothrow) ssqa_problem();
    if (!p) return fail(SSQA_ENOMEM, "host allocation failed");
    p->device = device;
    p->fp4_bound = fp4_bound;
    void* Jdev = nullptr;   // J on the device as given: int8 (one plane) or int32
    int32_t* h32 = nullptr;
    const size_t plane_bytes = (size_t)planes * np * np;
    const int kp4 = fp4_k_extent(np);
    hipError_t e = hipMalloc(&p->J_planes, plane_bytes);
    if (e == hipSuccess && fp4_exact) e = hipMalloc(&p->J_fp4, (size_t)np * kp4 / 2);
    if (e == hipSuccess) e = hipMalloc(&p->rowvec, (size_t)np * 4 * 3);
    const int elem = J8 ? 1 : 4;
    if (e == hipSuccess) e = hipMalloc(&Jdev, (size_t)n * n * elem);
    if (e == hipSuccess) e = hipMalloc(&h32, (size_t)n * 4);
    if (e == hipSuccess)
        e = hipMemcpy(Jdev, J8 ? static_cast<const void*>(J8) : static_cast<const void*>(J), (size_t)n * n * elem,
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h32, h, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_prepare_planes(Jdev, elem, h32, n, np, planes, p->J_planes, p->rowvec, nullptr);
    if (e == hipSuccess && fp4_exact) e = launch_prepare_fp4(Jdev, elem, n, np, kp4, p->J_fp4, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (Jdev) (void)hipFree(Jdev);
    if (h32) (void)hipFree(h32);
    if (e != hipSuccess) {
        ssqa_destroy_problem(p);
        return e == hipErrorOutOfMemory ? fail(SSQA_ENOMEM, "device allocation failed")
                                        : hip_fail(e, "create_problem");
    }
    p->dev.n = n;
    p->dev.np = np;
    p->dev.planes = planes;
    p->dev.J = p->J_planes;
    p->dev.J4 = p->J_fp4;
    p->dev.kp4 = kp4;
    p->dev.h = p->rowvec;
    p->dev.hr = p->rowvec + np;
    p->dev.er = p->rowvec + 2 * np;
    *out = p;
    return SSQA_OK;
}

}  // namespace detail
}  // namespace ssqa

using namespace ssqa::detail;

struct ssqa_batch {
    int device = 0;
    int blocks = 0;
    void* mem = nullptr;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* ssqa_status_string(ssqa_status s) {
    // A C caller may pass any int; reading the argument's bits as an int avoids loading an enum value outside
    // the enumeration's range, which C++ leaves undefined.
    int v;
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
        case SSQA_OK: return "SSQA_OK";
        case SSQA_EINVAL: return "SSQA_EINVAL";
        case SSQA_ENOMEM: return "SSQA_ENOMEM";
        case SSQA_ERANGE: return "SSQA_ERANGE";
        case SSQA_EDEVICE: return "SSQA_EDEVICE";
        case SSQA_ENOTSUP: return "SSQA_ENOTSUP";
    }
    return "SSQA_UNKNOWN";
}

const char* ssqa_last_error(void) { return g_last_error.c_str(); }

ssqa_status ssqa_create_problem(int32_t n, const int32_t* h, const int32_t* J, int32_t device,
                                ssqa_problem_t* out) {
    g_last_error.clear();
    if (!out) return fail(SSQA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 16384) return fail(SSQA_EINVAL, "n_spins = %d outside [1, 16384]", n);
    if (!h || !J) return fail(SSQA_EINVAL, "h or J is NULL");
    // Large problems are narrowed to int8 during the checking pass when J fits one plane, so that a quarter of
    // the bytes crosses to the device.
    std::unique_ptr<int8_t[]> j8;
    if ((long long)n * n >= (1LL << 20)) j8.reset(new (std::nothrow) int8_t[(size_t)n * n]);
    const CouplingScan sc = scan_couplings(n, h, J, j8.get());
    const ssqa_status st = check_couplings(sc, n, J);
    if (st != SSQA_OK) return st;
    return create_problem_impl(n, h, J, sc.planes == 1 ? j8.get() : nullptr, sc, device, out);
}

void ssqa_destroy_problem(ssqa_problem_t p) {
    if (!p) return;
    DeviceGuard guard(p->device);
    if (p->J_planes) (void)hipFree(p->J_planes);
    if (p->J_fp4) (void)hipFree(p->J_fp4);
    if (p->rowvec) (void)hipFree(p->rowvec);
    delete p;
}

int32_t ssqa_problem_spins(ssqa_problem_t p) { return p ? p->dev.n : 0; }
int32_t ssqa_problem_planes(ssqa_problem_t p) { return p ? p->dev.planes : 0; }
int32_t ssqa_problem_padded(ssqa_problem_t p) { return p ? p->dev.np : 0; }
int32_t ssqa_problem_fp4_exact(ssqa_problem_t p) { return p && p->J_fp4 ? 1 : 0; }

ssqa_status ssqa_anneal(ssqa_problem_t prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out,
                        void* hip_stream) {
    g_last_error.clear();
    return anneal_impl(prob, pa, out, reinterpret_cast<hipStream_t>(hip_stream), nullptr);
}

ssqa_status ssqa_anneal_noalloc(ssqa_problem_t prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out,
                                void* hip_stream) {
    g_last_error.clear();
    if (!prob || !pa || !out) return fail(SSQA_EINVAL, "NULL problem, params or outputs");
    const ssqa_status st = check_params(prob, pa, out);   // anneal_sizes needs valid parameters
    if (st != SSQA_OK) return st;
    const AnnealSizes z = anneal_sizes(prob, pa);
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t o_hist = align(z.is_bytes);
    const size_t o_sched = o_hist + align(z.hist_bytes);
    const size_t need = o_sched + align(z.sched_bytes);
    if (need > kFixedScratchBytes)
        return fail(SSQA_ENOTSUP, "anneal needs %zu bytes of device state; the fixed scratch of ssqa_anneal_noalloc "
                                  "holds %zu (use ssqa_anneal)", need, kFixedScratchBytes);
    DeviceGuard guard(prob->device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice failed");
    void* base = nullptr;
    const hipError_t e = fixed_scratch(prob->device, &base);
    if (e != hipSuccess) return hip_fail(e, "address of the fixed scratch");
    char* p = static_cast<char*>(base);
    const AnnealWorkspace ws{reinterpret_cast<int8_t*>(p), reinterpret_cast<uint32_t*>(p + o_hist),
                             reinterpret_cast<int32_t*>(p + o_sched)};
    return anneal_impl(prob, pa, out, reinterpret_cast<hipStream_t>(hip_stream), &ws);
}

}  // extern "C"

namespace ssqa {
namespace detail {

ssqa_status batch_create_impl(int32_t count, const ssqa_problem_t* problems, const ssqa_anneal_params* params,
                              const ssqa_anneal_outputs* outputs, ssqa_batch_t* out, int wide_rows) {
    if (!out) return fail(SSQA_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > 65535) return fail(SSQA_EINVAL, "count = %d outside [1, 65535]", count);
    if (!problems || !params || !outputs) return fail(SSQA_EINVAL, "NULL problems, params or outputs");
    const int device = problems[0] ? problems[0]->device : -1;
    // 128-column floor: the caller's, else the autotuner's for this batch, else the built-in one
    if (wide_rows < 0 && problems[0]) {
        bool all = true;
        for (int i = 0; i < count && all; ++i) all = problems[i] != nullptr;
        if (all) wide_rows = tuned_batch_rows(device, batch_signature(count, problems, params));
    }
    if (wide_rows < 0) wide_rows = kBatchWideRows;
    // sizes and validation
    size_t sched_words = 0, is_bytes = 0;
    std::vector<int> n_wg(count), tpw(count), nbs(count);
    for (int i = 0; i < count; ++i) {
        const ssqa_problem* p = problems[i];
        if (!p) return fail(SSQA_EINVAL, "problems[%d] is NULL", i);
        if (p->device != device) return fail(SSQA_EINVAL, "problems[%d] is on another device", i);
        const ssqa_status st = check_params(p, &params[i], &outputs[i]);
        if (st != SSQA_OK) {
            const std::string msg = g_last_error;
            return fail(st, "anneal %d: %s", i, msg.c_str());
        }
        if (params[i].cycles_per_launch != 0) return fail(SSQA_EINVAL, "anneal %d: cycles_per_launch must be 0", i);
        if (params[i].start_cycle != 0 || (params[i].stop_cycle != 0 && params[i].stop_cycle != params[i].cycles) ||
            outputs[i].checkpoint)
            return fail(SSQA_EINVAL, "anneal %d: start_cycle, stop_cycle and checkpoint are for ssqa_anneal", i);
        nbs[i] = wide_blocks_pay(p, &params[i], wide_rows) ? 128 : block_columns(p, &params[i]);
        tpw[i] = nbs[i] / params[i].replicas;
        n_wg[i] = (params[i].trials + tpw[i] - 1) / tpw[i];
        if (n_wg[i] > 65535) return fail(SSQA_ENOTSUP, "anneal %d needs more than 65535 blocks", i);
        sched_words += 2 * (size_t)std::max(params[i].cycles, 1);
        is_bytes += (size_t)n_wg[i] * nbs[i] * p->dev.np;
    }
    DeviceGuard guard(device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice failed");

    auto* b = new (std::nothrow) ssqa_batch();
    if (!b) return fail(SSQA_ENOMEM, "host allocation failed");
    b->device = device;
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t total_work = 0;
    for (int i = 0; i < count; ++i) total_work += n_wg[i];
    const size_t off_items = 0;
    const size_t off_work = align(off_items + sizeof(SweepArgs) * count);
    const size_t off_sched = align(off_work + sizeof(uint32_t) * total_work);
    const size_t off_is = align(off_sched + sizeof(int32_t) * sched_words);
    const size_t bytes = align(off_is + is_bytes);
    hipError_t e = hipMalloc(&b->mem, bytes);
    if (e != hipSuccess) {
        delete b;
        return fail(SSQA_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    char* base = static_cast<char*>(b->mem);
    auto* d_items = reinterpret_cast<SweepArgs*>(base + off_items);
    auto* d_work = reinterpret_cast<uint32_t*>(base + off_work);
    auto* d_sched = reinterpret_cast<int32_t*>(base + off_sched);
    int8_t* d_is = reinterpret_cast<int8_t*>(base + off_is);

    // host images of the argument blocks, the schedules and the work lists (one per kernel variant)
    std::vector<SweepArgs> items(count);
    std::vector<int32_t> sched(sched_words);
    size_t so = 0, io = 0;
    constexpr int kVariants = kSweepVariants;
    std::vector<WorkItem> lists[kVariants];
    int max_np[kVariants] = {}, max_delay[kVariants] = {};
    for (int i = 0; i < count; ++i) {
        const ssqa_anneal_params& pa = params[i];
        const int SC = pa.cycles;
        int32_t* jp = d_sched + so;
        int32_t* i0 = d_sched + so + std::max(SC, 1);
        if (SC > 0) {
            std::memcpy(&sched[so], pa.jperp, (size_t)SC * 4);
            std::memcpy(&sched[so + std::max(SC, 1)], pa.i0, (size_t)SC * 4);
        }
        so += 2 * (size_t)std::max(SC, 1);
        items[i] = make_args(problems[i], &pa, &outputs[i], jp, i0, d_is + io, nullptr, nbs[i], tpw[i]);
        items[i].t_begin = 0;
        items[i].t_end = SC;
        items[i].final_pass = 1;
        io += (size_t)n_wg[i] * nbs[i] * problems[i]->dev.np;
        const int v = sweep_variant(items[i].fast != 0, pa.coupling_mode, nbs[i], items[i].fp4 != 0);
        const double np = problems[i]->dev.np;
        const double cost = np * np * problems[i]->dev.planes * (SC + 1.0);
        for (int c = 0; c < n_wg[i]; ++c) lists[v].push_back({cost, ((uint32_t)i << 16) | (uint32_t)c});
        max_np[v] = std::max(max_np[v], problems[i]->dev.np);
        max_delay[v] = std::max(max_delay[v], pa.delay);
    }
    std::vector<uint32_t> work;
    size_t list_off[kVariants], list_len[kVariants];
    const int xcds = device_xcd_count(device);
    for (int v = 0; v < kVariants; ++v) {
        std::stable_sort(lists[v].begin(), lists[v].end(), [](const WorkItem& x, const WorkItem& y) { return x.cost > y.cost; });
        lists[v] = xcd_grouped(lists[v], xcds);
        list_off[v] = work.size();
        list_len[v] = lists[v].size();
        for (const WorkItem& en : lists[v]) work.push_back(en.code);
        if (list_len[v] && sweep_lds_bytes(max_np[v], max_delay[v], variant_columns(v)) > 160 * 1024) {
            ssqa_batch_destroy(b);
            return fail(SSQA_ENOTSUP, "batch needs more than 160 KiB of LDS per workgroup");
        }
    }
    e = hipMemcpy(d_items, items.data(), sizeof(SweepArgs) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_work, work.data(), sizeof(uint32_t) * work.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !sched.empty())
        e = hipMemcpy(d_sched, sched.data(), sizeof(int32_t) * sched.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = configure_sweep_kernels();
    // record the launches once; every run replays them
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        for (int v = 0; v < kVariants && le == hipSuccess; ++v) {
            if (!list_len[v]) continue;
            le = launch_sweep_batch(d_items, d_work + list_off[v], (int)list_len[v], max_np[v], max_delay[v], v,
                                    b->capture);
        }
        for (int i = 0; i < count && le == hipSuccess; ++i) {
            if (!outputs[i].final_is) continue;
            le = launch_copy_final_is(items[i].is_state, problems[i]->dev.np, problems[i]->dev.n, params[i].replicas,
                                      params[i].trials, tpw[i], nbs[i], outputs[i].final_is, b->capture);
        }
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->capture, &g);
        b->graph = g;
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        ssqa_batch_destroy(b);
        return hip_fail(e, "batch_create");
    }
    b->blocks = (int)work.size();
    *out = b;
    return SSQA_OK;
}

}  // namespace detail
}  // namespace ssqa

extern "C" {

ssqa_status ssqa_batch_create(int32_t count, const ssqa_problem_t* problems, const ssqa_anneal_params* params,
                              const ssqa_anneal_outputs* outputs, ssqa_batch_t* out) {
    g_last_error.clear();
    return batch_create_impl(count, problems, params, outputs, out, -1);
}

ssqa_status ssqa_batch_run(ssqa_batch_t b, void* hip_stream) {
    g_last_error.clear();
    if (!b) return fail(SSQA_EINVAL, "batch is NULL");
    DeviceGuard guard(b->device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice failed");
    SSQA_HIP(hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(hip_stream)), "batch_run");
    return SSQA_OK;
}

int32_t ssqa_batch_blocks(ssqa_batch_t b) { return b ? b->blocks : 0; }

void ssqa_batch_destroy(ssqa_batch_t b) {
    if (!b) return;
    DeviceGuard guard(b->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

ssqa_status ssqa_energy(ssqa_problem_t prob, const int8_t* spins, int32_t cols, int64_t* energies, void* hip_stream) {
    g_last_error.clear();
    if (!prob || !spins || !energies) return fail(SSQA_EINVAL, "NULL argument");
    if (cols < 0) return fail(SSQA_EINVAL, "cols < 0");
    if (cols == 0) return SSQA_OK;
    DeviceGuard guard(prob->device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice failed");
    SSQA_HIP(launch_energy(prob->dev, spins, cols, energies, reinterpret_cast<hipStream_t>(hip_stream)), "energy");
    return SSQA_OK;
}

ssqa_status ssqa_qmc_energy(ssqa_problem_t prob, const int8_t* counters, int32_t trials, int32_t replicas,
                            int32_t jperp, int64_t* energies, void* hip_stream) {
    g_last_error.clear();
    if (!prob || !counters || !energies) return fail(SSQA_EINVAL, "NULL argument");
    if (trials < 0 || replicas < 1) return fail(SSQA_EINVAL, "trials must be >= 0 and replicas >= 1");
    if (jperp < -(1 << 20) || jperp > (1 << 20)) return fail(SSQA_EINVAL, "jperp outside [-2^20, 2^20]");
    if (trials == 0) return SSQA_OK;
    DeviceGuard guard(prob->device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice failed");
    SSQA_HIP(launch_qmc_energy(prob->dev, counters, trials, replicas, jperp, energies,
                               reinterpret_cast<hipStream_t>(hip_stream)), "qmc_energy");
    return SSQA_OK;
}

ssqa_status ssqa_sa_anneal(ssqa_problem_t prob, const ssqa_sa_params* pa, const ssqa_sa_outputs* out,
                           void* hip_stream) {
    g_last_error.clear();
    if (!prob || !pa || !out) return fail(SSQA_EINVAL, "NULL problem, params or outputs");
    if (pa->trials < 1 || pa->trials > (1 << 24)) return fail(SSQA_EINVAL, "trials = %d outside [1, 2^24]", pa->trials);
    if (pa->cycles < 0) return fail(SSQA_EINVAL, "cycles < 0");
    if (pa->cycles > 0 && !pa->beta) return fail(SSQA_EINVAL, "beta is required");
    for (int t = 0; t < pa->cycles; ++t)
        if (!(pa->beta[t] >= 0.0) || !std::isfinite(pa->beta[t]))
            return fail(SSQA_EINVAL, "beta[%d] is negative or not finite", t);
    if (!out->best_energy || !out->first_hit) return fail(SSQA_EINVAL, "best_energy and first_hit are required");
    if (sa_waves_per_group(prob->dev.np) < 1) return fail(SSQA_ENOTSUP, "N = %d: one chain does not fit in LDS", prob->dev.n);
    DeviceGuard guard(prob->device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice(%d) failed", prob->device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    retain_pool_memory(prob->device);
    double* d_beta = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&d_beta), sizeof(double) * std::max(pa->cycles, 1), stream);
    if (e == hipSuccess && pa->cycles > 0) {
        const void* src = pa->beta;
        const size_t bytes = sizeof(double) * pa->cycles;
        e = staged_upload(prob->device, d_beta, &src, &bytes, 1, stream);
    }
    if (e == hipSuccess) {
        SAArgs a{};
        a.prob = prob->dev;
        a.T = pa->trials;
        a.cycles = pa->cycles;
        a.beta = d_beta;
        a.key0 = (uint32_t)(pa->seed & 0xFFFFFFFFu);
        a.key1 = (uint32_t)(pa->seed >> 32);
        a.target = pa->target_energy;
        a.best = out->best_energy;
        a.first_hit = out->first_hit;
        a.final_energy = out->final_energy;
        a.final_spins = out->final_spins;
        a.trace = out->energy_trace;
        e = launch_sa(a, stream);
    }
    if (d_beta) (void)hipFreeAsync(d_beta, stream);
    if (e != hipSuccess) return hip_fail(e, "sa_anneal");
    return SSQA_OK;
}

void ssqa_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const Philox4 r = philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    for (int w = 0; w < 4; ++w) out[w] = r.v[w];
}

}  // extern "C"
