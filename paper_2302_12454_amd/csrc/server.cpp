// Serving: continuous batching of anneal requests (see include/ssqa.h, "Serving").
//
// Requests wait in a FIFO queue.  Every step admits requests from the head of the queue while the device
// memory they need (problem planes + counters + bit-plane history + outputs) fits the budget and the slot
// limit allows, then runs K cycles of every admitted request in one launch of the batch kernel (each
// request continues from its own cycle; its counters and delayed bit planes stay in device memory between
// steps), reads back the per-trial best energies, and retires requests that reached their target (early
// exit) or their last cycle, releasing their memory.  A request's results depend only on its own inputs:
// the random stream is keyed by its seed and its own cycle counter, and retirement is decided at its own
// cycle boundaries, so a request gives the same result alone or among others.
//
// A request of large N would otherwise run on few workgroups (one per block of whole trials), each reading all
// of J every cycle.  From `split_rows` padded rows on it takes the row-split form instead: every block of
// trials is spread over row groups of workgroups, one launch per cycle on a second stream beside the
// persistent launch of the other requests, with sigma exchanged through device memory and the kernel boundary
// as the per-cycle barrier.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "internal.hpp"
#include "work_order.hpp"

using namespace ssqa;
using namespace ssqa::detail;

namespace {

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Request {
    int64_t id = 0;
    int32_t state = SSQA_REQ_QUEUED;
    int32_t status = SSQA_OK;
    int32_t early_exit = 0;
    int n = 0;
    int planes = 1;
    std::vector<int32_t> h, J;           // host copies until admission (J as int32 only when it needs planes > 1)
    std::unique_ptr<int8_t[]> J8;        // J narrowed to int8 (one plane), until admission
    CouplingScan scan;                   // checks and statistics of J, from submit
    ssqa_anneal_params params{};
    std::vector<int32_t> jperp, i0;
    // device side, from admission to retirement
    ssqa_problem_t prob = nullptr;
    void* mem = nullptr;                 // schedules | counters | history | best | first_hit
    int64_t bytes = 0;
    int nb = 64, n_wg = 0;
    bool split = false;                  // row-split form (args.n_groups row groups per block of trials)
    SweepArgs* d_args = nullptr;         // device copy of args (split form)
    SweepArgs args{};
    int cycle = 0;
    // results
    std::vector<int64_t> best;
    std::vector<int32_t> first_hit;
    double submit_s = 0, admit_s = -1, done_s = -1;
};

int padded_rows(int n) { return (n + kTileRows - 1) / kTileRows * kTileRows; }

// Workgroups of a request: whole trials per block of the width admission takes (block_columns_for), at least
// one trial per block (a request whose replicas exceed the width is refused at admission).
int64_t request_blocks(int n, const ssqa_anneal_params& pa) {
    const int nb = block_columns_for(padded_rows(n), &pa);
    const int64_t tpw = std::max(1, nb / pa.replicas);
    return (pa.trials + tpw - 1) / tpw;
}

// Padded rows from which a request takes the row-split form (0 in the configuration: 4096; -1: never).
int split_floor(int split_rows) { return split_rows == 0 ? 4096 : split_rows < 0 ? INT32_MAX : split_rows; }

// Whether a request takes the row-split form: enough rows, and a block narrower than 128 columns.
bool takes_split(int np, int nb, int split_rows) { return np >= split_floor(split_rows) && nb <= 64; }

// Device bytes of one admitted request: int8 planes, the fp4 copy of J (counted whether or not the
// problem turns out to be fp4-exact), row vectors, counters, bit-plane history (or, in the row-split form,
// the bit-plane ring and energy sums), outputs, schedules.
int64_t request_bytes(int n, int planes_hint, const ssqa_anneal_params& pa, int split_rows) {
    const int64_t np = padded_rows(n);
    const int64_t kp4 = fp4_k_extent((int)np);
    const int64_t nb = block_columns_for((int)np, &pa);
    const int64_t n_wg = request_blocks(n, pa);
    const int64_t state = takes_split((int)np, (int)nb, split_rows)
                              ? (pa.delay + 2LL) * n_wg * nb * np / 8 + 8 * n_wg * nb + (int64_t)sizeof(SweepArgs)
                              : n_wg * std::max(pa.delay, 1) * nb * np / 8;
    return planes_hint * np * np + np * kp4 / 2 + 12 * np + n_wg * nb * np + state + 12LL * pa.trials +
           8LL * std::max(pa.cycles, 1) + 4096;
}

}  // namespace

struct ssqa_server {
    ssqa_server_config cfg{};
    std::chrono::steady_clock::time_point t0;
    int64_t next_id = 1;
    int64_t bytes_in_use = 0;
    std::deque<Request*> queue;
    std::vector<Request*> active;
    std::map<int64_t, std::unique_ptr<Request>> all;
    // per-step launch tables (device) and their host images
    void* table = nullptr;
    size_t table_bytes = 0;
    std::vector<SweepArgs> items;
    std::vector<uint32_t> work;
    int64_t cycles_run = 0;
    double spin_updates = 0;
    // streams of the row-split requests' launches (request k of a step on stream k mod kSideStreams, so that
    // several large requests advance together), the event that forks them from the caller's stream and one
    // per stream that joins it back (created at the first split request)
    static constexpr int kSideStreams = 4;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSideStreams] = {};
};

namespace {

void release_device(Request* r) {
    if (r->mem) (void)hipFree(r->mem);
    r->mem = nullptr;
    if (r->prob) ssqa_destroy_problem(r->prob);
    r->prob = nullptr;
}

// Upload the problem and allocate the request's state; returns SSQA_OK or the failure.
ssqa_status admit(ssqa_server* s, Request* r) {
    // J was checked at submit; its int8 copy (or int32 one when it needs several planes) goes to the device
    ssqa_status st = create_problem_impl(r->n, r->h.data(), r->J8 ? nullptr : r->J.data(), r->J8.get(), r->scan,
                                         s->cfg.device, &r->prob);
    if (st != SSQA_OK) return st;
    ssqa_anneal_params& pa = r->params;
    pa.jperp = r->jperp.data();
    pa.i0 = r->i0.data();
    const ssqa_anneal_outputs probe{reinterpret_cast<int64_t*>(1), reinterpret_cast<int32_t*>(1), nullptr, nullptr};
    st = check_params(r->prob, &pa, &probe);
    if (st != SSQA_OK) return st;
    r->nb = block_columns(r->prob, &pa);
    const int tpw = r->nb / pa.replicas;   // >= 1: check_params refused R > nb
    r->n_wg = (pa.trials + tpw - 1) / tpw;
    if (r->n_wg > 65535) return fail(SSQA_EINVAL, "request needs %d workgroups (> 65535)", r->n_wg);
    const int np = r->prob->dev.np;
    r->split = takes_split(np, r->nb, s->cfg.split_rows);
    const int n_groups = r->split ? split_groups(np, device_xcd_count(s->cfg.device)) : 0;
    if (r->split && (int64_t)n_groups * r->n_wg > (1LL << 30))
        return fail(SSQA_EINVAL, "request needs too many row-split workgroups");
    const int SC = std::max(pa.cycles, 1);
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t o_sched = 0;
    const size_t o_is = align((size_t)2 * SC * 4);
    const size_t is_bytes = (size_t)r->n_wg * r->nb * np;
    const size_t o_hist = o_is + align(is_bytes);
    // history for the persistent form; the ring of d + 2 planes and two energy slots for the row-split form
    const size_t hist_bytes = r->split ? (size_t)(pa.delay + 2) * r->n_wg * r->nb * (np / 32) * 4
                                       : (size_t)r->n_wg * std::max(pa.delay, 1) * r->nb * (np / 32) * 4;
    const size_t o_esum = o_hist + align(hist_bytes);
    const size_t esum_bytes = r->split ? (size_t)2 * r->n_wg * r->nb * 4 : 0;
    const size_t o_item = o_esum + align(esum_bytes);
    const size_t o_best = o_item + align(r->split ? sizeof(SweepArgs) : 0);
    const size_t o_hit = o_best + align((size_t)pa.trials * 8);
    const size_t total = o_hit + (size_t)pa.trials * 4;
    DeviceGuard guard(s->cfg.device);
    if (hipMalloc(&r->mem, total) != hipSuccess) return fail(SSQA_ENOMEM, "device allocation of %zu bytes failed", total);
    char* base = static_cast<char*>(r->mem);
    int32_t* d_jperp = reinterpret_cast<int32_t*>(base + o_sched);
    int32_t* d_i0 = d_jperp + SC;
    if (pa.cycles > 0) {
        if (hipMemcpy(d_jperp, r->jperp.data(), (size_t)pa.cycles * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_i0, r->i0.data(), (size_t)pa.cycles * 4, hipMemcpyHostToDevice) != hipSuccess)
            return fail(SSQA_EDEVICE, "schedule upload failed");
    }
    const ssqa_anneal_outputs outs{reinterpret_cast<int64_t*>(base + o_best), reinterpret_cast<int32_t*>(base + o_hit),
                                   nullptr, nullptr};
    r->args = make_args(r->prob, &pa, &outs, d_jperp, d_i0, reinterpret_cast<int8_t*>(base + o_is),
                        reinterpret_cast<uint32_t*>(base + o_hist));
    if (r->split) {
        SweepArgs& a = r->args;
        a.hist_state = nullptr;
        a.n_cb = r->n_wg;
        a.n_groups = n_groups;
        a.group_tiles = kGroupTiles;
        a.ring = reinterpret_cast<uint32_t*>(base + o_hist);
        a.e_sum = reinterpret_cast<int32_t*>(base + o_esum);
        r->d_args = reinterpret_cast<SweepArgs*>(base + o_item);
        // the energy slots start at zero (each close clears the slot it read); the arguments never change
        if (hipMemset(a.e_sum, 0, esum_bytes) != hipSuccess ||
            hipMemcpy(r->d_args, &a, sizeof(SweepArgs), hipMemcpyHostToDevice) != hipSuccess)
            return fail(SSQA_EDEVICE, "row-split state upload failed");
    }
    r->bytes = (int64_t)total + (int64_t)r->prob->dev.planes * np * np + 12LL * np;
    r->cycle = 0;
    r->best.assign(pa.trials, INT64_MAX);
    r->first_hit.assign(pa.trials, -1);
    // host copies of the problem are no longer needed
    std::vector<int32_t>().swap(r->h);
    std::vector<int32_t>().swap(r->J);
    r->J8.reset();
    return SSQA_OK;
}

}  // namespace

extern "C" {

ssqa_status ssqa_server_create(const ssqa_server_config* cfg, ssqa_server_t* out) {
    g_last_error.clear();
    if (!cfg || !out) return fail(SSQA_EINVAL, "NULL config or out");
    *out = nullptr;
    if (cfg->cycles_per_step < 1) return fail(SSQA_EINVAL, "cycles_per_step must be >= 1");
    if (cfg->max_active < 1 || cfg->max_active > 65535) return fail(SSQA_EINVAL, "max_active outside [1, 65535]");
    if (cfg->memory_budget < 1) return fail(SSQA_EINVAL, "memory_budget must be positive");
    if (cfg->device < 0) return fail(SSQA_EINVAL, "device must be >= 0");
    auto* s = new (std::nothrow) ssqa_server();
    if (!s) return fail(SSQA_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return SSQA_OK;
}

ssqa_status ssqa_server_submit(ssqa_server_t s, const ssqa_request* req, int64_t* id) {
    g_last_error.clear();
    if (!s || !req || !id) return fail(SSQA_EINVAL, "NULL argument");
    const ssqa_anneal_params& pa = req->params;
    if (req->n_spins < 1 || req->n_spins > 16384 || !req->h || !req->J)
        return fail(SSQA_EINVAL, "bad problem (n_spins = %d)", req->n_spins);
    if (pa.cycles < 0 || pa.replicas < 1 || pa.trials < 1 || (pa.cycles > 0 && (!pa.jperp || !pa.i0)))
        return fail(SSQA_EINVAL, "bad anneal parameters");
    if (pa.cycles_per_launch != 0) return fail(SSQA_EINVAL, "cycles_per_launch must be 0 for served requests");
    if (pa.start_cycle != 0 || (pa.stop_cycle != 0 && pa.stop_cycle != pa.cycles))
        return fail(SSQA_EINVAL, "start_cycle and stop_cycle must be 0 for served requests");
    if (req->early_exit != 0 && req->early_exit != 1) return fail(SSQA_EINVAL, "early_exit must be 0 or 1");
    if (pa.replicas > 64) return fail(SSQA_ENOTSUP, "replicas = %d: served requests take at most 64", pa.replicas);
    if (pa.block_columns != 0 && pa.block_columns != 32 && pa.block_columns != 64 && pa.block_columns != 128)
        return fail(SSQA_EINVAL, "block_columns must be 0, 32, 64 or 128");
    if ((long long)pa.trials * pa.replicas > (1LL << 28)) return fail(SSQA_EINVAL, "trials * replicas too large");
    // A launch's work code keeps the block index in 16 bits.
    const int64_t blocks = request_blocks(req->n_spins, pa);
    if (blocks > 65535)
        return fail(SSQA_EINVAL, "request needs %lld workgroups of whole trials (> 65535): fewer trials per request",
                    (long long)blocks);
    // J is checked here, once (a J the problem upload would refuse is refused at submit), and kept as int8 when
    // it fits one plane: a quarter of the host memory to copy and of the bytes to upload at admission.
    const int n = req->n_spins;
    std::unique_ptr<int8_t[]> j8(new (std::nothrow) int8_t[(size_t)n * n]);
    const CouplingScan sc = scan_couplings(n, req->h, req->J, j8.get());
    const ssqa_status st = check_couplings(sc, n, req->J);
    if (st != SSQA_OK) return st;
    auto r = std::make_unique<Request>();
    r->id = s->next_id++;
    r->n = n;
    r->early_exit = req->early_exit;
    r->h.assign(req->h, req->h + n);
    if (sc.planes == 1 && j8) r->J8 = std::move(j8);
    else r->J.assign(req->J, req->J + (size_t)n * n);
    r->scan = sc;
    r->params = pa;
    r->jperp.assign(pa.jperp, pa.jperp + pa.cycles);
    r->i0.assign(pa.i0, pa.i0 + pa.cycles);
    r->planes = sc.planes;
    r->submit_s = now_s(s->t0);
    s->queue.push_back(r.get());
    *id = r->id;
    s->all[r->id] = std::move(r);
    return SSQA_OK;
}

ssqa_status ssqa_server_step(ssqa_server_t s, void* hip_stream, int32_t* active_out) {
    g_last_error.clear();
    if (!s) return fail(SSQA_EINVAL, "server is NULL");
    DeviceGuard guard(s->cfg.device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice(%d) failed", s->cfg.device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);

    // 1. admission, first come first served
    while (!s->queue.empty() && (int)s->active.size() < s->cfg.max_active) {
        Request* r = s->queue.front();
        if (r->state == SSQA_REQ_CANCELLED) {
            s->queue.pop_front();
            continue;
        }
        const int64_t need = request_bytes(r->n, r->planes, r->params, s->cfg.split_rows);
        if (need > s->cfg.memory_budget) {          // can never fit: refuse it
            s->queue.pop_front();
            r->state = SSQA_REQ_FAILED;
            r->status = SSQA_ENOMEM;
            r->done_s = now_s(s->t0);
            continue;
        }
        if (s->bytes_in_use + need > s->cfg.memory_budget) break;   // wait for memory to free up
        s->queue.pop_front();
        const ssqa_status st = admit(s, r);
        if (st != SSQA_OK) {
            release_device(r);
            r->state = SSQA_REQ_FAILED;
            r->status = st;
            r->done_s = now_s(s->t0);
            continue;
        }
        r->bytes = std::max(r->bytes, need);
        s->bytes_in_use += r->bytes;
        r->state = SSQA_REQ_RUNNING;
        r->admit_s = now_s(s->t0);
        s->active.push_back(r);
    }
    // drop cancelled requests
    for (size_t i = 0; i < s->active.size();) {
        Request* r = s->active[i];
        if (r->state == SSQA_REQ_CANCELLED) {
            release_device(r);
            s->bytes_in_use -= r->bytes;
            r->done_s = now_s(s->t0);
            s->active.erase(s->active.begin() + i);
        } else {
            ++i;
        }
    }
    if (active_out) *active_out = (int32_t)s->active.size();
    if (s->active.empty()) return SSQA_OK;

    // 2. one launch per kernel variant over the blocks of every active request, K cycles each
    const int K = s->cfg.cycles_per_step;
    const int n = (int)s->active.size();
    constexpr int kVariants = kSweepVariants;
    std::vector<WorkItem> lists[kVariants];
    int max_np[kVariants] = {}, max_delay[kVariants] = {};
    s->items.resize(n);
    double updates = 0;
    bool any_split = false;
    for (int i = 0; i < n; ++i) {
        Request* r = s->active[i];
        SweepArgs a = r->args;
        a.t_begin = r->cycle;
        a.t_end = std::min(r->params.cycles, r->cycle + K);
        a.final_pass = a.t_end == r->params.cycles ? 1 : 0;
        a.save_hist = a.final_pass ? 0 : 1;
        s->items[i] = a;
        updates += (double)r->n * r->params.replicas * r->params.trials * (a.t_end - a.t_begin);
        if (r->split) {
            any_split = true;
            continue;
        }
        const int v = sweep_variant(a.fast != 0, a.mode, a.nb, a.fp4 != 0);
        const double np = a.prob.np;
        const double cost = np * np * a.prob.planes * (a.t_end - a.t_begin + 1);
        for (int c = 0; c < r->n_wg; ++c) lists[v].push_back({cost, ((uint32_t)i << 16) | (uint32_t)c});
        max_np[v] = std::max(max_np[v], a.prob.np);
        max_delay[v] = std::max(max_delay[v], a.delay);
    }
    s->work.clear();
    size_t off[kVariants], len[kVariants];
    const int xcds = device_xcd_count(s->cfg.device);
    for (int v = 0; v < kVariants; ++v) {
        std::stable_sort(lists[v].begin(), lists[v].end(), [](const WorkItem& x, const WorkItem& y) { return x.cost > y.cost; });
        lists[v] = xcd_grouped(lists[v], xcds);
        off[v] = s->work.size();
        len[v] = lists[v].size();
        for (const WorkItem& e : lists[v]) s->work.push_back(e.code);
    }
    const size_t need = (sizeof(SweepArgs) * n + 255) / 256 * 256 + sizeof(uint32_t) * s->work.size();
    if (need > s->table_bytes) {
        if (s->table) {
            (void)hipStreamSynchronize(stream);
            (void)hipFree(s->table);
        }
        s->table = nullptr;
        s->table_bytes = 0;
        const size_t cap = need * 2;
        if (hipMalloc(&s->table, cap) != hipSuccess) return fail(SSQA_ENOMEM, "launch table allocation failed");
        s->table_bytes = cap;
    }
    auto* d_items = static_cast<SweepArgs*>(s->table);
    auto* d_work = reinterpret_cast<uint32_t*>(static_cast<char*>(s->table) + (sizeof(SweepArgs) * n + 255) / 256 * 256);
    SSQA_HIP(configure_sweep_kernels(), "configure");
    SSQA_HIP(hipMemcpyAsync(d_items, s->items.data(), sizeof(SweepArgs) * n, hipMemcpyHostToDevice, stream), "upload");
    if (!s->work.empty())
        SSQA_HIP(hipMemcpyAsync(d_work, s->work.data(), sizeof(uint32_t) * s->work.size(), hipMemcpyHostToDevice,
                                stream), "upload");
    // Row-split requests: their K cycles as one launch per cycle on the second stream, beside the persistent
    // launches below.  Launch t closes cycle t - 1 (except the step's first) and runs cycle t; a last launch
    // closes the step's last cycle, so that best energies and first hits are current at the readback.
    int used = 0;   // side streams this step
    if (any_split) {
        if (!s->fork) {
            SSQA_HIP(hipEventCreateWithFlags(&s->fork, hipEventDisableTiming), "event");
            for (int k = 0; k < ssqa_server::kSideStreams; ++k) {
                SSQA_HIP(hipStreamCreateWithFlags(&s->side[k], hipStreamNonBlocking), "side stream");
                SSQA_HIP(hipEventCreateWithFlags(&s->join[k], hipEventDisableTiming), "event");
            }
        }
        SSQA_HIP(hipEventRecord(s->fork, stream), "fork");
        int next = 0;
        for (int i = 0; i < n; ++i) {
            Request* r = s->active[i];
            if (!r->split) continue;
            const int k = next++ % ssqa_server::kSideStreams;
            hipStream_t side = s->side[k];
            if (k >= used) {
                SSQA_HIP(hipStreamWaitEvent(side, s->fork, 0), "fork");
                used = k + 1;
            }
            const SweepArgs& a = s->items[i];
            const int c0 = a.t_begin, c1 = a.t_end;
            const int32_t *jp = r->jperp.data(), *ip = r->i0.data();
            if (c0 == 0) SSQA_HIP(launch_sweep_split(r->d_args, a, 0, kSplitInit, jp, ip, side), "split init");
            for (int t = c0; t < c1; ++t)
                SSQA_HIP(launch_sweep_split(r->d_args, a, t, kSplitRun | kSplitUpdate | (t > c0 ? kSplitClose : 0),
                                            jp, ip, side), "split cycle");
            int last = c1 - 1;
            if (a.final_pass) {   // the energy of sigma(SC)
                SSQA_HIP(launch_sweep_split(r->d_args, a, c1, kSplitRun | (c1 > c0 ? kSplitClose : 0), jp, ip, side),
                         "split final");
                last = c1;
            }
            if (last >= c0) SSQA_HIP(launch_sweep_split(r->d_args, a, last + 1, kSplitClose, jp, ip, side), "split close");
        }
        for (int k = 0; k < used; ++k) SSQA_HIP(hipEventRecord(s->join[k], s->side[k]), "join");
    }
    for (int v = 0; v < kVariants; ++v) {
        if (!len[v]) continue;
        SSQA_HIP(launch_sweep_batch(d_items, d_work + off[v], (int)len[v], max_np[v], max_delay[v], v, stream), "step");
    }
    for (int k = 0; k < used; ++k) SSQA_HIP(hipStreamWaitEvent(stream, s->join[k], 0), "join");
    // 3. read back and retire at the requests' own cycle boundaries
    for (int i = 0; i < n; ++i) {
        Request* r = s->active[i];
        SSQA_HIP(hipMemcpyAsync(r->best.data(), s->items[i].best, sizeof(int64_t) * r->params.trials,
                                hipMemcpyDeviceToHost, stream), "readback");
        SSQA_HIP(hipMemcpyAsync(r->first_hit.data(), s->items[i].first_hit, sizeof(int32_t) * r->params.trials,
                                hipMemcpyDeviceToHost, stream), "readback");
    }
    SSQA_HIP(hipStreamSynchronize(stream), "step");
    s->cycles_run += K;
    s->spin_updates += updates;
    std::vector<Request*> still;
    for (int i = 0; i < n; ++i) {
        Request* r = s->active[i];
        r->cycle = s->items[i].t_end;
        bool done = r->cycle >= r->params.cycles;
        if (!done && r->early_exit && r->params.target_energy != SSQA_NO_TARGET) {
            for (int b = 0; b < r->params.trials && !done; ++b) done = r->best[b] == r->params.target_energy;
        }
        if (done) {
            release_device(r);
            s->bytes_in_use -= r->bytes;
            r->state = SSQA_REQ_DONE;
            r->done_s = now_s(s->t0);
        } else {
            still.push_back(r);
        }
    }
    s->active.swap(still);
    if (active_out) *active_out = (int32_t)s->active.size();
    return SSQA_OK;
}

ssqa_status ssqa_server_poll(ssqa_server_t s, int64_t id, ssqa_request_info* info, int64_t* best, int32_t* first_hit) {
    g_last_error.clear();
    if (!s || !info) return fail(SSQA_EINVAL, "NULL argument");
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(SSQA_EINVAL, "unknown request %lld", (long long)id);
    const Request* r = it->second.get();
    info->state = r->state;
    info->status = r->status;
    info->cycles_done = r->cycle;
    info->trials = r->params.trials;
    info->submit_s = r->submit_s;
    info->admit_s = r->admit_s;
    info->done_s = r->done_s;
    info->memory_bytes = r->bytes;
    if (r->state == SSQA_REQ_DONE || r->state == SSQA_REQ_RUNNING) {
        if (best && !r->best.empty()) std::memcpy(best, r->best.data(), sizeof(int64_t) * r->params.trials);
        if (first_hit && !r->first_hit.empty())
            std::memcpy(first_hit, r->first_hit.data(), sizeof(int32_t) * r->params.trials);
    }
    return SSQA_OK;
}

ssqa_status ssqa_server_cancel(ssqa_server_t s, int64_t id) {
    g_last_error.clear();
    if (!s) return fail(SSQA_EINVAL, "server is NULL");
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(SSQA_EINVAL, "unknown request %lld", (long long)id);
    Request* r = it->second.get();
    if (r->state == SSQA_REQ_QUEUED || r->state == SSQA_REQ_RUNNING) {
        if (r->state == SSQA_REQ_QUEUED) r->done_s = now_s(s->t0);
        r->state = SSQA_REQ_CANCELLED;
    }
    return SSQA_OK;
}

ssqa_status ssqa_server_stats(ssqa_server_t s, ssqa_server_stats_t* out) {
    g_last_error.clear();
    if (!s || !out) return fail(SSQA_EINVAL, "NULL argument");
    out->queued = (int32_t)s->queue.size();
    out->active = (int32_t)s->active.size();
    out->memory_in_use = s->bytes_in_use;
    out->spin_updates = s->spin_updates;
    out->elapsed_s = now_s(s->t0);
    return SSQA_OK;
}

void ssqa_server_destroy(ssqa_server_t s) {
    if (!s) return;
    DeviceGuard guard(s->cfg.device);
    for (hipStream_t side : s->side)
        if (side) (void)hipStreamSynchronize(side);
    for (auto& kv : s->all) release_device(kv.second.get());
    if (s->table) (void)hipFree(s->table);
    if (s->fork) (void)hipEventDestroy(s->fork);
    for (int k = 0; k < ssqa_server::kSideStreams; ++k) {
        if (s->join[k]) (void)hipEventDestroy(s->join[k]);
        if (s->side[k]) (void)hipStreamDestroy(s->side[k]);
    }
    delete s;
}

}  // extern "C"
