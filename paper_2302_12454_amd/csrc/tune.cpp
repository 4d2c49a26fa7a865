// Autotuner of the sweep's tiling (see include/ssqa.h, "Autotuner").
//
// The field product's tiling (columns and trials per workgroup, fp4 or int8 operands, and for the batched form
// the padded size from which anneals take 128-column blocks) changes only the speed of an anneal, never its
// results.  The tuner times every legal candidate on the device on a prefix of the anneal's own cycles and
// records the fastest in a process-wide cache keyed by the device, the kernel build and the anneal's shape;
// automatic requests (block_columns = 0, operand_format = 0) then take the recorded tile.  The cache can be
// written to and read from a JSON file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "internal.hpp"

#ifndef SSQA_KERNEL_HASH
#define SSQA_KERNEL_HASH "unversioned"
#endif

using namespace ssqa;
using namespace ssqa::detail;

namespace {

constexpr const char* kFormat = "ssqa-tune-1";

struct Entry {
    std::string device, kernel, form;   // form: "plain" or "batch"
    // plain shape
    int np = 0, planes = 0, R = 0, T = 0, delay = 0, mode = 0, fast = 0, fp4_ok = 0;
    // plain tile
    int nb = 0, tpw = 0, fp4 = 0;
    // batch shape and floor
    uint64_t signature = 0;
    int instances = 0, wide_rows = 0;
    double ms_per_cycle = 0;

    bool same_key(const Entry& o) const {
        if (device != o.device || kernel != o.kernel || form != o.form) return false;
        if (form == "batch") return signature == o.signature;
        return np == o.np && planes == o.planes && R == o.R && T == o.T && delay == o.delay && mode == o.mode &&
               fast == o.fast && fp4_ok == o.fp4_ok;
    }
};

std::mutex g_mutex;
std::vector<Entry> g_entries;

void put(const Entry& e) {
    for (Entry& x : g_entries)
        if (x.same_key(e)) {
            x = e;
            return;
        }
    g_entries.push_back(e);
}

// "name|gcn arch|compute units" of a device, looked up once.
std::string device_identity(int device) {
    static std::mutex m;
    static std::string ids[64];
    if (device < 0 || device >= 64) return "invalid";
    std::lock_guard<std::mutex> lock(m);
    if (ids[device].empty()) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
        ids[device] = std::string(prop.name) + "|" + prop.gcnArchName + "|" + std::to_string(prop.multiProcessorCount);
    }
    return ids[device];
}

Entry plain_key(const ssqa_problem* prob, const ssqa_anneal_params* pa) {
    Entry e;
    e.device = device_identity(prob->device);
    e.kernel = SSQA_KERNEL_HASH;
    e.form = "plain";
    e.np = prob->dev.np;
    e.planes = prob->dev.planes;
    e.R = pa->replicas;
    e.T = pa->trials;
    e.delay = pa->delay;
    e.mode = pa->coupling_mode;
    e.fast = fast_epilogue(pa) ? 1 : 0;
    e.fp4_ok = use_fp4(prob, pa) ? 1 : 0;
    return e;
}

// ---------------------------------------------------------------------------------------------
// A small JSON reader for the cache file (objects, arrays, strings, numbers, true / false / null).
// ---------------------------------------------------------------------------------------------
struct Json {
    enum Kind { kNull, kBool, kNum, kStr, kArr, kObj } kind = kNull;
    double num = 0;
    bool b = false;
    std::string str;
    std::vector<Json> arr;
    std::vector<std::pair<std::string, Json>> obj;

    const Json* get(const char* key) const {
        for (const auto& kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct Parser {
    const char* p;
    const char* end;
    std::string err;
    int depth = 0;

    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool fail_at(const char* what) {
        if (err.empty()) err = what;
        return false;
    }
    bool literal(const char* word) {
        const size_t n = std::strlen(word);
        if ((size_t)(end - p) < n || std::strncmp(p, word, n) != 0) return fail_at("unexpected token");
        p += n;
        return true;
    }
    bool string(std::string& out) {
        if (p >= end || *p != '"') return fail_at("expected a string");
        ++p;
        out.clear();
        while (p < end && *p != '"') {
            char c = *p++;
            if (c == '\\') {
                if (p >= end) return fail_at("unterminated escape");
                const char x = *p++;
                if (x == '"' || x == '\\' || x == '/') c = x;
                else if (x == 'n') c = '\n';
                else if (x == 't') c = '\t';
                else return fail_at("unsupported escape");
            } else if ((unsigned char)c < 0x20) {
                return fail_at("control character in string");
            }
            out.push_back(c);
        }
        if (p >= end) return fail_at("unterminated string");
        ++p;
        return true;
    }
    bool number(double& out) {
        const char* q = p;
        if (q < end && (*q == '-' || *q == '+')) ++q;
        while (q < end && ((*q >= '0' && *q <= '9') || *q == '.' || *q == 'e' || *q == 'E' || *q == '-' || *q == '+'))
            ++q;
        if (q == p) return fail_at("expected a value");
        const std::string text(p, q);
        char* stop = nullptr;
        errno = 0;
        out = std::strtod(text.c_str(), &stop);
        if (stop != text.c_str() + text.size() || errno != 0) return fail_at("bad number");
        p = q;
        return true;
    }
    bool value(Json& v) {
        if (++depth > 32) return fail_at("nesting too deep");
        ws();
        bool ok = true;
        if (p >= end) {
            ok = fail_at("unexpected end of file");
        } else if (*p == '{') {
            v.kind = Json::kObj;
            ++p;
            ws();
            if (p < end && *p == '}') {
                ++p;
            } else {
                for (;;) {
                    ws();
                    std::string key;
                    if (!string(key)) { ok = false; break; }
                    ws();
                    if (p >= end || *p != ':') { ok = fail_at("expected ':'"); break; }
                    ++p;
                    Json item;
                    if (!value(item)) { ok = false; break; }
                    v.obj.emplace_back(std::move(key), std::move(item));
                    ws();
                    if (p < end && *p == ',') { ++p; continue; }
                    if (p < end && *p == '}') { ++p; break; }
                    ok = fail_at("expected ',' or '}'");
                    break;
                }
            }
        } else if (*p == '[') {
            v.kind = Json::kArr;
            ++p;
            ws();
            if (p < end && *p == ']') {
                ++p;
            } else {
                for (;;) {
                    Json item;
                    if (!value(item)) { ok = false; break; }
                    v.arr.push_back(std::move(item));
                    ws();
                    if (p < end && *p == ',') { ++p; continue; }
                    if (p < end && *p == ']') { ++p; break; }
                    ok = fail_at("expected ',' or ']'");
                    break;
                }
            }
        } else if (*p == '"') {
            v.kind = Json::kStr;
            ok = string(v.str);
        } else if (*p == 't') {
            v.kind = Json::kBool;
            v.b = true;
            ok = literal("true");
        } else if (*p == 'f') {
            v.kind = Json::kBool;
            ok = literal("false");
        } else if (*p == 'n') {
            ok = literal("null");
        } else {
            v.kind = Json::kNum;
            ok = number(v.num);
        }
        --depth;
        return ok;
    }
};

bool get_int(const Json& o, const char* key, int lo, int hi, int* out, std::string& err) {
    const Json* v = o.get(key);
    if (!v || v->kind != Json::kNum || v->num != (double)(long long)v->num || v->num < lo || v->num > hi) {
        err = std::string("entry field '") + key + "' missing or not an integer in range";
        return false;
    }
    *out = (int)v->num;
    return true;
}

bool get_str(const Json& o, const char* key, std::string* out, std::string& err) {
    const Json* v = o.get(key);
    if (!v || v->kind != Json::kStr) {
        err = std::string("entry field '") + key + "' missing or not a string";
        return false;
    }
    *out = v->str;
    return true;
}

bool entry_from_json(const Json& o, Entry* e, std::string& err) {
    if (o.kind != Json::kObj) {
        err = "entry is not an object";
        return false;
    }
    if (!get_str(o, "form", &e->form, err) || !get_str(o, "device", &e->device, err) ||
        !get_str(o, "kernel", &e->kernel, err))
        return false;
    const Json* ms = o.get("ms_per_cycle");
    if (!ms || ms->kind != Json::kNum || !(ms->num >= 0)) {
        err = "entry field 'ms_per_cycle' missing or negative";
        return false;
    }
    e->ms_per_cycle = ms->num;
    if (e->form == "plain") {
        int fmt = 0;
        if (!get_int(o, "np", kTileRows, 1 << 20, &e->np, err) || !get_int(o, "planes", 1, 4, &e->planes, err) ||
            !get_int(o, "replicas", 1, 128, &e->R, err) || !get_int(o, "trials", 1, 1 << 28, &e->T, err) ||
            !get_int(o, "delay", 0, kMaxDelay, &e->delay, err) || !get_int(o, "mode", 0, 1, &e->mode, err) ||
            !get_int(o, "fast", 0, 1, &e->fast, err) || !get_int(o, "fp4_ok", 0, 1, &e->fp4_ok, err) ||
            !get_int(o, "block_columns", 32, 128, &e->nb, err) || !get_int(o, "trials_per_block", 1, 128, &e->tpw, err) ||
            !get_int(o, "operand_format", 1, 2, &fmt, err))
            return false;
        if (e->np % kTileRows != 0 || (e->nb != 32 && e->nb != 64 && e->nb != 128)) {
            err = "entry has a padded size or block width the library does not use";
            return false;
        }
        e->fp4 = fmt == 2 ? 1 : 0;
        return true;
    }
    if (e->form == "batch") {
        std::string sig;
        if (!get_str(o, "signature", &sig, err) || !get_int(o, "instances", 1, 65535, &e->instances, err) ||
            !get_int(o, "wide_rows", 0, 1 << 20, &e->wide_rows, err))
            return false;
        char* stop = nullptr;
        e->signature = std::strtoull(sig.c_str(), &stop, 16);
        if (sig.size() != 16 || !stop || *stop != '\0') {
            err = "entry field 'signature' is not 16 hexadecimal digits";
            return false;
        }
        return true;
    }
    err = "entry form must be \"plain\" or \"batch\"";
    return false;
}

std::string json_escape(const std::string& s) {
    std::string r;
    for (const char c : s) {
        if (c == '"' || c == '\\') r.push_back('\\');
        if ((unsigned char)c < 0x20) continue;
        r.push_back(c);
    }
    return r;
}

std::string entry_to_json(const Entry& e) {
    char buf[640];
    std::string head = "{\"form\": \"" + json_escape(e.form) + "\", \"device\": \"" + json_escape(e.device) +
                       "\", \"kernel\": \"" + json_escape(e.kernel) + "\", ";
    if (e.form == "plain") {
        std::snprintf(buf, sizeof buf,
                      "\"np\": %d, \"planes\": %d, \"replicas\": %d, \"trials\": %d, \"delay\": %d, \"mode\": %d, "
                      "\"fast\": %d, \"fp4_ok\": %d, \"block_columns\": %d, \"trials_per_block\": %d, "
                      "\"operand_format\": %d, \"ms_per_cycle\": %.9g}",
                      e.np, e.planes, e.R, e.T, e.delay, e.mode, e.fast, e.fp4_ok, e.nb, e.tpw, e.fp4 ? 2 : 1,
                      e.ms_per_cycle);
    } else {
        std::snprintf(buf, sizeof buf,
                      "\"signature\": \"%016llx\", \"instances\": %d, \"wide_rows\": %d, \"ms_per_cycle\": %.9g}",
                      (unsigned long long)e.signature, e.instances, e.wide_rows, e.ms_per_cycle);
    }
    return head + buf;
}

// Device memory freed on scope exit.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

namespace ssqa {
namespace detail {

bool tuned_plain(const ssqa_problem* prob, const ssqa_anneal_params* pa, TunedTile* out) {
    const Entry key = plain_key(prob, pa);
    std::lock_guard<std::mutex> lock(g_mutex);
    for (const Entry& e : g_entries)
        if (e.same_key(key)) {
            if (!tile_legal(prob, pa, e.nb, e.tpw, e.fp4 != 0)) return false;
            *out = TunedTile{e.nb, e.tpw, e.fp4, e.ms_per_cycle};
            return true;
        }
    return false;
}

uint64_t batch_signature(int count, const ssqa_problem_t* problems, const ssqa_anneal_params* params) {
    uint64_t h = 1469598103934665603ull;   // FNV-1a
    auto mix = [&h](int64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (uint64_t)((v >> (8 * k)) & 0xFF);
            h *= 1099511628211ull;
        }
    };
    mix(count);
    for (int i = 0; i < count; ++i) {
        const ssqa_problem* p = problems[i];
        const ssqa_anneal_params& pa = params[i];
        mix(p->dev.np);
        mix(p->dev.planes);
        mix(pa.replicas);
        mix(pa.trials);
        mix(pa.delay);
        mix(pa.coupling_mode);
        mix(pa.block_columns);
        mix(fast_epilogue(&pa) ? 1 : 0);
        mix(use_fp4(p, &pa) ? 1 : 0);
    }
    return h;
}

int tuned_batch_rows(int device, uint64_t signature) {
    Entry key;
    key.device = device_identity(device);
    key.kernel = SSQA_KERNEL_HASH;
    key.form = "batch";
    key.signature = signature;
    std::lock_guard<std::mutex> lock(g_mutex);
    for (const Entry& e : g_entries)
        if (e.same_key(key)) return e.wide_rows;
    return -1;
}

}  // namespace detail
}  // namespace ssqa

extern "C" {

ssqa_status ssqa_tune_anneal(ssqa_problem_t prob, const ssqa_anneal_params* pa, int32_t probe_cycles, void* hip_stream,
                             ssqa_tile* candidates, int32_t capacity, int32_t* count, ssqa_tile* chosen) {
    g_last_error.clear();
    if (!prob || !pa || !chosen) return fail(SSQA_EINVAL, "NULL problem, params or chosen");
    if (capacity < 0 || (capacity > 0 && !candidates)) return fail(SSQA_EINVAL, "candidates is NULL");
    if (probe_cycles < 1) return fail(SSQA_EINVAL, "probe_cycles must be >= 1");
    if (pa->block_columns != 0 || pa->operand_format != 0)
        return fail(SSQA_EINVAL, "the tuner chooses block_columns and operand_format: pass 0 for both");
    if (pa->start_cycle != 0 || (pa->stop_cycle != 0 && pa->stop_cycle != pa->cycles) || pa->cycles_per_launch != 0)
        return fail(SSQA_EINVAL, "start_cycle, stop_cycle and cycles_per_launch must be 0 for tuning");
    int64_t dummy_best = 0;
    int32_t dummy_hit = 0;
    ssqa_anneal_outputs probe_out{};
    probe_out.best_energy = &dummy_best;   // host addresses: check_params only tests them for NULL
    probe_out.first_hit = &dummy_hit;
    ssqa_status st = check_params(prob, pa, &probe_out);
    if (st != SSQA_OK) return st;

    const int R = pa->replicas, T = pa->trials, np = prob->dev.np;
    const int cus = device_cu_count(prob->device);
    const bool fp4_ok = use_fp4(prob, pa);
    const bool fast = fast_epilogue(pa);
    struct Cand {
        int nb, tpw;
        bool fp4;
        double ms;
    };
    std::vector<Cand> cands;
    for (const bool fp4 : {true, false}) {
        if (fp4 && !fp4_ok) continue;
        for (const int nb : {32, 64, 128}) {
            if (R > nb || !tile_legal(prob, pa, nb, nb / R, fp4)) continue;
            const int full = nb / R;
            std::set<int> tpws = {full};
            for (const int m : {1, 2, 4}) {
                const int t = (T + m * cus - 1) / (m * cus);
                if (t >= 1 && t < full) tpws.insert(t);
            }
            for (const int t : tpws) cands.push_back({nb, t, fp4, 0.0});
        }
    }
    if (cands.empty()) return fail(SSQA_ENOTSUP, "no tile can run this anneal");

    // The probe: the first probe_cycles cycles of the anneal (the same kernel variant as the whole anneal).
    ssqa_anneal_params p2 = *pa;
    p2.cycles = std::min(pa->cycles, probe_cycles);
    const int SC = p2.cycles;
    size_t is_bytes = 0, hist_bytes = 0;
    for (const Cand& c : cands) {
        const size_t n_wg = (size_t)(T + c.tpw - 1) / c.tpw;
        is_bytes = std::max(is_bytes, n_wg * c.nb * np);
        hist_bytes = std::max(hist_bytes, n_wg * std::max(pa->delay, 1) * c.nb * (np / 32) * 4);
    }
    DeviceGuard guard(prob->device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice failed");
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    DevBuf is_buf, hist_buf, sched_buf, best_buf, hit_buf;
    hipError_t e = hipMalloc(&is_buf.p, is_bytes);
    if (e == hipSuccess) e = hipMalloc(&hist_buf.p, hist_bytes);
    if (e == hipSuccess) e = hipMalloc(&sched_buf.p, 2 * (size_t)std::max(SC, 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&best_buf.p, (size_t)T * 8);
    if (e == hipSuccess) e = hipMalloc(&hit_buf.p, (size_t)T * 4);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(SSQA_ENOMEM, "device allocation failed") : hip_fail(e, "tune");
    int32_t* d_sched = static_cast<int32_t*>(sched_buf.p);
    if (SC > 0) {
        e = hipMemcpy(d_sched, pa->jperp, (size_t)SC * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_sched + SC, pa->i0, (size_t)SC * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "tune: schedule copy");
    }
    ssqa_anneal_outputs outs{};
    outs.best_energy = static_cast<int64_t*>(best_buf.p);
    outs.first_hit = static_cast<int32_t*>(hit_buf.p);
    EventPair ev;
    e = hipEventCreate(&ev.a);
    if (e == hipSuccess) e = hipEventCreate(&ev.b);
    if (e != hipSuccess) return hip_fail(e, "tune: events");

    for (Cand& c : cands) {
        SweepArgs a = make_args(prob, &p2, &outs, d_sched, d_sched + std::max(SC, 1), static_cast<int8_t*>(is_buf.p),
                                static_cast<uint32_t*>(hist_buf.p), c.nb, c.tpw, c.fp4 ? 1 : 0);
        a.fast = fast ? 1 : 0;   // the whole schedule's epilogue variant (the prefix admits it too)
        a.t_begin = 0;
        a.t_end = SC;
        a.final_pass = 1;
        a.save_hist = 0;
        const int n_wg = (T + c.tpw - 1) / c.tpw;
        double best_ms = 1e30;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {   // one warm-up, then the best of two
            e = hipEventRecord(ev.a, stream);
            if (e == hipSuccess) e = launch_sweep(a, n_wg, stream);
            if (e == hipSuccess) e = hipEventRecord(ev.b, stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev.b);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
            if (e == hipSuccess && rep > 0) best_ms = std::min(best_ms, (double)ms);
        }
        if (e != hipSuccess) return hip_fail(e, "tune: probe launch");
        c.ms = best_ms / std::max(SC, 1);
    }
    const auto best = std::min_element(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
    Entry rec = plain_key(prob, pa);
    rec.nb = best->nb;
    rec.tpw = best->tpw;
    rec.fp4 = best->fp4 ? 1 : 0;
    rec.ms_per_cycle = best->ms;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        put(rec);
    }
    auto tile = [T](const Cand& c) {
        return ssqa_tile{c.nb, c.tpw, c.fp4 ? 2 : 1, (T + c.tpw - 1) / c.tpw, c.ms};
    };
    for (int i = 0; i < (int)cands.size() && i < capacity; ++i) candidates[i] = tile(cands[i]);
    if (count) *count = (int32_t)cands.size();
    *chosen = tile(*best);
    return SSQA_OK;
}

ssqa_status ssqa_tune_batch(int32_t count, const ssqa_problem_t* problems, const ssqa_anneal_params* params,
                            int32_t probe_cycles, void* hip_stream, int32_t* wide_rows, double* ms_per_cycle) {
    g_last_error.clear();
    if (count < 1 || count > 65535) return fail(SSQA_EINVAL, "count = %d outside [1, 65535]", count);
    if (!problems || !params || !wide_rows) return fail(SSQA_EINVAL, "NULL problems, params or wide_rows");
    if (probe_cycles < 1) return fail(SSQA_EINVAL, "probe_cycles must be >= 1");
    for (int i = 0; i < count; ++i)
        if (!problems[i]) return fail(SSQA_EINVAL, "problems[%d] is NULL", i);
    const int device = problems[0]->device;
    // Candidate floors: every distinct padded size of an anneal that could take 128 columns, and "never".
    std::set<int> floors = {0};
    int max_t = 1;
    int64_t dummy_best = 0;
    int32_t dummy_hit = 0;
    for (int i = 0; i < count; ++i) {
        ssqa_anneal_outputs probe_out{};
        probe_out.best_energy = &dummy_best;
        probe_out.first_hit = &dummy_hit;
        const ssqa_status st = check_params(problems[i], &params[i], &probe_out);
        if (st != SSQA_OK) {
            const std::string msg = g_last_error;
            return fail(st, "anneal %d: %s", i, msg.c_str());
        }
        if (batch_wide(problems[i], &params[i], 1)) floors.insert(problems[i]->dev.np);
        max_t = std::max(max_t, params[i].trials);
    }
    std::vector<ssqa_anneal_params> p2(params, params + count);
    int64_t probe_len = 0;   // cycles of the longest probe anneal
    for (auto& p : p2) {
        p.cycles = std::min(p.cycles, probe_cycles);
        probe_len = std::max<int64_t>(probe_len, p.cycles);
    }
    DeviceGuard guard(device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice failed");
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    DevBuf best_buf, hit_buf;
    hipError_t e = hipMalloc(&best_buf.p, (size_t)count * max_t * 8);
    if (e == hipSuccess) e = hipMalloc(&hit_buf.p, (size_t)count * max_t * 4);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(SSQA_ENOMEM, "device allocation failed") : hip_fail(e, "tune");
    std::vector<ssqa_anneal_outputs> outs(count);
    for (int i = 0; i < count; ++i) {
        outs[i] = ssqa_anneal_outputs{};
        outs[i].best_energy = static_cast<int64_t*>(best_buf.p) + (size_t)i * max_t;
        outs[i].first_hit = static_cast<int32_t*>(hit_buf.p) + (size_t)i * max_t;
    }
    EventPair ev;
    e = hipEventCreate(&ev.a);
    if (e == hipSuccess) e = hipEventCreate(&ev.b);
    if (e != hipSuccess) return hip_fail(e, "tune: events");
    int best_floor = kBatchWideRows;
    double best_ms = 1e30;
    for (const int fl : floors) {
        ssqa_batch_t b = nullptr;
        const ssqa_status st = batch_create_impl(count, problems, p2.data(), outs.data(), &b, fl);
        if (st != SSQA_OK) return st;
        double ms_min = 1e30;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(ev.a, stream);
            if (e == hipSuccess) e = ssqa_batch_run(b, stream) == SSQA_OK ? hipSuccess : hipErrorLaunchFailure;
            if (e == hipSuccess) e = hipEventRecord(ev.b, stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev.b);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
            if (e == hipSuccess && rep > 0) ms_min = std::min(ms_min, (double)ms);
        }
        ssqa_batch_destroy(b);
        if (e != hipSuccess) return hip_fail(e, "tune: batch probe");
        if (ms_min < best_ms) {
            best_ms = ms_min;
            best_floor = fl;
        }
    }
    Entry rec;
    rec.device = device_identity(device);
    rec.kernel = SSQA_KERNEL_HASH;
    rec.form = "batch";
    rec.signature = batch_signature(count, problems, params);
    rec.instances = count;
    rec.wide_rows = best_floor;
    rec.ms_per_cycle = best_ms / std::max<int64_t>(probe_len, 1);
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        put(rec);
    }
    *wide_rows = best_floor;
    if (ms_per_cycle) *ms_per_cycle = rec.ms_per_cycle;
    return SSQA_OK;
}

ssqa_status ssqa_tune_lookup(ssqa_problem_t prob, const ssqa_anneal_params* pa, ssqa_tile* tile, int32_t* tuned) {
    g_last_error.clear();
    if (!prob || !pa || !tile) return fail(SSQA_EINVAL, "NULL problem, params or tile");
    int64_t dummy_best = 0;
    int32_t dummy_hit = 0;
    ssqa_anneal_outputs probe_out{};
    probe_out.best_energy = &dummy_best;
    probe_out.first_hit = &dummy_hit;
    const ssqa_status st = check_params(prob, pa, &probe_out);
    if (st != SSQA_OK) return st;
    const PlainLayout lay = plain_layout(prob, pa);
    TunedTile t{};
    const bool hit = lay.tuned && tuned_plain(prob, pa, &t);
    *tile = ssqa_tile{lay.nb, lay.tpw, lay.fp4 ? 2 : 1, lay.n_wg, hit ? t.ms_per_cycle : 0.0};
    if (tuned) *tuned = lay.tuned ? 1 : 0;
    return SSQA_OK;
}

ssqa_status ssqa_tune_set(ssqa_problem_t prob, const ssqa_anneal_params* pa, const ssqa_tile* tile) {
    g_last_error.clear();
    if (!prob || !pa || !tile) return fail(SSQA_EINVAL, "NULL problem, params or tile");
    if (pa->block_columns != 0 || pa->operand_format != 0)
        return fail(SSQA_EINVAL, "tiles are recorded for automatic requests: pass block_columns = operand_format = 0");
    int64_t dummy_best = 0;
    int32_t dummy_hit = 0;
    ssqa_anneal_outputs probe_out{};
    probe_out.best_energy = &dummy_best;
    probe_out.first_hit = &dummy_hit;
    const ssqa_status st = check_params(prob, pa, &probe_out);
    if (st != SSQA_OK) return st;
    if (tile->operand_format != 1 && tile->operand_format != 2) return fail(SSQA_EINVAL, "operand_format must be 1 or 2");
    if (!tile_legal(prob, pa, tile->block_columns, tile->trials_per_block, tile->operand_format == 2))
        return fail(SSQA_ENOTSUP, "tile %d columns x %d trials (%s) cannot run this anneal", tile->block_columns,
                    tile->trials_per_block, tile->operand_format == 2 ? "fp4" : "int8");
    Entry rec = plain_key(prob, pa);
    rec.nb = tile->block_columns;
    rec.tpw = tile->trials_per_block;
    rec.fp4 = tile->operand_format == 2 ? 1 : 0;
    rec.ms_per_cycle = tile->ms_per_cycle >= 0 ? tile->ms_per_cycle : 0;
    std::lock_guard<std::mutex> lock(g_mutex);
    put(rec);
    return SSQA_OK;
}

ssqa_status ssqa_tune_save(const char* path) {
    g_last_error.clear();
    if (!path) return fail(SSQA_EINVAL, "path is NULL");
    std::string text = std::string("{\"format\": \"") + kFormat + "\", \"entries\": [";
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        for (size_t i = 0; i < g_entries.size(); ++i) text += (i ? ",\n  " : "\n  ") + entry_to_json(g_entries[i]);
    }
    text += "\n]}\n";
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(SSQA_EINVAL, "cannot open %s for writing", path);
    const size_t w = std::fwrite(text.data(), 1, text.size(), f);
    const int c = std::fclose(f);
    if (w != text.size() || c != 0) return fail(SSQA_EINVAL, "write to %s failed", path);
    return SSQA_OK;
}

ssqa_status ssqa_tune_load(const char* path, int32_t* loaded) {
    g_last_error.clear();
    if (!path) return fail(SSQA_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SSQA_EINVAL, "cannot open %s", path);
    std::string text;
    char buf[65536];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) {
        text.append(buf, n);
        if (text.size() > (64u << 20)) {
            std::fclose(f);
            return fail(SSQA_EINVAL, "%s is larger than 64 MiB", path);
        }
    }
    std::fclose(f);
    Parser ps{text.data(), text.data() + text.size(), {}, 0};
    Json root;
    if (!ps.value(root)) return fail(SSQA_EINVAL, "%s: %s at byte %zu", path, ps.err.c_str(), (size_t)(ps.p - text.data()));
    ps.ws();
    if (ps.p != ps.end) return fail(SSQA_EINVAL, "%s: trailing data at byte %zu", path, (size_t)(ps.p - text.data()));
    const Json* fmt = root.get("format");
    const Json* entries = root.get("entries");
    if (root.kind != Json::kObj || !fmt || fmt->kind != Json::kStr || fmt->str != kFormat)
        return fail(SSQA_EINVAL, "%s: not a tuning cache of format %s", path, kFormat);
    if (!entries || entries->kind != Json::kArr) return fail(SSQA_EINVAL, "%s: 'entries' is not an array", path);
    std::vector<Entry> parsed;
    for (size_t i = 0; i < entries->arr.size(); ++i) {
        Entry e;
        std::string err;
        if (!entry_from_json(entries->arr[i], &e, err)) return fail(SSQA_EINVAL, "%s: entry %zu: %s", path, i, err.c_str());
        parsed.push_back(e);
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    for (const Entry& e : parsed) put(e);
    if (loaded) *loaded = (int32_t)parsed.size();
    return SSQA_OK;
}

int32_t ssqa_tune_entries(void) {
    std::lock_guard<std::mutex> lock(g_mutex);
    return (int32_t)g_entries.size();
}

void ssqa_tune_clear(void) {
    std::lock_guard<std::mutex> lock(g_mutex);
    g_entries.clear();
}

}  // extern "C"
