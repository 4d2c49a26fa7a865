// C ABI of the SSQA library: argument checking, device memory, launches (see include/ssqa.h).
#include "ssqa.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "philox.hpp"

using namespace ssqa;

struct ssqa_problem {
    int32_t device;
    DeviceProblem dev;
    int8_t* J_planes;
    int32_t* rowvec;   // [h | h - rowsum | 2h - rowsum], np each
};

namespace {

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

#define SSQA_HIP(call, what)                          \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Device scope guard: makes `device` current and restores the previous device on exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int device) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(device) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

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

int planes_needed(int32_t v) {
    int p = 0;
    do {
        const int8_t d = (int8_t)(v & 0xFF);
        v = (v - d) >> 8;
        ++p;
    } while (v != 0);
    return p;
}

}  // namespace

extern "C" {

const char* ssqa_status_string(ssqa_status s) {
    switch (s) {
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
    long long total = 0;
    int planes = 1;
    for (int i = 0; i < n; ++i) {
        total += 2LL * std::llabs((long long)h[i]);
        if (J[(size_t)i * n + i] != 0) return fail(SSQA_EINVAL, "J[%d][%d] = %d, diagonal must be zero", i, i,
                                                   J[(size_t)i * n + i]);
        for (int j = 0; j < n; ++j) {
            const int32_t v = J[(size_t)i * n + j];
            if (v != J[(size_t)j * n + i]) return fail(SSQA_EINVAL, "J not symmetric at (%d, %d)", i, j);
            total += std::llabs((long long)v);
            planes = std::max(planes, planes_needed(v));
        }
        if (total >= (1LL << 30)) return fail(SSQA_ERANGE, "2 sum|h| + sum|J| >= 2^30: int32 fields could overflow");
    }
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
    int32_t* J32 = nullptr;
    int32_t* h32 = nullptr;
    const size_t plane_bytes = (size_t)planes * np * np;
    hipError_t e = hipMalloc(&p->J_planes, plane_bytes);
    if (e == hipSuccess) e = hipMalloc(&p->rowvec, (size_t)np * 4 * 3);
    if (e == hipSuccess) e = hipMalloc(&J32, (size_t)n * n * 4);
    if (e == hipSuccess) e = hipMalloc(&h32, (size_t)n * 4);
    if (e == hipSuccess) e = hipMemcpy(J32, J, (size_t)n * n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h32, h, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_prepare_planes(J32, h32, n, np, planes, p->J_planes, p->rowvec, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (J32) (void)hipFree(J32);
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
    p->dev.h = p->rowvec;
    p->dev.hr = p->rowvec + np;
    p->dev.er = p->rowvec + 2 * np;
    *out = p;
    return SSQA_OK;
}

void ssqa_destroy_problem(ssqa_problem_t p) {
    if (!p) return;
    DeviceGuard guard(p->device);
    if (p->J_planes) (void)hipFree(p->J_planes);
    if (p->rowvec) (void)hipFree(p->rowvec);
    delete p;
}

int32_t ssqa_problem_spins(ssqa_problem_t p) { return p ? p->dev.n : 0; }
int32_t ssqa_problem_planes(ssqa_problem_t p) { return p ? p->dev.planes : 0; }
int32_t ssqa_problem_padded(ssqa_problem_t p) { return p ? p->dev.np : 0; }

ssqa_status ssqa_anneal(ssqa_problem_t prob, const ssqa_anneal_params* pa, const ssqa_anneal_outputs* out,
                        void* hip_stream) {
    g_last_error.clear();
    if (!prob || !pa || !out) return fail(SSQA_EINVAL, "NULL problem, params or outputs");
    const int R = pa->replicas, T = pa->trials, SC = pa->cycles;
    if (R < 1 || T < 1 || SC < 0) return fail(SSQA_EINVAL, "replicas, trials must be >= 1 and cycles >= 0");
    if (R > sweep_columns_per_wg())
        return fail(SSQA_ENOTSUP, "replicas = %d exceeds %d", R, sweep_columns_per_wg());
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

    if (sweep_lds_bytes(prob->dev.np, pa->delay) > 160 * 1024)
        return fail(SSQA_ENOTSUP, "N = %d with delay %d needs %zu bytes of LDS per workgroup (> 160 KiB)",
                    prob->dev.n, pa->delay, sweep_lds_bytes(prob->dev.np, pa->delay));

    DeviceGuard guard(prob->device);
    if (!guard.ok) return fail(SSQA_EDEVICE, "hipSetDevice failed");
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    retain_pool_memory(prob->device);
    const int nb = sweep_columns_per_wg();
    const int tpw = nb / R;
    const int n_wg = (T + tpw - 1) / tpw;
    const int np = prob->dev.np;
    const size_t is_bytes = (size_t)n_wg * nb * np;
    const size_t hist_bytes = (size_t)n_wg * std::max(pa->delay, 1) * nb * (np / 32) * 4;
    const size_t sched_bytes = (size_t)std::max(SC, 1) * 4;

    int8_t* is_state = nullptr;
    uint32_t* hist = nullptr;
    int32_t* d_jperp = nullptr;
    int32_t* d_i0 = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&is_state), is_bytes, stream);
    if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&hist), hist_bytes, stream);
    if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&d_jperp), sched_bytes, stream);
    if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&d_i0), sched_bytes, stream);
    if (e == hipSuccess && SC > 0) e = hipMemcpyAsync(d_jperp, pa->jperp, (size_t)SC * 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && SC > 0) e = hipMemcpyAsync(d_i0, pa->i0, (size_t)SC * 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // host schedules may be freed on return

    if (e == hipSuccess) {
        SweepArgs a{};
        a.prob = prob->dev;
        a.R = R;
        a.T = T;
        a.tpw = tpw;
        a.cols_wg = tpw * R;
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
        const int chunk = pa->cycles_per_launch > 0 ? pa->cycles_per_launch : std::max(SC, 1);
        int t = 0;
        do {
            a.t_begin = t;
            a.t_end = std::min(SC, t + chunk);
            a.final_pass = (a.t_end == SC) ? 1 : 0;
            e = launch_sweep(a, n_wg, stream);
            t = a.t_end;
        } while (e == hipSuccess && t < SC);
        if (e == hipSuccess && out->final_is)
            e = launch_copy_final_is(is_state, np, prob->dev.n, R, T, tpw, out->final_is, stream);
    }
    if (is_state) (void)hipFreeAsync(is_state, stream);
    if (hist) (void)hipFreeAsync(hist, stream);
    if (d_jperp) (void)hipFreeAsync(d_jperp, stream);
    if (d_i0) (void)hipFreeAsync(d_i0, stream);
    if (e != hipSuccess) {
        return e == hipErrorOutOfMemory ? fail(SSQA_ENOMEM, "device allocation failed") : hip_fail(e, "anneal");
    }
    return SSQA_OK;
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

void ssqa_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const Philox4 r = philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    for (int w = 0; w < 4; ++w) out[w] = r.v[w];
}

}  // extern "C"
