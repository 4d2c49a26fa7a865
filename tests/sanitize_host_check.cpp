// Host paths of the library under AddressSanitizer and UndefinedBehaviorSanitizer: every call here runs on
// the CPU (schedules, the graph-isomorphism mapping, the Philox block function, the XCD-aware work order and
// the argument checks of the C ABI that happen before any device work).  Output buffers are heap arrays of
// exactly the documented size, so that any write past them is reported.  Prints "ok" and exits 0 when every
// expected status was returned; a sanitizer finding aborts the program.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <random>
#include <vector>

#include "ssqa.h"
#include "work_order.hpp"

static int g_bad = 0;

#define EXPECT(cond)                                                  \
    do {                                                              \
        if (!(cond)) {                                                \
            std::printf("failed at line %d: %s\n", __LINE__, #cond);  \
            ++g_bad;                                                  \
        }                                                             \
    } while (0)

static void schedules() {
    for (int cycles : {0, 1, 7, 100, 2001})
        for (int tau : {1, 3, 100})
            for (int beta : {1, 3, 5}) {
                std::vector<int32_t> out(cycles > 0 ? cycles : 0);
                EXPECT(ssqa_jperp_schedule(cycles, tau, beta, 0, 1, 2, 12 * beta, cycles ? out.data() : nullptr) ==
                       SSQA_OK);
                for (int growth : {2, 3})
                    EXPECT(ssqa_ssa_i0_schedule(cycles, tau, growth, 1, 16, 12, cycles ? out.data() : nullptr) ==
                           SSQA_OK);
            }
    std::vector<int32_t> small(5);
    EXPECT(ssqa_jperp_schedule(5, 1, 3, 0, 1, 2, 1, small.data()) == SSQA_EINVAL);   // 1/6 not an integer at S = 1
    EXPECT(ssqa_jperp_schedule(5, 0, 3, 0, 1, 2, 12, small.data()) == SSQA_EINVAL);
    EXPECT(ssqa_jperp_schedule(5, 1, 3, 0, 1, 2, 12, nullptr) == SSQA_EINVAL);
    EXPECT(ssqa_ssa_i0_schedule(5, 1, 2, 1, 16, 12, nullptr) == SSQA_EINVAL);
    for (int cycles : {1, 2, 40000}) {
        std::vector<double> beta(cycles);
        EXPECT(ssqa_sa_schedule(cycles, 1000.0, 0.1, 12, beta.data()) == SSQA_OK);
    }
    EXPECT(ssqa_sa_schedule(0, 1000.0, 0.1, 12, nullptr) == SSQA_EINVAL);
    double acc = 0;
    for (int64_t de : {0, 1, 12, 600, 100000})
        for (double b : {0.0, 1e-4, 0.05, 1.0, 1e6}) acc += ssqa_sa_accept_threshold(de, b);
    EXPECT(acc > 0);
}

static void gi_mapping(std::mt19937& rng) {
    for (int n = 1; n <= 12; ++n)
        for (int rep = 0; rep < 3; ++rep) {
            std::vector<uint8_t> a1((size_t)n * n, 0), a2((size_t)n * n, 0);
            std::vector<int> perm(n);
            for (int i = 0; i < n; ++i) perm[i] = i;
            std::shuffle(perm.begin(), perm.end(), rng);
            for (int i = 0; i < n; ++i)
                for (int j = i + 1; j < n; ++j)
                    if (rng() & 1) a1[i * n + j] = a1[j * n + i] = 1;
            for (int u = 0; u < n; ++u)
                for (int v = 0; v < n; ++v) a2[u * n + v] = a1[perm[u] * n + perm[v]];
            const int N = n * n;
            std::vector<int32_t> h(N), J((size_t)N * N);
            int64_t e_star = 0;
            const int c1 = 1 + rep, c2 = 1 + (rep + 1) % 3, scale = rep == 1 ? 4 : 12;
            EXPECT(ssqa_gi_to_ising(n, a1.data(), a2.data(), c1, c2, scale, h.data(), J.data(), &e_star) == SSQA_OK);
            // the isomorphism's spin configuration has energy e_star (Eq. 1 evaluated directly)
            std::vector<int> s(N, -1);
            for (int u = 0; u < n; ++u) s[u * n + perm[u]] = 1;
            long long e = 0;
            for (int p = 0; p < N; ++p) {
                e -= (long long)h[p] * s[p];
                for (int q = p + 1; q < N; ++q) e -= (long long)J[(size_t)p * N + q] * s[p] * s[q];
            }
            EXPECT(e == e_star);
        }
    std::vector<uint8_t> a(9, 0), b(9, 0);
    std::vector<int32_t> h(9), J(81);
    int64_t e = 0;
    a[1] = 1;   // not symmetric
    EXPECT(ssqa_gi_to_ising(3, a.data(), b.data(), 1, 1, 12, h.data(), J.data(), &e) == SSQA_EINVAL);
    a[1] = 0;
    a[4] = 1;   // diagonal
    EXPECT(ssqa_gi_to_ising(3, a.data(), b.data(), 1, 1, 12, h.data(), J.data(), &e) == SSQA_EINVAL);
    a[4] = 0;
    EXPECT(ssqa_gi_to_ising(3, a.data(), b.data(), 1, 1, 6, h.data(), J.data(), &e) == SSQA_EINVAL);
    EXPECT(ssqa_gi_to_ising(0, a.data(), b.data(), 1, 1, 12, h.data(), J.data(), &e) == SSQA_EINVAL);
    EXPECT(ssqa_gi_to_ising(129, a.data(), b.data(), 1, 1, 12, h.data(), J.data(), &e) == SSQA_EINVAL);
}

static void philox() {
    // Salmon et al. (SC'11) known answer: counter and key all zero.
    const uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0};
    uint32_t out[4];
    ssqa_philox4x32_10(ctr, key, out);
    EXPECT(out[0] == 0x6627e8d5u && out[1] == 0xe169c58du && out[2] == 0xbc57ac4cu && out[3] == 0x9b00dbd8u);
}

static void work_order(std::mt19937& rng) {
    using ssqa::detail::WorkItem;
    for (int rep = 0; rep < 50; ++rep) {
        const int anneals = 1 + (int)(rng() % 40), wg = 1 + (int)(rng() % 9), xcds = 1 + (int)(rng() % 8);
        std::vector<WorkItem> items;
        for (int a = 0; a < anneals; ++a)
            for (int c = 0; c < wg; ++c) items.push_back({(double)(anneals - a), ((uint32_t)a << 16) | (uint32_t)c});
        const auto out = ssqa::detail::xcd_grouped(items, xcds);
        EXPECT(out.size() == items.size());
    }
}

static ssqa_request request(int n, const std::vector<int32_t>& h, const std::vector<int32_t>& J,
                            const std::vector<int32_t>& q, const std::vector<int32_t>& i0, int R, int T) {
    ssqa_request r;
    std::memset(&r, 0, sizeof(r));
    r.n_spins = n;
    r.h = h.data();
    r.J = J.data();
    r.params.replicas = R;
    r.params.trials = T;
    r.params.cycles = (int32_t)q.size();
    r.params.delay = 1;
    r.params.alpha = 1;
    r.params.noise_amp = 12;
    r.params.jperp = q.data();
    r.params.i0 = i0.data();
    r.params.target_energy = SSQA_NO_TARGET;
    return r;
}

static void abi_checks() {
    for (int s : {0, -1, -2, -3, -4, -5, -99}) EXPECT(ssqa_status_string((ssqa_status)s) != nullptr);
    EXPECT(ssqa_last_error() != nullptr);
    // problems: every check before the device lookup
    const int n = 5;
    std::vector<int32_t> h(n, 3), J((size_t)n * n, 0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) J[(size_t)i * n + j] = -3 * ((i + j) % 3);
    ssqa_problem_t p = nullptr;
    EXPECT(ssqa_create_problem(0, h.data(), J.data(), 0, &p) == SSQA_EINVAL);
    EXPECT(ssqa_create_problem(n, nullptr, J.data(), 0, &p) == SSQA_EINVAL);
    EXPECT(ssqa_create_problem(n, h.data(), nullptr, 0, &p) == SSQA_EINVAL);
    std::vector<int32_t> Jb = J;
    Jb[1] = 7;   // not symmetric
    EXPECT(ssqa_create_problem(n, h.data(), Jb.data(), 0, &p) == SSQA_EINVAL);
    Jb = J;
    Jb[2 * n + 2] = 1;   // diagonal
    EXPECT(ssqa_create_problem(n, h.data(), Jb.data(), 0, &p) == SSQA_EINVAL);
    std::vector<int32_t> Jbig((size_t)n * n, 1 << 28);
    for (int i = 0; i < n; ++i) Jbig[(size_t)i * n + i] = 0;
    EXPECT(ssqa_create_problem(n, h.data(), Jbig.data(), 0, &p) == SSQA_ERANGE);
    {
        // a size whose checks run over host threads: an asymmetric pair and a diagonal entry are found
        const int big = 2100;
        std::vector<int32_t> hb(big, 1), Jb2((size_t)big * big, 0);
        for (int i = 0; i < big; ++i)
            for (int j = 0; j < big; ++j)
                if (i != j) Jb2[(size_t)i * big + j] = -3 * ((i + j) % 3);
        Jb2[(size_t)1500 * big + 77] = 5;
        EXPECT(ssqa_create_problem(big, hb.data(), Jb2.data(), 0, &p) == SSQA_EINVAL);
        EXPECT(std::strstr(ssqa_last_error(), "(77, 1500)") != nullptr);
        Jb2[(size_t)1500 * big + 77] = Jb2[(size_t)77 * big + 1500];
        Jb2[(size_t)2000 * big + 2000] = 1;
        EXPECT(ssqa_create_problem(big, hb.data(), Jb2.data(), 0, &p) == SSQA_EINVAL);
        EXPECT(std::strstr(ssqa_last_error(), "diagonal") != nullptr);
        Jb2[(size_t)2000 * big + 2000] = 0;
        const ssqa_status sb = ssqa_create_problem(big, hb.data(), Jb2.data(), 0, &p);
        EXPECT(sb == SSQA_OK || sb == SSQA_EDEVICE);
        if (sb == SSQA_OK) ssqa_destroy_problem(p);
    }
    const ssqa_status st = ssqa_create_problem(n, h.data(), J.data(), 0, &p);
    EXPECT(st == SSQA_OK || st == SSQA_EDEVICE);   // EDEVICE where no GPU is present
    if (st == SSQA_OK) ssqa_destroy_problem(p);
    EXPECT(ssqa_problem_spins(nullptr) == 0 && ssqa_problem_planes(nullptr) == 0);
    ssqa_destroy_problem(nullptr);
    // anneals
    ssqa_anneal_params pa;
    std::memset(&pa, 0, sizeof(pa));
    ssqa_anneal_outputs o;
    std::memset(&o, 0, sizeof(o));
    EXPECT(ssqa_anneal(nullptr, &pa, &o, nullptr) == SSQA_EINVAL);
    EXPECT(ssqa_anneal_noalloc(nullptr, &pa, &o, nullptr) == SSQA_EINVAL);
    ssqa_batch_t b = nullptr;
    EXPECT(ssqa_batch_create(0, nullptr, nullptr, nullptr, &b) == SSQA_EINVAL);
    EXPECT(ssqa_batch_create(1, nullptr, nullptr, nullptr, &b) == SSQA_EINVAL);
    EXPECT(ssqa_batch_run(nullptr, nullptr) == SSQA_EINVAL);
    ssqa_batch_destroy(nullptr);
    // server: creation, the submit-time bounds (host copies of h, J and schedules), poll, cancel, destroy
    ssqa_server_config cfg{0, 10, 16, int64_t(1) << 30};
    ssqa_server_t s = nullptr;
    EXPECT(ssqa_server_create(&cfg, &s) == SSQA_OK);
    std::vector<int32_t> q(40, 2), i0(40, 24);
    int64_t id = -1;
    ssqa_request r = request(n, h, J, q, i0, 8, 16);
    EXPECT(ssqa_server_submit(s, &r, &id) == SSQA_OK && id >= 0);
    int64_t id2 = -1;
    r = request(n, h, J, q, i0, 65, 4);
    EXPECT(ssqa_server_submit(s, &r, &id2) == SSQA_ENOTSUP);
    r = request(n, h, J, q, i0, 64, 70000);
    EXPECT(ssqa_server_submit(s, &r, &id2) == SSQA_EINVAL);
    r = request(n, h, J, q, i0, 1, 65535 * 64 + 1);
    EXPECT(ssqa_server_submit(s, &r, &id2) == SSQA_EINVAL);
    r = request(n, h, Jb, q, i0, 8, 4);   // the diagonal entry: J is checked at submit
    EXPECT(ssqa_server_submit(s, &r, &id2) == SSQA_EINVAL);
    std::vector<int32_t> Jw = J;             // entries beyond int8: kept as int32 until admission
    Jw[1] = Jw[n] = 1000;
    r = request(n, h, Jw, q, i0, 8, 4);
    EXPECT(ssqa_server_submit(s, &r, &id2) == SSQA_OK);
    r = request(n, h, J, q, i0, 33, 3);
    EXPECT(ssqa_server_submit(s, &r, &id2) == SSQA_OK);
    ssqa_request_info info;
    std::vector<int64_t> best(16);
    std::vector<int32_t> hit(16);
    EXPECT(ssqa_server_poll(s, id, &info, best.data(), hit.data()) == SSQA_OK && info.state == SSQA_REQ_QUEUED);
    EXPECT(ssqa_server_poll(s, 12345, &info, nullptr, nullptr) == SSQA_EINVAL);
    EXPECT(ssqa_server_cancel(s, id) == SSQA_OK);
    ssqa_server_stats_t stats;
    EXPECT(ssqa_server_stats(s, &stats) == SSQA_OK);
    ssqa_server_destroy(s);
    ssqa_server_destroy(nullptr);
    cfg.cycles_per_step = 0;
    EXPECT(ssqa_server_create(&cfg, &s) == SSQA_EINVAL);
}

// The autotuner's cache reader on a valid file, on every prefix of it (each must be refused) and on a few
// malformed variants; then a save / load round trip.
static void tune_cache(const char* dir) {
    const std::string path = std::string(dir) + "/tune_cache.json";
    const std::string good =
        "{\"format\": \"ssqa-tune-1\", \"entries\": [\n"
        "  {\"form\": \"plain\", \"device\": \"dev\\\"x\", \"kernel\": \"k\", \"np\": 256, \"planes\": 1, "
        "\"replicas\": 8, \"trials\": 64, \"delay\": 1, \"mode\": 0, \"fast\": 1, \"fp4_ok\": 1, "
        "\"block_columns\": 64, \"trials_per_block\": 8, \"operand_format\": 2, \"ms_per_cycle\": 1.5e-2},\n"
        "  {\"form\": \"batch\", \"device\": \"dev\", \"kernel\": \"k\", \"signature\": \"0123456789abcdef\", "
        "\"instances\": 3, \"wide_rows\": 0, \"ms_per_cycle\": 0, \"extra\": [true, false, null, {}]}\n]}\n";
    auto write = [&path](const std::string& text) {
        FILE* f = std::fopen(path.c_str(), "wb");
        if (!f) return false;
        std::fwrite(text.data(), 1, text.size(), f);
        std::fclose(f);
        return true;
    };
    ssqa_tune_clear();
    int32_t n = -1;
    EXPECT(write(good) && ssqa_tune_load(path.c_str(), &n) == SSQA_OK && n == 2);
    EXPECT(ssqa_tune_entries() == 2);
    const size_t body = good.size() - 2;   // without the closing brace and newline
    for (size_t len = 0; len < body; ++len) {
        EXPECT(write(good.substr(0, len)));
        EXPECT(ssqa_tune_load(path.c_str(), &n) == SSQA_EINVAL);
    }
    for (const char* bad : {"{", "[", "\"", "{\"format\": \"ssqa-tune-1\", \"entries\": [{\"form\": 1}]}",
                            "{\"a\": [[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[1]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]}",
                            "{\"format\": \"ssqa-tune-1\", \"entries\": [], \"x\": \"\\u0041\"}", "-", "1e999"}) {
        EXPECT(write(bad));
        EXPECT(ssqa_tune_load(path.c_str(), &n) == SSQA_EINVAL);
    }
    EXPECT(ssqa_tune_entries() == 2);
    EXPECT(ssqa_tune_save(path.c_str()) == SSQA_OK);
    ssqa_tune_clear();
    EXPECT(ssqa_tune_load(path.c_str(), &n) == SSQA_OK && n == 2);
    ssqa_tune_clear();
    EXPECT(ssqa_tune_load(nullptr, &n) == SSQA_EINVAL && ssqa_tune_save(nullptr) == SSQA_EINVAL);
}

int main(int argc, char** argv) {
    std::mt19937 rng(12345);
    schedules();
    gi_mapping(rng);
    philox();
    work_order(rng);
    abi_checks();
    tune_cache(argc > 1 ? argv[1] : ".");
    if (g_bad) {
        std::printf("%d checks failed\n", g_bad);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
