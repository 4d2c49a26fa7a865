// Host check of the XCD-aware launch order (paper_2302_12454_amd/csrc/work_order.hpp): a worked example,
// then random work lists.  Prints "ok" and exits 0 when every property holds.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <map>
#include <random>
#include <vector>

#include "work_order.hpp"

using ssqa::detail::WorkItem;
using ssqa::detail::xcd_grouped;

static uint32_t code(uint32_t anneal, uint32_t wg) { return (anneal << 16) | wg; }

static std::vector<WorkItem> sorted_items(const std::vector<int>& sizes, const std::vector<double>& costs) {
    std::vector<WorkItem> items;
    for (size_t a = 0; a < sizes.size(); ++a)
        for (int c = 0; c < sizes[a]; ++c) items.push_back({costs[a], code((uint32_t)a, (uint32_t)c)});
    std::stable_sort(items.begin(), items.end(), [](const WorkItem& x, const WorkItem& y) { return x.cost > y.cost; });
    return items;
}

int main() {
    int bad = 0;
    // Worked example: 2 XCDs, anneals 0..4 of 2 items with costs 5..1.  Whole rounds deal 0 -> XCD 0,
    // 1 -> XCD 1, then (snake) 2 -> XCD 1, 3 -> XCD 0; anneal 4 is left over and dealt item by item.
    // XCD 0 runs 0.0 0.1 3.0 3.1 4.0 and XCD 1 runs 1.0 1.1 2.0 2.1 4.1, interleaved by position.
    {
        const auto out = xcd_grouped(sorted_items({2, 2, 2, 2, 2}, {5, 4, 3, 2, 1}), 2);
        const std::vector<uint32_t> want = {code(0, 0), code(1, 0), code(0, 1), code(1, 1), code(3, 0),
                                            code(2, 0), code(3, 1), code(2, 1), code(4, 0), code(4, 1)};
        std::vector<uint32_t> got;
        for (const auto& e : out) got.push_back(e.code);
        if (got != want) {
            std::printf("worked example differs\n");
            ++bad;
        }
    }
    // Unchanged cases: one XCD, fewer anneals than XCDs, anneals of different sizes.
    {
        const auto a = sorted_items({3, 3, 3}, {3, 2, 1});
        const auto b = sorted_items({3, 4, 3, 3, 3, 3, 3, 3, 3}, {9, 8, 7, 6, 5, 4, 3, 2, 1});
        for (const auto& [items, xcds] : {std::make_pair(a, 1), std::make_pair(a, 8), std::make_pair(b, 8)}) {
            const auto out = xcd_grouped(items, xcds);
            bool same = out.size() == items.size();
            for (size_t i = 0; same && i < out.size(); ++i) same = out[i].code == items[i].code;
            if (!same) {
                std::printf("order changed where it should be kept\n");
                ++bad;
            }
        }
    }
    // Random lists: a permutation; per XCD (position mod xcds) cost never rises; with equal sizes only the
    // anneals left over after whole rounds run on more than one XCD.
    std::mt19937 rng(1);
    for (int trial = 0; trial < 2000; ++trial) {
        const int xcds = (trial % 3 == 0) ? 8 : 1 + (int)(rng() % 9);
        const int groups = 1 + (int)(rng() % 300);
        const bool equal = trial % 4 != 0;
        const int g0 = 1 + (int)(rng() % 40);
        std::vector<int> sizes(groups);
        std::vector<double> costs(groups);
        for (int a = 0; a < groups; ++a) {
            sizes[a] = equal ? g0 : 1 + (int)(rng() % 40);
            costs[a] = (double)(rng() % 50);
        }
        const auto items = sorted_items(sizes, costs);
        const auto out = xcd_grouped(items, xcds);
        std::vector<uint32_t> x, y;
        for (const auto& e : items) x.push_back(e.code);
        for (const auto& e : out) y.push_back(e.code);
        std::sort(x.begin(), x.end());
        std::sort(y.begin(), y.end());
        if (x != y) {
            std::printf("trial %d: not a permutation\n", trial);
            ++bad;
            continue;
        }
        std::vector<double> last(xcds, 1e300);
        std::map<uint32_t, uint32_t> on;   // anneal -> bit set of XCDs it runs on
        for (size_t p = 0; p < out.size(); ++p) {
            const int q = (int)(p % xcds);
            if (out[p].cost > last[q]) {
                std::printf("trial %d: cost rises on XCD %d\n", trial, q);
                ++bad;
                break;
            }
            last[q] = out[p].cost;
            on[out[p].code >> 16] |= 1u << q;
        }
        if (xcds >= 2 && equal && groups >= xcds) {
            int spread = 0;
            for (const auto& kv : on) spread += __builtin_popcount(kv.second) > 1;
            if (spread > groups % xcds) {
                std::printf("trial %d: %d anneals spread, %d left over\n", trial, spread, groups % xcds);
                ++bad;
            }
        }
    }
    if (bad == 0) std::printf("ok\n");
    return bad != 0;
}
