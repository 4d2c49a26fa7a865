// Launch order of the work items of the batched and served launches (host code, no HIP dependency).
#pragma once

#include <cstdint>
#include <vector>

namespace ssqa {
namespace detail {

// One work item of a launch: workgroup (code & 0xFFFF) of anneal (code >> 16), with its cost.
struct WorkItem {
    double cost;
    uint32_t code;
};

// Launch order of a launch's work items for a device whose workgroups go to its XCDs in turn (workgroup b to
// XCD b mod xcds).  `sorted` holds the items by decreasing cost, each anneal's items together.  When every
// anneal has the same number of items, whole anneals are dealt to the XCDs (in a snake order over the
// anneals by decreasing cost, so that the XCDs' totals stay close), and each XCD's items keep decreasing
// cost.  An XCD then runs the workgroups of few anneals at a time, whose J stays in its L2, instead of a
// share of every anneal in flight.  The anneals left over after whole rounds of xcds are dealt item by item.
// Any order gives the same results; this one only changes where J is read from.
inline std::vector<WorkItem> xcd_grouped(const std::vector<WorkItem>& sorted, int xcds) {
    if (xcds < 2 || sorted.empty()) return sorted;
    std::vector<size_t> starts;   // first item of each anneal
    for (size_t i = 0; i < sorted.size(); ++i)
        if (i == 0 || (sorted[i].code >> 16) != (sorted[i - 1].code >> 16)) starts.push_back(i);
    const size_t groups = starts.size();
    const size_t g = sorted.size() / groups;
    for (size_t k = 0; k < groups; ++k) {
        const size_t end = k + 1 < groups ? starts[k + 1] : sorted.size();
        if (end - starts[k] != g) return sorted;   // anneals of different item counts: keep the cost order
    }
    if (groups < (size_t)xcds) return sorted;
    std::vector<std::vector<WorkItem>> q(xcds);
    const size_t full = groups - groups % xcds;
    for (size_t k = 0; k < full; ++k) {
        const size_t round = k / xcds, pos = k % xcds;
        const size_t x = (round % 2 == 0) ? pos : xcds - 1 - pos;
        q[x].insert(q[x].end(), sorted.begin() + starts[k], sorted.begin() + starts[k] + g);
    }
    size_t j = 0;
    for (size_t i = full * g; i < sorted.size(); ++i, ++j) q[j % xcds].push_back(sorted[i]);
    // queue lengths are non-increasing in x and differ by at most one, so position k * xcds + x is q[x][k]
    std::vector<WorkItem> out;
    out.reserve(sorted.size());
    for (size_t k = 0; out.size() < sorted.size(); ++k)
        for (int x = 0; x < xcds; ++x)
            if (k < q[x].size()) out.push_back(q[x][k]);
    return out;
}

// XCDs (accelerator complexes, each with its own L2) of a device; 1 when the runtime does not report them.
int device_xcd_count(int device);

}  // namespace detail
}  // namespace ssqa
