// Launch order of the work items of the batched and served launches (host code).
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
std::vector<WorkItem> xcd_grouped(const std::vector<WorkItem>& sorted, int xcds);

// XCDs (accelerator complexes, each with its own L2) of a device; 1 when the runtime does not report them.
int device_xcd_count(int device);

}  // namespace detail
}  // namespace ssqa
