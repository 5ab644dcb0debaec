// fw_route.h -- which graphs of a batch fw_apsp_batched hands to fw_apsp
// instead of its persistent launch.  Plain C++: the runtime calls it, and a
// host-only test checks it.
#pragma once
#include <stdint.h>

namespace fw {

constexpr int32_t kRouteMinN = 256;
constexpr double kRouteFactor = 4.0;

// In the persistent launch one workgroup solves one graph, so a graph that
// alone holds much more than the batch's work per resident workgroup (`slots`
// of them) would finish long after the rest.  route = 0: graphs with
// n >= kRouteMinN and n^3 > kRouteFactor * (sum of n^3) / slots; -1: none;
// k > 0: every graph with n >= k.  Sets routed[b] to 1 for a routed graph, else
// 0, and returns how many are routed.
inline int32_t batched_route(const int32_t *n, int32_t batch, int64_t slots, int32_t route, uint8_t *routed) {
    double work = 0.0;
    for (int32_t b = 0; b < batch; ++b) work += (double)n[b] * n[b] * n[b];
    const double share = work / (double)(slots > 0 ? slots : 1);
    int32_t count = 0;
    for (int32_t b = 0; b < batch; ++b) {
        const double nb = n[b];
        bool r = false;
        if (route > 0)
            r = n[b] >= route;
        else if (route == 0)
            r = n[b] >= kRouteMinN && nb * nb * nb > kRouteFactor * share;
        routed[b] = r ? 1 : 0;
        count += r ? 1 : 0;
    }
    return count;
}

}  // namespace fw
