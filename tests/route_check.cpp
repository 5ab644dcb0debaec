// Host-only driver of the batched routing rule (csrc/fw_route.h): reads cases
// from stdin, one per line -- "slots route n_0 n_1 ..." -- and prints, per case,
// the routed flags as a string of 0 and 1.  tests/test_route.py checks them.
#include <cstdio>
#include <sstream>
#include <string>
#include <vector>
#include <iostream>

#include "../paper_2105_07298_amd/csrc/fw_route.h"

int main() {
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        long long slots = 0;
        int route = 0;
        if (!(in >> slots >> route)) continue;
        std::vector<int32_t> n;
        int32_t v;
        while (in >> v) n.push_back(v);
        std::vector<uint8_t> r(n.size());
        const int32_t count = fw::batched_route(n.data(), (int32_t)n.size(), slots, route, r.data());
        std::string flags;
        for (uint8_t x : r) flags += x ? '1' : '0';
        std::printf("%d %s\n", count, flags.c_str());
    }
    return 0;
}
