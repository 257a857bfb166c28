// The work plan of the banded pair sweep (plan_band in
// paper_2312_10044_amd/csrc/pb_host.cpp) for a list of (npad, target items)
// cases given on the command line, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  For each case
// it prints "case npad target n_items run band n_records", one
// "item m0 m1 j0 j1 rslot cslot" line per item and one "list K idx..." line
// per tile, which the test checks for coverage.
#include "pb_host.h"

#include <cstdio>
#include <cstdlib>
#include <vector>

int main(int argc, char **argv)
{
    for (int a = 1; a + 1 < argc; a += 2) {
        const long long npad = std::atoll(argv[a]);
        const int target = std::atoi(argv[a + 1]);
        std::vector<pbk::BandItem> items;
        std::vector<int32_t> rs, ri;
        const pbk::BandPlan pl = pbk::plan_band(npad, target, items, rs, ri);
        std::printf("case %lld %d %d %d %d %lld\n", npad, target, pl.n_items, pl.run, pl.band,
                    (long long)pl.n_records);
        for (const auto &it : items)
            std::printf("item %d %d %d %d %d %d\n", it.m0, it.m1, it.j0, it.j1, it.rslot,
                        it.cslot);
        for (int K = 0; K + 1 < (int)rs.size(); ++K) {
            std::printf("list %d", K);
            for (int q = rs[K]; q < rs[K + 1]; ++q)
                std::printf(" %d", ri[q]);
            std::printf("\n");
        }
    }
    return 0;
}
