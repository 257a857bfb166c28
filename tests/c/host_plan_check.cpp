// The work plans of the pair sweeps (plan_sym and plan_band in
// paper_2312_10044_amd/csrc/pb_host.cpp) for a list of (kind, npad, target)
// cases given on the command line, kind "sym" or "band", built with
// AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py, which checks what it prints.
//   sym:  "case sym npad target n_items tiles_per_item strips", one
//         "item I J0 J1 slot" line per item in launch order, and
//         "rowstart r0 r1 ... rT";
//   band: "case band npad target n_items run band n_records", one
//         "item m0 m1 j0 j1 rslot cslot" line per item and one
//         "list K idx..." line per tile.
#include "pb_host.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

int main(int argc, char **argv)
{
    for (int a = 1; a + 2 < argc; a += 3) {
        const bool sym = std::strcmp(argv[a], "sym") == 0;
        const long long npad = std::atoll(argv[a + 1]);
        const int target = std::atoi(argv[a + 2]);
        if (sym) {
            std::vector<int32_t> items, rs;
            const pbk::SymPlan pl = pbk::plan_sym(npad, target, items, rs);
            std::printf("case sym %lld %d %d %d %d\n", npad, target, pl.n_items, pl.tiles_per_item,
                        pl.strips);
            for (size_t k = 0; k + 3 < items.size(); k += 4)
                std::printf("item %d %d %d %d\n", items[k], items[k + 1], items[k + 2],
                            items[k + 3]);
            std::printf("rowstart");
            for (int32_t v : rs)
                std::printf(" %d", v);
            std::printf("\n");
            continue;
        }
        std::vector<pbk::BandItem> items;
        std::vector<int32_t> rs, ri;
        const pbk::BandPlan pl = pbk::plan_band(npad, target, items, rs, ri);
        std::printf("case band %lld %d %d %d %d %lld\n", npad, target, pl.n_items, pl.run,
                    pl.band, (long long)pl.n_records);
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
