// The library's host octree (paper_2312_10044_amd/csrc/pb_host.cpp) on a point
// set read from a file, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Input: n, n0
// (int64) then x [n], y [n], z [n] (double).  Output file: for the threaded
// and the single-threaded build, the leaf count, start [L + 1] and perm [n]
// (int64), which the test compares with the oracle's leaves.
#include "pb_host.h"

#include <cstdint>
#include <cstdio>
#include <vector>

int main(int argc, char **argv)
{
    if (argc != 3)
        return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f)
        return 2;
    int64_t hdr[2];
    if (std::fread(hdr, sizeof(int64_t), 2, f) != 2)
        return 2;
    const int64_t n = hdr[0];
    std::vector<double> xyz(3 * n);
    if (std::fread(xyz.data(), sizeof(double), 3 * n, f) != (size_t)(3 * n))
        return 2;
    std::fclose(f);
    FILE *o = std::fopen(argv[2], "wb");
    if (!o)
        return 2;
    for (int threads = 1; threads >= 0; --threads) {
        std::vector<int32_t> perm, start;
        pbk::build_leaves(xyz.data(), xyz.data() + n, xyz.data() + 2 * n, n, (int)hdr[1], perm,
                          start, threads != 0);
        const int64_t L = (int64_t)start.size() - 1;
        std::fwrite(&L, sizeof(int64_t), 1, o);
        for (int32_t v : start) {
            const int64_t w = v;
            std::fwrite(&w, sizeof(int64_t), 1, o);
        }
        for (int32_t v : perm) {
            const int64_t w = v;
            std::fwrite(&w, sizeof(int64_t), 1, o);
        }
    }
    std::fclose(o);
    return 0;
}
