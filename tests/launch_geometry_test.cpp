// CPU test of the traversal launch geometry (paper_1901_08088_amd/csrc/
// launch_geometry.h): for systems of several types, the workgroups the host
// launches (trav_blocks) hold every wavefront the device maps queries to
// (type_waves per stretch), and the stretches together cover every query of
// every type exactly once; for one type, the workgroups cover all queries.
// Built with g++ by tests/test_launch_geometry.py; exits non-zero on failure.
#include <stdio.h>
#include <stdint.h>

#include <algorithm>
#include <random>
#include <vector>

#include "../paper_1901_08088_amd/csrc/launch_geometry.h"

using namespace qbi;

static int check(int64_t n, const std::vector<int64_t> &counts, int32_t block, int32_t qpw) {
    const int32_t ntypes = (int32_t)counts.size();
    const int64_t blocks = trav_blocks(n, ntypes, block, qpw);
    if (ntypes == 1) {
        if (blocks * (block / 64) * qpw < n) {
            fprintf(stderr, "one type: n=%lld block=%d qpw=%d blocks=%lld too few\n", (long long)n, block, qpw,
                    (long long)blocks);
            return 1;
        }
        return 0;
    }
    if (blocks % 8 != 0) {
        fprintf(stderr, "blocks %lld not a multiple of 8\n", (long long)blocks);
        return 1;
    }
    const int64_t capacity = blocks / 8 * (block / 64);  // wavefronts per stretch
    std::vector<int64_t> covered(ntypes, 0);
    for (int64_t part = 0; part < 8; ++part) {
        int64_t waves = 0;
        for (int t = 0; t < ntypes; ++t) {
            const int32_t len = stretch_lo(counts[t], part + 1) - stretch_lo(counts[t], part);
            const int32_t nw = type_waves(counts[t], n, qpw, part);
            const int32_t qt = type_qpw(counts[t], n, qpw);
            if ((int64_t)nw * qt < len || (nw > 0 && (int64_t)(nw - 1) * qt >= len)) {
                fprintf(stderr, "type %d part %lld: %d wavefronts of %d for %d queries\n", t, (long long)part, nw,
                        qt, len);
                return 1;
            }
            if (stretch_lo(counts[t], part) != covered[t]) {
                fprintf(stderr, "type %d part %lld starts at %d, expected %lld\n", t, (long long)part,
                        stretch_lo(counts[t], part), (long long)covered[t]);
                return 1;
            }
            covered[t] += len;
            waves += nw;
        }
        if (waves > capacity) {
            fprintf(stderr, "n=%lld ntypes=%d block=%d qpw=%d part %lld: %lld wavefronts, room for %lld\n",
                    (long long)n, ntypes, block, qpw, (long long)part, (long long)waves, (long long)capacity);
            return 1;
        }
    }
    for (int t = 0; t < ntypes; ++t)
        if (covered[t] != counts[t]) {
            fprintf(stderr, "type %d: %lld of %lld queries covered\n", t, (long long)covered[t],
                    (long long)counts[t]);
            return 1;
        }
    return 0;
}

int main() {
    std::mt19937_64 rng(19010888);
    const int32_t blocks[] = {64, 128, 192, 256};
    const int32_t qpws[] = {1, 2, 4, 8, 16, 32, 64};
    int64_t cases = 0;
    for (int trial = 0; trial < 300000; ++trial) {
        const int32_t ntypes = 1 + (int32_t)(rng() % 4);
        const int scale = (int)(rng() % 3);
        const int64_t nmax = scale == 0 ? 100 : (scale == 1 ? 20000 : 134217727);
        const int64_t n = (int64_t)(rng() % (uint64_t)(nmax + 1));
        std::vector<int64_t> cuts(ntypes - 1);
        for (auto &c : cuts) c = n ? (int64_t)(rng() % (uint64_t)(n + 1)) : 0;
        std::sort(cuts.begin(), cuts.end());
        std::vector<int64_t> counts(ntypes);
        int64_t prev = 0;
        for (int t = 0; t < ntypes - 1; ++t) {
            counts[t] = cuts[t] - prev;
            prev = cuts[t];
        }
        counts[ntypes - 1] = n - prev;
        if (rng() % 4 == 0) {  // everything in one type, the others empty
            for (auto &c : counts) c = 0;
            counts[rng() % ntypes] = n;
        }
        const int32_t block = blocks[rng() % 4];
        const int32_t qpw = qpws[rng() % 7];
        if (check(n, counts, block, qpw)) return 1;
        ++cases;
    }
    printf("all checks passed (%lld cases)\n", (long long)cases);
    return 0;
}
