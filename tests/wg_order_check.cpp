// Property checks of the work-group orders of the grouped launches (host
// code of the library, compiled here with the system C++ compiler): every
// (product, tile) entry of a table appears exactly once after reordering,
// padding entries are item -1, the tiles that an order promises to keep on
// one XCD (entry index mod 8) are there, and the reordered table fits the
// capacity the library allocates for it. Prints "ok" or the first failure.
#include <cstdio>
#include <map>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "wg_order.h"

using Table = std::vector<int>;

static bool same_entries(const Table& wi0, const Table& wt0, const Table& wi, const Table& wt) {
    std::multiset<std::pair<int, int>> a, b;
    for (size_t e = 0; e < wi0.size(); ++e) a.insert({wi0[e], wt0[e]});
    for (size_t e = 0; e < wi.size(); ++e) {
        if (wi[e] < 0) {
            if (wt[e] != 0) return false;
            continue;
        }
        b.insert({wi[e], wt[e]});
    }
    return a == b;
}

int main() {
    std::mt19937 rng(12345);
    for (int trial = 0; trial < 3000; ++trial) {
        const int G = 1 + (int)(rng() % 50);
        std::vector<int> tr(G), ts(G), act(G), trs;
        std::vector<double> w(G);
        size_t full = 0;
        for (int g = 0; g < G; ++g) {
            tr[g] = 1 + (int)(rng() % 3);   // row tiles
            ts[g] = 1 + (int)(rng() % 12);  // operator column tiles
            w[g] = 8.0 * (1 + rng() % 6);   // cost of one tile
            act[g] = rng() % 4 != 0;
            full += (size_t)tr[g] * ts[g];
            trs.push_back(tr[g]);
        }
        Table wi0, wt0;
        for (int g = 0; g < G; ++g)
            if (act[g])
                for (int t = 0; t < tr[g] * ts[g]; ++t) {
                    wi0.push_back(g);
                    wt0.push_back(t);
                }
        for (int mode = 0; mode <= 3; ++mode) {
            Table wi = wi0, wt = wt0;
            pe::wg_order(mode, wi, wt, [&](int g) { return w[g]; }, [&](int g) { return tr[g]; });
            if (!same_entries(wi0, wt0, wi, wt)) {
                std::printf("mode %d trial %d: entries changed\n", mode, trial);
                return 1;
            }
            const size_t cap = (mode == 1 || mode == 3) ? 8 * full + 8 : mode == 2 ? pe::rowtile_cap(full, trs) : full;
            if (wi.size() > cap) {
                std::printf("mode %d trial %d: %zu entries over the capacity %zu\n", mode, trial, wi.size(), cap);
                return 1;
            }
            if (!wi.empty() && wi.back() < 0) {
                std::printf("mode %d trial %d: trailing padding\n", mode, trial);
                return 1;
            }
            // XCD of each group the order keeps together
            std::map<std::pair<int, int>, int> xcd;
            for (size_t e = 0; e < wi.size(); ++e) {
                if (wi[e] < 0) continue;
                const int g = wi[e];
                std::pair<int, int> key{g, 0};
                if (mode == 0) continue;
                if (mode == 2) key.second = wt[e] / tr[g];  // one operator column tile
                auto it = xcd.find(key);
                if (it == xcd.end())
                    xcd[key] = (int)(e % 8);
                else if (it->second != (int)(e % 8)) {
                    std::printf("mode %d trial %d: item %d split over XCDs\n", mode, trial, g);
                    return 1;
                }
            }
            if (mode == 0 && (wi != wi0 || wt != wt0)) {
                std::printf("mode 0 trial %d: plain order changed\n", trial);
                return 1;
            }
        }
    }
    std::printf("ok\n");
    return 0;
}
