// Work-group orders of the grouped launches of a batch (host code only).
// A table lists, per work-group, the product (item) and the tile of that
// product it computes; the GPU's dispatcher sends work-group w to XCD w % 8,
// each XCD with its own L2. Entries with item -1 are padding: those
// work-groups return at once.
#pragma once
#include <algorithm>
#include <cstddef>
#include <map>
#include <set>
#include <utility>
#include <vector>

namespace pe {

// XCD-aware order of a grouped launch's work-group table. The dispatcher
// sends work-group w to XCD w % 8, and each XCD has its own L2: with this
// order all tiles of one product run on one XCD (its state operand is read
// into one L2, its row tiles of one operator tile share it), the products
// are spread over the XCDs by weight (greedy, heaviest first), and the eight
// lists are interleaved, the shorter ones padded with item -1 (work-groups
// that return at once). weight(item) is the cost of one tile of the item.
template <typename W>
void xcd_order(std::vector<int>& wi, std::vector<int>& wt, W weight) {
    constexpr int X = 8;
    std::vector<std::pair<size_t, size_t>> runs;
    for (size_t a = 0; a < wi.size();) {
        size_t b = a;
        while (b < wi.size() && wi[b] == wi[a]) ++b;
        runs.push_back({a, b});
        a = b;
    }
    std::vector<double> w(runs.size());
    for (size_t r = 0; r < runs.size(); ++r) w[r] = weight(wi[runs[r].first]) * (double)(runs[r].second - runs[r].first);
    std::vector<size_t> idx(runs.size());
    for (size_t r = 0; r < idx.size(); ++r) idx[r] = r;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t p, size_t q) { return w[p] > w[q]; });
    std::vector<std::vector<int>> bi(X), bt(X);
    std::vector<double> load(X, 0.0);
    for (size_t r : idx) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (size_t e = runs[r].first; e < runs[r].second; ++e) {
            bi[x].push_back(wi[e]);
            bt[x].push_back(wt[e]);
        }
        load[x] += w[r];
    }
    size_t L = 0;
    for (int x = 0; x < X; ++x) L = std::max(L, bi[x].size());
    std::vector<int> oi, ot;
    oi.reserve(L * X);
    ot.reserve(L * X);
    for (size_t j = 0; j < L; ++j)
        for (int x = 0; x < X; ++x) {
            oi.push_back(j < bi[x].size() ? bi[x][j] : -1);
            ot.push_back(j < bt[x].size() ? bt[x][j] : 0);
        }
    while (!oi.empty() && oi.back() < 0) {
        oi.pop_back();
        ot.pop_back();
    }
    wi.swap(oi);
    wt.swap(ot);
}

// Row-tile grouping of a grouped launch's work-group table: the row tiles
// of one product that share an operator column tile (tiles ts * g ..
// ts * g + g - 1, g = tiles_r(item)) are placed 8 entries apart, so the
// dispatcher (work-group w to XCD w % 8) sends them to one XCD at about
// the same time and that XCD's L2 serves the operator panel to all of
// them. Runs of 8 groups of one size g fill 8 g consecutive entries (every
// run starts at a multiple of 8); the last run of each size is padded with
// item -1 (at most 7 g entries per size).
template <typename TR>
void rowtile_order(std::vector<int>& wi, std::vector<int>& wt, TR tiles_r) {
    constexpr int X = 8;
    std::map<int, std::vector<std::pair<int, int>>> pend;  // group size -> (item, first tile)
    std::vector<int> oi, ot;
    oi.reserve(wi.size() + 64);
    ot.reserve(wi.size() + 64);
    auto flush = [&](int g, std::vector<std::pair<int, int>>& v) {
        for (int rr = 0; rr < g; ++rr)
            for (int x = 0; x < X; ++x) {
                const bool live = x < (int)v.size();
                oi.push_back(live ? v[x].first : -1);
                ot.push_back(live ? v[x].second + rr : 0);
            }
        v.clear();
    };
    for (size_t e = 0; e < wi.size(); ++e) {
        const int g = std::max(1, tiles_r(wi[e]));
        if (wt[e] % g) continue;  // not the first row tile of its group
        std::vector<std::pair<int, int>>& v = pend[g];
        v.push_back({wi[e], wt[e]});
        if ((int)v.size() == X) flush(g, v);
    }
    for (auto& kv : pend)
        if (!kv.second.empty()) flush(kv.first, kv.second);
    while (!oi.empty() && oi.back() < 0) {
        oi.pop_back();
        ot.pop_back();
    }
    wi.swap(oi);
    wt.swap(ot);
}

// Product-per-XCD order in lockstep: the products are sorted by tile cost
// and tile count and taken in groups of 8 of about the same size; within a
// group product x goes to XCD x, and the group's tile lists are
// interleaved (entry 8 j + x is tile j of product x; a shorter list is
// padded with item -1). Every tile of a product then runs on one XCD, so
// its state operand is fetched into one L2 and shared by all of that
// product's tiles there, while the eight XCDs work on tiles of equal cost
// at every point of the launch (work-groups are handed to the XCDs in
// turn, so a list of heavier tiles on one XCD would hold the others back).
template <typename W>
void lockstep_order(std::vector<int>& wi, std::vector<int>& wt, W weight) {
    constexpr int X = 8;
    struct Run {
        size_t a, b;
        double w;
    };
    std::vector<Run> runs;
    for (size_t a = 0; a < wi.size();) {
        size_t b = a;
        while (b < wi.size() && wi[b] == wi[a]) ++b;
        runs.push_back({a, b, weight(wi[a])});
        a = b;
    }
    std::stable_sort(runs.begin(), runs.end(), [](const Run& p, const Run& q) {
        return p.w != q.w ? p.w > q.w : (p.b - p.a) > (q.b - q.a);
    });
    std::vector<int> oi, ot;
    oi.reserve(wi.size() + 64);
    ot.reserve(wi.size() + 64);
    for (size_t g0 = 0; g0 < runs.size(); g0 += X) {
        const size_t g1 = std::min(runs.size(), g0 + X);
        size_t L = 0;
        for (size_t r = g0; r < g1; ++r) L = std::max(L, runs[r].b - runs[r].a);
        for (size_t j = 0; j < L; ++j)
            for (size_t x = 0; x < (size_t)X; ++x) {
                const size_t r = g0 + x;
                const bool live = r < g1 && j < runs[r].b - runs[r].a;
                oi.push_back(live ? wi[runs[r].a + j] : -1);
                ot.push_back(live ? wt[runs[r].a + j] : 0);
            }
    }
    while (!oi.empty() && oi.back() < 0) {
        oi.pop_back();
        ot.pop_back();
    }
    wi.swap(oi);
    wt.swap(ot);
}

// entries a table can need after rowtile_order: the plain count plus the
// padding of one partial run per distinct group size
inline size_t rowtile_cap(size_t n, const std::vector<int>& sizes) {
    std::set<int> d(sizes.begin(), sizes.end());
    size_t pad = 0;
    for (int g : d) pad += 8 * (size_t)std::max(1, g);
    return n + pad;
}

// work-group order of a grouped launch's table (PE_BATCH_XCD: 1 every tile
// of a product on one XCD, balanced by weight; 2 the row tiles of an
// operator column tile on one XCD; 3 every tile of a product on one XCD,
// eight products of equal size in lockstep; 0 the plain order)
template <typename W, typename TR>
void wg_order(int mode, std::vector<int>& wi, std::vector<int>& wt, W weight, TR tiles_r) {
    if (mode == 1) xcd_order(wi, wt, weight);
    if (mode == 2) rowtile_order(wi, wt, tiles_r);
    if (mode == 3) lockstep_order(wi, wt, weight);
}

}  // namespace pe
