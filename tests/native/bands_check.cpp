// Host checks of the batched two-step basis's band tables and dispatch order
// (bands.h).  Reads "nrhs cus" and then one "nx ny nz" line per system from
// stdin; prints one line per failed check ("FAIL ...") and, at the end, the
// largest per-XCD work over the mean for both dispatch orders.
#include <cmath>
#include <cstdio>
#include <iostream>
#include <vector>

#include "bands.h"

using namespace sstep;

static int fails = 0;

static void check(bool ok, const char *what, long a = 0, long b = 0)
{
    if (!ok) {
        ++fails;
        std::printf("FAIL %s (%ld, %ld)\n", what, a, b);
    }
}

// Every system's rows x planes covered exactly once, each band within the
// thread budget (its rows plus one on each side, or the whole plane), ranges
// at most kzt planes, entries grouped by system in order.
static void check_table(const std::vector<BF2Tile> &tab, const std::vector<BandGrid> &g, int kzt)
{
    int last_q = -1;
    for (size_t q = 0; q < g.size(); ++q) {
        std::vector<int> cover(size_t(g[q].ny * g[q].nz), 0);
        for (const BF2Tile &t : tab) {
            if (t.q != int(q))
                continue;
            check(t.y0 >= 0 && t.y0 < t.y1 && t.y1 <= g[q].ny, "band rows in the grid", t.y0, t.y1);
            check(t.k0 >= 0 && t.k0 < t.k1 && t.k1 <= g[q].nz, "range planes in the grid", t.k0, t.k1);
            check(t.k1 - t.k0 <= kzt, "range no longer than asked", t.k1 - t.k0, kzt);
            const int64_t rows = t.y1 - t.y0 + (t.y0 > 0) + (t.y1 < g[q].ny);
            check(rows * g[q].nx <= kBf2Threads, "band and ring rows fit one block", long(rows), long(g[q].nx));
            for (int y = t.y0; y < t.y1; ++y)
                for (int k = t.k0; k < t.k1; ++k)
                    ++cover[size_t(k) * size_t(g[q].ny) + size_t(y)];
        }
        for (int c : cover)
            check(c == 1, "every row and plane in exactly one band", long(q), c);
    }
    for (const BF2Tile &t : tab) {
        check(t.q >= last_q, "entries grouped by system", t.q, last_q);
        last_q = t.q;
    }
}

// Each logical block once, padding elsewhere; a band's right-hand sides run
// consecutively on one XCD; with whole systems, a system on one XCD.
// Returns the largest per-XCD work over the mean.
static double check_map(const std::vector<uint32_t> &map, const std::vector<BF2Tile> &tab,
                        const std::vector<BandGrid> &g, int nrhs, bool whole, int nxcd)
{
    const size_t nbl = tab.size() * size_t(nrhs);
    check(map.size() % size_t(nxcd) == 0, "map a whole number of rounds", long(map.size()), nxcd);
    std::vector<int> seen(nbl, 0);
    std::vector<int> xcd_of(nbl, -1);
    std::vector<long> pos_of(nbl, -1);
    for (size_t b = 0; b < map.size(); ++b) {
        if (map[b] == kBf2NoBlock)
            continue;
        check(map[b] < nbl, "map entry in range", long(map[b]), long(nbl));
        if (map[b] >= nbl)
            continue;
        ++seen[map[b]];
        xcd_of[map[b]] = int(b % size_t(nxcd));
        pos_of[map[b]] = long(b / size_t(nxcd));
    }
    for (size_t l = 0; l < nbl; ++l)
        check(seen[l] == 1, "every logical block exactly once", long(l), seen[l]);
    // padding only after an XCD's queue
    for (int x = 0; x < nxcd; ++x) {
        bool pad = false;
        for (size_t b = size_t(x); b < map.size(); b += size_t(nxcd)) {
            if (map[b] == kBf2NoBlock)
                pad = true;
            else
                check(!pad, "no block after an XCD's padding", x, long(b));
        }
    }
    for (size_t e = 0; e < tab.size(); ++e)
        for (int r = 1; r < nrhs; ++r) {
            const size_t l = e * size_t(nrhs) + size_t(r);
            check(xcd_of[l] == xcd_of[l - 1] && pos_of[l] == pos_of[l - 1] + 1,
                  "right-hand sides of a band consecutive on one XCD", long(e), r);
        }
    if (whole)
        for (size_t e = 1; e < tab.size(); ++e)
            if (tab[e].q == tab[e - 1].q)
                check(xcd_of[e * size_t(nrhs)] == xcd_of[(e - 1) * size_t(nrhs)] &&
                          pos_of[e * size_t(nrhs)] == pos_of[(e - 1) * size_t(nrhs)] + nrhs,
                      "a system's bands consecutive on one XCD", long(tab[e].q), long(e));
    // balance: greedy largest-first assignment ends within one unit of the mean
    std::vector<double> load(size_t(nxcd), 0.0);
    double total = 0.0, largest = 0.0, unit = 0.0;
    for (size_t e = 0; e < tab.size(); ++e) {
        const double w = bf2_work(tab[e], g);
        load[size_t(xcd_of[e * size_t(nrhs)])] += w;
        total += w;
        unit = (whole && e > 0 && tab[e].q == tab[e - 1].q) ? unit + w : w;
        largest = std::max(largest, unit);
    }
    const double mean = total / nxcd;
    double worst = 0.0;
    for (double l : load)
        worst = std::max(worst, l);
    check(worst <= mean + largest * (1.0 + 1e-12), "per-XCD work within one unit of the mean", long(worst),
          long(mean + largest));
    return worst / mean;
}

int main()
{
    int nrhs = 0, cus = 0;
    std::cin >> nrhs >> cus;
    std::vector<BandGrid> g;
    BandGrid t{};
    while (std::cin >> t.nx >> t.ny >> t.nz)
        g.push_back(t);
    check(nrhs > 0 && cus > 0 && !g.empty(), "input");
    const std::vector<BF2Tile> whole = bf2_bands(g, 8, true, kBf2Threads, nrhs, cus);
    const std::vector<BF2Tile> shrt = bf2_bands_kz(g, 8, true, kBf2Threads, kBf2MinPlanes);
    check(!whole.empty() && !shrt.empty(), "tables built");
    if (fails)
        return 1;
    int kz = 0;
    for (const BF2Tile &b : whole)
        kz = std::max(kz, b.k1 - b.k0);
    // the rule: the longest candidate range giving kBf2BlocksPerCu per CU
    check(int64_t(whole.size()) * nrhs >= int64_t(kBf2BlocksPerCu) * cus || kz <= kBf2MinPlanes,
          "whole-batch table fills the chip or takes the shortest ranges", long(whole.size()), kz);
    check_table(whole, g, kBf2MaxPlanes);
    check_table(shrt, g, kBf2MinPlanes);
    const double b1 = check_map(bf2_dispatch(whole, g, nrhs, true, 8), whole, g, nrhs, true, 8);
    const double b2 = check_map(bf2_dispatch(shrt, g, nrhs, false, 8), shrt, g, nrhs, false, 8);
    check_map(bf2_dispatch(whole, g, nrhs, true, 1), whole, g, nrhs, true, 1);
    check_map(bf2_dispatch(shrt, g, nrhs, false, 3), shrt, g, nrhs, false, 3);
    std::printf("bands %zu short %zu longest_range %d balance_whole %.4f balance_short %.4f\n", whole.size(),
                shrt.size(), kz, b1, b2);
    return fails ? 1 : 0;
}
