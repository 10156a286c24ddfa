// Band tables and dispatch order of the batched two-step basis (host code,
// no HIP dependency: the set-up in api.cpp and a host test both use it).
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace sstep {

// Two basis steps per launch (recurrence and moments Gram kinds): a band of
// whole grid rows [y0, y1) of system q over the planes [k0, k1); the block
// also forms the first step on the row below and the row above the band.
struct BF2Tile {
    int32_t q, y0, y1, k0, k1, pad;
};
constexpr int kBf2Threads = 1024;    // threads per block of the two-step batched basis
constexpr int kBf2MaxPlanes = 128;   // longest z-range of one block
constexpr int kBf2MinPlanes = 16;    // shortest z-range (small batches, end of a solve)
constexpr int kBf2BlocksPerCu = 4;   // blocks per CU the longest ranges must still give
constexpr uint32_t kBf2NoBlock = 0xFFFFFFFFu;  // dispatch entry past an XCD's queue

// One system's grid for the band tables.
struct BandGrid {
    int64_t nx, ny, nz;
};

// Bands of the two-step batched basis: each system's rows split into bands
// of equal height (a band and its two neighbouring rows fill at most one
// block of nt threads; a grid whose planes fit in one block is one band),
// its planes into ranges of at most kzt, system by system, bands then
// ranges.  Empty when some system does not fit that shape (a row wider than
// a third of a block) or the windows of its buffer accesses (elem bytes per
// entry, face arrays included) would reach 1 GiB: the batch then takes one
// step per launch.
inline std::vector<BF2Tile> bf2_bands_kz(const std::vector<BandGrid> &grids, size_t elem, bool faces, int nt,
                                         int kzt)
{
    std::vector<BF2Tile> out;
    for (size_t q = 0; q < grids.size(); ++q) {
        const int64_t nx = grids[q].nx, ny = grids[q].ny, nz = grids[q].nz;
        const int64_t nxy = nx * ny;
        const int64_t lim = (int64_t(1) << 30) - 1;
        int64_t bytes = nxy * nz;
        if (faces)
            bytes = std::max({bytes, nz * ny * (nx + 1), nz * (ny + 1) * nx, (nz + 1) * nxy});
        if (bytes * int64_t(elem) > lim)
            return {};
        int64_t bands = 1;
        if (nxy > nt) {
            const int64_t inner = nt / nx - 2;  // band rows a block can hold
            if (inner < 1)
                return {};
            bands = (ny + inner - 1) / inner;
        }
        const int64_t h = (ny + bands - 1) / bands;
        const int64_t ranges = (nz + kzt - 1) / kzt;
        const int64_t kz = (nz + ranges - 1) / ranges;
        for (int64_t y0 = 0; y0 < ny; y0 += h)
            for (int64_t k0 = 0; k0 < nz; k0 += kz)
                out.push_back({int32_t(q), int32_t(y0), int32_t(std::min(y0 + h, ny)), int32_t(k0),
                               int32_t(std::min(k0 + kz, nz)), 0});
    }
    return out;
}

// The longest z-ranges (at most kBf2MaxPlanes planes) that still give every
// CU kBf2BlocksPerCu blocks, else ranges of kBf2MinPlanes: a long range
// re-reads fewer halo planes and starts fewer blocks (the batched workload:
// 2.10 s with whole-system ranges of up to 96 planes against 2.30 s with
// 16), a short one keeps small batches spread over the chip.
inline std::vector<BF2Tile> bf2_bands(const std::vector<BandGrid> &grids, size_t elem, bool faces, int nt, int nrhs,
                                      int cus)
{
    std::vector<BF2Tile> out;
    for (int kzt : {kBf2MaxPlanes, 96, 64, 48, 32, 24, kBf2MinPlanes}) {
        out = bf2_bands_kz(grids, elem, faces, nt, kzt);
        if (out.empty() || int64_t(out.size()) * nrhs >= int64_t(kBf2BlocksPerCu) * cus)
            break;
    }
    return out;
}

// Work of a band: its points with the ring rows and planes.
inline double bf2_work(const BF2Tile &t, const std::vector<BandGrid> &grids)
{
    return double(t.y1 - t.y0 + 2) * double(grids[size_t(t.q)].nx) * double(t.k1 - t.k0 + 2);
}

// The order the two-step basis's logical blocks (band e, right-hand side r:
// e * nrhs + r) run in.  Hardware block b runs on XCD b % nxcd, as the
// (b / nxcd)-th block that XCD starts, so map[b] lists each XCD's queue
// interleaved.  Units (whole systems, or single bands) go, largest first, to
// the XCD with the least work so far; a unit's blocks stay together in table
// order, so the right-hand sides of a band (and, for whole systems,
// neighbouring bands) share one L2.  Entries past an XCD's queue are
// kBf2NoBlock.
inline std::vector<uint32_t> bf2_dispatch(const std::vector<BF2Tile> &tab, const std::vector<BandGrid> &grids,
                                          int nrhs, bool whole_systems, int nxcd)
{
    struct Unit {
        double w;
        size_t e0, e1;
    };
    std::vector<Unit> units;
    for (size_t e = 0; e < tab.size();) {
        size_t f = e + 1;
        if (whole_systems)
            while (f < tab.size() && tab[f].q == tab[e].q)
                ++f;
        double w = 0.0;
        for (size_t k = e; k < f; ++k)
            w += bf2_work(tab[k], grids);
        units.push_back({w, e, f});
        e = f;
    }
    std::stable_sort(units.begin(), units.end(), [](const Unit &u, const Unit &v) { return u.w > v.w; });
    std::vector<std::vector<uint32_t>> queue(static_cast<size_t>(nxcd));
    std::vector<double> load(size_t(nxcd), 0.0);
    for (const Unit &u : units) {
        size_t x = 0;
        for (size_t k = 1; k < size_t(nxcd); ++k)
            if (load[k] < load[x])
                x = k;
        load[x] += u.w;
        for (size_t e = u.e0; e < u.e1; ++e)
            for (int r = 0; r < nrhs; ++r)
                queue[x].push_back(uint32_t(e * size_t(nrhs) + size_t(r)));
    }
    size_t len = 0;
    for (const auto &v : queue)
        len = std::max(len, v.size());
    std::vector<uint32_t> map(len * size_t(nxcd), kBf2NoBlock);
    for (size_t x = 0; x < size_t(nxcd); ++x)
        for (size_t k = 0; k < queue[x].size(); ++k)
            map[k * size_t(nxcd) + x] = queue[x][k];
    return map;
}

}  // namespace sstep
