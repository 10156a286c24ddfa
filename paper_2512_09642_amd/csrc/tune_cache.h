// On-disk cache of autotuned launch schedules (host code only, no HIP).
//
// The cache is a JSON object written one entry per line:
//   "key": {"nbg": 256, "slab": 0, "us": 507.3},
// Keys start with the schema tag kTuneSchema, so entries written by a
// library whose schedules meant something else are never looked up.  Every
// entry read back is range-checked by the caller's validator before use: a
// corrupt or foreign file can only cost a re-tune, never an out-of-range
// launch.
#pragma once

#include <cstdint>
#include <cstdio>
#include <fstream>
#include <map>
#include <string>

#include <unistd.h>

namespace sstep {

constexpr const char *kTuneSchema = "sstep-tune-v2";

struct TuneEntry {
    int nbg;       // Gram: partial blocks (stored AP) or block cap (operator-applying); batched: grid factor
    int64_t slab;  // Gram: 0 contiguous, > 0 rows per strided slab; batched: rows per chunk tile
    double us;     // measured time (0 = not measured)
};

inline std::map<std::string, TuneEntry> read_tune_cache(const std::string &path)
{
    std::map<std::string, TuneEntry> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"'), b = line.find("\": {");
        if (a == std::string::npos || b == std::string::npos || b <= a)
            continue;
        TuneEntry g{0, 0, 0.0};
        long long slab = 0;
        if (std::sscanf(line.c_str() + b, "\": {\"nbg\": %d, \"slab\": %lld, \"us\": %lf", &g.nbg, &slab, &g.us) ==
            3) {
            g.slab = slab;
            m[line.substr(a + 1, b - a - 1)] = g;
        }
    }
    return m;
}

inline void write_tune_cache(const std::string &path, const std::map<std::string, TuneEntry> &m)
{
    const std::string tmp = path + ".tmp" + std::to_string(::getpid());
    {
        std::ofstream f(tmp);
        if (!f)
            return;
        f << "{\n";
        size_t q = 0;
        for (const auto &kv : m) {
            f << "  \"" << kv.first << "\": {\"nbg\": " << kv.second.nbg << ", \"slab\": " << kv.second.slab
              << ", \"us\": " << kv.second.us << "}" << (++q < m.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path.c_str());
}

// A Gram schedule the kernels and the partial buffer (max_blocks slots per
// entry) can take: 1 <= nbg <= max_blocks, and either the contiguous schedule
// (slab 0) or slabs that are a positive multiple of pad rows, at most 2^24.
inline bool gram_entry_ok(const TuneEntry &g, int max_blocks, int64_t pad)
{
    if (g.nbg < 1 || g.nbg > max_blocks)
        return false;
    if (g.slab == 0)
        return true;
    return g.slab > 0 && g.slab % pad == 0 && g.slab <= (int64_t(1) << 24);
}

// A batched schedule the tile tables and partial buffers (sized for tiles of
// min_chunk rows) can take: grid factor in [1, 8], chunk a multiple of pad
// rows in [min_chunk, 2^24].
inline bool batched_entry_ok(const TuneEntry &g, int64_t pad, int64_t min_chunk)
{
    return g.nbg >= 1 && g.nbg <= 8 && g.slab >= min_chunk && g.slab % pad == 0 && g.slab <= (int64_t(1) << 24);
}

}  // namespace sstep
