// Host-only check of the autotuner cache: parsing, schema-tagged keys and the
// range checks applied before a cached schedule is used.  Built with g++ by
// tests/test_tune_cache.py; prints one line per check and exits non-zero on
// the first failure.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>

#include "tune_cache.h"

using namespace sstep;

static int fails = 0;
static void check(bool ok, const char *what)
{
    std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
    if (!ok)
        ++fails;
}

int main(int argc, char **argv)
{
    if (argc < 2)
        return 2;
    const std::string path = argv[1];
    {
        std::ofstream f(path);
        f << "{\n"
          << "  \"good\": {\"nbg\": 256, \"slab\": 0, \"us\": 12.5},\n"
          << "  \"too many blocks\": {\"nbg\": 100000, \"slab\": 0, \"us\": 1},\n"
          << "  \"zero blocks\": {\"nbg\": 0, \"slab\": 0, \"us\": 1},\n"
          << "  \"negative slab\": {\"nbg\": 256, \"slab\": -2048, \"us\": 1},\n"
          << "  \"ragged slab\": {\"nbg\": 256, \"slab\": 1000, \"us\": 1},\n"
          << "  \"truncated\": {\"nbg\": 256, \"sl\n"
          << "  garbage line without a key\n"
          << "  \"batched ok\": {\"nbg\": 4, \"slab\": 8192, \"us\": 3},\n"
          << "  \"batched chunk 0\": {\"nbg\": 4, \"slab\": 0, \"us\": 3},\n"
          << "  \"batched small chunk\": {\"nbg\": 4, \"slab\": 1024, \"us\": 3},\n"
          << "  \"batched factor 0\": {\"nbg\": 0, \"slab\": 8192, \"us\": 3},\n"
          << "  \"batched factor 99\": {\"nbg\": 99, \"slab\": 8192, \"us\": 3}\n"
          << "}\n";
    }
    auto m = read_tune_cache(path);
    check(m.size() == 10, "ten well-formed entries parsed, truncated and garbage lines skipped");
    check(m.count("truncated") == 0, "truncated entry dropped");
    check(m["good"].nbg == 256 && m["good"].slab == 0 && m["good"].us == 12.5, "values read back");
    const int maxb = 2048;
    const int64_t pad = 256;
    check(gram_entry_ok(m["good"], maxb, pad), "valid Gram entry accepted");
    check(!gram_entry_ok(m["too many blocks"], maxb, pad), "block count above the partial buffer rejected");
    check(!gram_entry_ok(m["zero blocks"], maxb, pad), "zero blocks rejected");
    check(!gram_entry_ok(m["negative slab"], maxb, pad), "negative slab rejected");
    check(!gram_entry_ok(m["ragged slab"], maxb, pad), "slab not a multiple of the padding rejected");
    check(gram_entry_ok(TuneEntry{512, 2048, 0.0}, maxb, pad), "strided schedule accepted");
    const int64_t minc = 2048;
    check(batched_entry_ok(m["batched ok"], pad, minc), "valid batched entry accepted");
    check(!batched_entry_ok(m["batched chunk 0"], pad, minc), "batched chunk 0 rejected (no division by zero)");
    check(!batched_entry_ok(m["batched small chunk"], pad, minc), "batched chunk below the table sizing rejected");
    check(!batched_entry_ok(m["batched factor 0"], pad, minc), "batched grid factor 0 rejected");
    check(!batched_entry_ok(m["batched factor 99"], pad, minc), "batched grid factor above 8 rejected");
    // round trip through the writer
    m.erase("truncated");
    write_tune_cache(path, m);
    auto m2 = read_tune_cache(path);
    check(m2.size() == m.size() && m2["batched ok"].slab == 8192, "write/read round trip");
    check(std::string(kTuneSchema).rfind("sstep-tune-v", 0) == 0, "keys carry a schema tag");
    auto missing = read_tune_cache(path + ".does-not-exist");
    check(missing.empty(), "missing file reads as empty");
    return fails ? 1 : 0;
}
