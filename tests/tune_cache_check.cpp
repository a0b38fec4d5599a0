// Host-only driver for the tuning-cache reader and writer (built with g++ by
// test_tune_cache.py; no GPU code involved).
//   key ARCH CUS MIXED KC N S         print the cache key
//   load PATH                         print "ok <n>" and one line per entry, or "bad"
//   put PATH KEY RE DR RC TI FR FM BF MS  add an entry if the file is readable: "stored" / "refused"
#include <cstdio>
#include <cstdlib>
#include <string>

#include "../paper_1702_02939_amd/csrc/spv_tune.hpp"

int main(int argc, char** argv)
{
    if (argc < 2) return 2;
    const std::string cmd = argv[1];
    if (cmd == "key" && argc == 8) {
        std::printf("%s\n", spv::tune_key(argv[2], std::atoi(argv[3]), std::atoi(argv[4]) != 0, std::atoi(argv[5]),
                                          std::atoll(argv[6]), std::atoi(argv[7]))
                                .c_str());
        return 0;
    }
    if (cmd == "load" && argc == 3) {
        std::map<std::string, spv::TuneEntry> m;
        if (spv::cache_load(argv[2], m) != 0) {
            std::printf("bad\n");
            return 0;
        }
        std::printf("ok %zu\n", m.size());
        for (const auto& kv : m)
            std::printf("%s %d %d %d %d %d %d %.17g %.17g\n", kv.first.c_str(), kv.second.k.resort_every,
                        kv.second.k.device_rounds, kv.second.k.repair_cells, kv.second.k.tail_items,
                        kv.second.k.full_rounds, kv.second.k.force_mode, kv.second.k.bin_factor,
                        kv.second.ms_per_step);
        return 0;
    }
    if (cmd == "put" && argc == 12) {
        std::map<std::string, spv::TuneEntry> m;
        if (spv::cache_load(argv[2], m) != 0) {
            std::printf("refused\n");
            return 0;
        }
        spv::TuneEntry e;
        e.k.resort_every = std::atoi(argv[4]);
        e.k.device_rounds = std::atoi(argv[5]);
        e.k.repair_cells = std::atoi(argv[6]);
        e.k.tail_items = std::atoi(argv[7]);
        e.k.full_rounds = std::atoi(argv[8]);
        e.k.force_mode = std::atoi(argv[9]);
        e.k.bin_factor = std::atof(argv[10]);
        e.ms_per_step = std::atof(argv[11]);
        m[argv[3]] = e;
        std::printf(spv::cache_store(argv[2], m) ? "stored\n" : "failed\n");
        return 0;
    }
    return 2;
}
