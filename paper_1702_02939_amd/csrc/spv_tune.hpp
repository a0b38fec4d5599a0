// spv_tune.hpp -- launch-configuration knobs and the autotuner's cache.
//
// The knobs change how the step is scheduled, never what it computes: cell
// order, bin sizes, the repair grid and the split of repair rounds between
// the device and the host all leave every ring, force and position bitwise
// unchanged (rings are canonical, forces are summed in ring order, the repair
// result is the unique Delaunay ring whatever the search radius).  They only
// move time, so the library may pick them by timing trial runs.
//
// Cache: a flat JSON object mapping a key (architecture, compute units,
// precision, ring capacity, power-of-two buckets of total cells and of
// systems) to the chosen knobs and the trial time per step, e.g.
//   {"gfx950/cu256/fp64/kc16/n2^17/s2^0": {"resort_every": 32,
//     "device_rounds": 8, "repair_cells": 64, "tail_items": 64,
//     "full_rounds": 1, "force_mode": 1, "bin_factor": 1.5, "ms_per_step": 0.081}}
// Reads accept only this shape; an unreadable file counts as empty and is
// never overwritten.
#pragma once
#include <cctype>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

namespace spv {

struct Knobs {
    int resort_every = 32;    // steps per re-sort period (even)
    int device_rounds = 2;    // repair rounds inside each step on the device
    int repair_cells = 64;    // flagged-cell capacity per repair wavefront: grid = N / this
    int tail_items = 64;      // largest late repair round finished on the device
    int full_rounds = 1;      // repair rounds over the whole grid before the tail
    int force_mode = 0;       // force kernel: 1 lanes per cell, 2 per (cell, slot) item, 0 by size
    double bin_factor = 1.0;  // bin side in mean cell spacings sqrt(L_x L_y / n)
};

struct TuneEntry {
    Knobs k;
    double ms_per_step = 0.0;
};

inline int log2_bucket(int64_t v)
{
    int b = 0;
    while (((int64_t)1 << b) < v) b++;
    return b;
}

inline std::string tune_key(const std::string& arch, int cus, bool mixed, int kc, int64_t N, int S)
{
    std::ostringstream o;
    o << arch << "/cu" << cus << "/" << (mixed ? "mixed" : "fp64") << "/kc" << kc << "/n2^" << log2_bucket(N)
      << "/s2^" << log2_bucket(S);
    return o.str();
}

// ---------------------------------------------------------------- JSON (flat, two levels)
class JsonReader {
   public:
    explicit JsonReader(const std::string& t) : s_(t) {}

    bool parse(std::map<std::string, TuneEntry>& out)
    {
        ws();
        if (!eat('{')) return false;
        ws();
        if (eat('}')) return end();
        while (true) {
            std::string key;
            if (!str(key)) return false;
            ws();
            if (!eat(':')) return false;
            TuneEntry e;
            if (!entry(e)) return false;
            out[key] = e;
            ws();
            if (eat(',')) {
                ws();
                continue;
            }
            if (eat('}')) return end();
            return false;
        }
    }

   private:
    const std::string s_;
    size_t i_ = 0;

    void ws()
    {
        while (i_ < s_.size() && std::isspace((unsigned char)s_[i_])) i_++;
    }
    bool eat(char c)
    {
        if (i_ < s_.size() && s_[i_] == c) {
            i_++;
            return true;
        }
        return false;
    }
    bool end()
    {
        ws();
        return i_ == s_.size();
    }
    bool str(std::string& out)
    {
        if (!eat('"')) return false;
        while (i_ < s_.size() && s_[i_] != '"') {
            if (s_[i_] == '\\' || (unsigned char)s_[i_] < 0x20) return false;  // keys never need escapes
            out.push_back(s_[i_++]);
        }
        return eat('"');
    }
    bool num(double& v)
    {
        const size_t b = i_;
        while (i_ < s_.size() && (std::isdigit((unsigned char)s_[i_]) || s_[i_] == '-' || s_[i_] == '+' ||
                                  s_[i_] == '.' || s_[i_] == 'e' || s_[i_] == 'E'))
            i_++;
        if (i_ == b) return false;
        const std::string t = s_.substr(b, i_ - b);
        char* e = nullptr;
        v = std::strtod(t.c_str(), &e);
        return e && *e == '\0' && std::isfinite(v);
    }
    bool entry(TuneEntry& e)
    {
        ws();
        if (!eat('{')) return false;
        int seen = 0;
        ws();
        while (!eat('}')) {
            std::string k;
            double v = 0.0;
            if (!str(k)) return false;
            ws();
            if (!eat(':')) return false;
            ws();
            if (!num(v)) return false;
            if (k == "resort_every") e.k.resort_every = (int)v, seen |= 1;
            else if (k == "device_rounds") e.k.device_rounds = (int)v, seen |= 2;
            else if (k == "repair_cells") e.k.repair_cells = (int)v, seen |= 4;
            else if (k == "bin_factor") e.k.bin_factor = v, seen |= 8;
            else if (k == "tail_items") e.k.tail_items = (int)v, seen |= 16;
            else if (k == "full_rounds") e.k.full_rounds = (int)v, seen |= 32;
            else if (k == "force_mode") e.k.force_mode = (int)v, seen |= 64;
            else if (k == "ms_per_step") e.ms_per_step = v;
            else return false;
            ws();
            if (eat(',')) {
                ws();
                continue;
            }
            if (!eat('}')) return false;
            break;
        }
        return seen == 127 && knobs_valid(e.k);
    }

   public:
    static bool knobs_valid(const Knobs& k)
    {
        return k.resort_every >= 2 && k.resort_every <= 4096 && k.device_rounds >= 1 && k.device_rounds <= 32 &&
               k.repair_cells >= 1 && k.repair_cells <= 1 << 20 && k.tail_items >= 1 && k.tail_items <= 1 << 20 &&
               k.full_rounds >= 1 && k.full_rounds <= 4 && k.force_mode >= 0 && k.force_mode <= 2 &&
               k.bin_factor >= 0.5 && k.bin_factor <= 8.0;
    }
};

// 0: loaded (or no file), -1: the file exists but is not a cache of this shape
inline int cache_load(const std::string& path, std::map<std::string, TuneEntry>& out)
{
    std::ifstream f(path);
    if (!f) return 0;
    std::stringstream b;
    b << f.rdbuf();
    std::map<std::string, TuneEntry> m;
    JsonReader r(b.str());
    if (!r.parse(m)) return -1;
    out.swap(m);
    return 0;
}

inline std::string cache_dump(const std::map<std::string, TuneEntry>& m)
{
    std::ostringstream o;
    o.precision(17);
    o << "{";
    bool first = true;
    for (const auto& kv : m) {
        o << (first ? "\n" : ",\n") << "  \"" << kv.first << "\": {\"resort_every\": " << kv.second.k.resort_every
          << ", \"device_rounds\": " << kv.second.k.device_rounds << ", \"repair_cells\": " << kv.second.k.repair_cells
          << ", \"tail_items\": " << kv.second.k.tail_items << ", \"full_rounds\": " << kv.second.k.full_rounds
          << ", \"force_mode\": " << kv.second.k.force_mode << ", \"bin_factor\": " << kv.second.k.bin_factor << ", \"ms_per_step\": " << kv.second.ms_per_step << "}";
        first = false;
    }
    o << "\n}\n";
    return o.str();
}

// write-then-rename, so a reader never sees half a file
inline bool cache_store(const std::string& path, const std::map<std::string, TuneEntry>& m)
{
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return false;
        f << cache_dump(m);
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace spv
