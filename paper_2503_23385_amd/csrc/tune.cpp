// Tuning table of the TSQR trees (see tune.h).
#include "tune.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

namespace figaro {
namespace {

struct Entry {
    TreeTune t;
    double ms;
};

using Key4 = std::tuple<int, int, int, int>;

std::mutex g_mu;
std::map<Key4, Entry> g_table;
bool g_loaded_env = false;
bool g_override_on = false;
TuneKey g_override_key;
TreeTune g_override;

Key4 key4(const TuneKey &k) { return std::make_tuple(k.acc_f64, k.np, k.batched, k.rows_log2); }

// FIGARO_TUNE_CACHE names a cache to merge in at first use.
void load_env_locked();

bool parse_int(const std::string &line, const char *name, int *out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    *out = std::atoi(line.c_str() + p + pat.size());
    return true;
}

bool parse_double(const std::string &line, const char *name, double *out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    *out = std::atof(line.c_str() + p + pat.size());
    return true;
}

int load_locked(const std::string &path)
{
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return -1;
    char buf[512];
    int n = 0;
    while (std::fgets(buf, sizeof buf, f)) {
        const std::string line(buf);
        if (line.find("\"gfx950\"") == std::string::npos) continue;
        TuneKey k{};
        TreeTune t{};
        double ms = 0.0;
        if (!parse_int(line, "acc_f64", &k.acc_f64) || !parse_int(line, "np", &k.np) ||
            !parse_int(line, "batched", &k.batched) || !parse_int(line, "rows_log2", &k.rows_log2) ||
            !parse_int(line, "kind", &t.kind) || !parse_int(line, "leaf_blocks", &t.leaf_blocks) ||
            !parse_int(line, "arity", &t.arity))
            continue;
        parse_double(line, "ms", &ms);
        if ((t.kind != TREE_WG && t.kind != TREE_WAVE) || t.leaf_blocks < 0 || t.leaf_blocks > 1024 || t.arity < 2 ||
            t.arity > 32 || k.acc_f64 < 0 || k.acc_f64 > TUNE_PLAN)
            continue;
        g_table[key4(k)] = Entry{t, ms};
        n++;
    }
    std::fclose(f);
    return n;
}

void load_env_locked()
{
    if (g_loaded_env) return;
    g_loaded_env = true;
    const char *p = std::getenv("FIGARO_TUNE_CACHE");
    if (p && *p) (void)load_locked(p);
}

}  // namespace

int rows_log2(int64_t rows)
{
    int l = 0;
    while (l < 62 && ((int64_t)1 << l) < rows) l++;
    return l;
}

TreeTune tune_default(const TuneKey &k)
{
    if (k.acc_f64 == TUNE_SIGMA) return TreeTune{SIGMA_MSECT, 0, 2};
    if (k.acc_f64 == TUNE_PLAN) return TreeTune{0, 0, 2};  // chains one after the other
    if (k.np > 64) return TreeTune{TREE_WG, 0, 2};  // width 128: the panel tree
    if (k.batched) {
        // measured on the 256-instance batch (all widths in one launch): 16 blocks per leaf
        // at padded width 64, 64 at 32, 32 at 16 and 64 below; trees of arity 4 (a binary
        // climb over short leaves costs more node stores and loads than its shorter merges
        // save)
        const int b = k.np >= 64 ? 16 : (k.np == 32 ? 64 : (k.np == 16 ? 32 : 64));
        return TreeTune{TREE_WAVE, b, 4};
    }
    return TreeTune{TREE_WG, 0, 0};
}

std::vector<TreeTune> tune_candidates(const TuneKey &k)
{
    std::vector<TreeTune> c;
    if (k.acc_f64 == TUNE_SIGMA) {
        c.push_back(TreeTune{SIGMA_MSECT, 0, 2});
        c.push_back(TreeTune{SIGMA_DQDS, 0, 2});
        return c;
    }
    if (k.np > 64) {
        // width 128: the panel tree (the workgroup kernel of this width) or one wave per leaf
        c.push_back(TreeTune{TREE_WG, 0, 2});
        for (int b : {4, 8, 16, 32})
            for (int a : {2, 4}) c.push_back(TreeTune{TREE_WAVE, b, a});
        return c;
    }
    if (k.batched) {
        for (int b : {4, 8, 16, 32, 64})
            for (int a : {2, 4, 8}) c.push_back(TreeTune{TREE_WAVE, b, a});
    } else {
        for (int b : {0, 2, 4, 8}) c.push_back(TreeTune{TREE_WG, b, 0});
        for (int b : {8, 16, 32})
            for (int a : {2, 4}) c.push_back(TreeTune{TREE_WAVE, b, a});
    }
    return c;
}

TreeTune tune_get(const TuneKey &k)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    if (g_override_on && g_override_key.acc_f64 == k.acc_f64 && g_override_key.np == k.np &&
        g_override_key.batched == k.batched)
        return g_override;
    auto it = g_table.find(key4(k));
    if (it != g_table.end()) return it->second.t;
    // nearest tuned row count (within a factor of 4) of the same family
    const Entry *best = nullptr;
    int bd = 3;
    for (auto &kv : g_table) {
        if (std::get<0>(kv.first) != k.acc_f64 || std::get<1>(kv.first) != k.np || std::get<2>(kv.first) != k.batched)
            continue;
        const int d = std::abs(std::get<3>(kv.first) - k.rows_log2);
        if (d < bd) {
            bd = d;
            best = &kv.second;
        }
    }
    return best ? best->t : tune_default(k);
}

void tune_set(const TuneKey &k, const TreeTune &t, double ms)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[key4(k)] = Entry{t, ms};
}

void tune_override(const TuneKey *k, const TreeTune *t)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_override_on = k != nullptr && t != nullptr;
    if (g_override_on) {
        g_override_key = *k;
        g_override = *t;
    }
}

int tune_load(const std::string &path)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    return load_locked(path);
}

std::string tune_dump()
{
    std::lock_guard<std::mutex> lk(g_mu);
    std::ostringstream o;
    for (auto &kv : g_table) {
        const TreeTune &t = kv.second.t;
        o << "{\"arch\":\"gfx950\",\"acc_f64\":" << std::get<0>(kv.first) << ",\"np\":" << std::get<1>(kv.first)
          << ",\"batched\":" << std::get<2>(kv.first) << ",\"rows_log2\":" << std::get<3>(kv.first)
          << ",\"kind\":" << t.kind << ",\"leaf_blocks\":" << t.leaf_blocks << ",\"arity\":" << t.arity
          << ",\"ms\":" << kv.second.ms << "}\n";
    }
    return o.str();
}

int tune_save(const std::string &path)
{
    const std::string s = tune_dump();
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return -1;
    const size_t w = std::fwrite(s.data(), 1, s.size(), f);
    std::fclose(f);
    if (w != s.size()) return -1;
    return std::rename(tmp.c_str(), path.c_str()) == 0 ? 0 : -1;
}

}  // namespace figaro
