// Tuning table of the TSQR trees: which tree kernel reduces a region and how long its
// leaves are, per (accumulation type, padded width, single call or batch, row count).
// Entries come from built-in defaults (measured on MI355X) or from the autotuner
// (figaro_plan_autotune / figaro_r_autotune), which times the candidates on the caller's
// own problem and can keep its choices in a JSON-lines cache file.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace figaro {

enum : int { TREE_WG = 0, TREE_WAVE = 1 };
// Entries with acc_f64 == TUNE_SIGMA hold the route of a plan's sigma width class np
// (kind SIGMA_MSECT or SIGMA_DQDS after the bidiagonalisation).
enum : int { TUNE_SIGMA = 2, SIGMA_MSECT = 0, SIGMA_DQDS = 1 };
// Entries with acc_f64 == TUNE_PLAN (np: 1 for plans accumulating in FP64, else 0;
// batched 1, rows_log2 0) hold how plans schedule their chains: kind 1 side by side on
// side streams, 0 one after the other.
enum : int { TUNE_PLAN = 3 };

struct TreeTune {
    int kind;         // TREE_WG: one workgroup per leaf; TREE_WAVE: one wave per leaf
    int leaf_blocks;  // blocks of rows per leaf (0: the workgroup tree's default leaf rule)
    int arity;        // tree arity (wave tree; the workgroup tree derives its own)
};

struct TuneKey {
    int acc_f64;    // FP64 accumulation (plain form) or FP32 (mixed forms)
    int np;         // padded width (4 .. 128; the class width for sigma entries)
    int batched;    // regions of a plan (1) or of a single call (0)
    int rows_log2;  // ceil(log2) of the rows the launch reduces
};

int rows_log2(int64_t rows);
// The tuned entry of the key (or of the nearest row count with the same acc/np/batched),
// else the default.  While an override is set (by the autotuner), it wins for its
// (acc, np, batched).
TreeTune tune_get(const TuneKey &k);
TreeTune tune_default(const TuneKey &k);
std::vector<TreeTune> tune_candidates(const TuneKey &k);
void tune_set(const TuneKey &k, const TreeTune &t, double ms);
void tune_override(const TuneKey *k, const TreeTune *t);  // nullptr: clear
// Cache file: one JSON object per line.  Load merges its entries into the table.
int tune_load(const std::string &path);
int tune_save(const std::string &path);
// The table as JSON lines (for reports).
std::string tune_dump();

}  // namespace figaro
