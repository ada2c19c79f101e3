// Tuning table: per scalar type and size class of the Gauss-Jordan boxes, the
// compact panel shape (width, rows per thread, threads) and the second-level block
// width. Filled by hss_tuning_set / hss_tuning_load (a JSON file written by the
// project's autotuner); empty entries keep the built-in rules.
#pragma once

#include <string>
#include <vector>

namespace hss {

struct TuneEntry {
  int nb = 0, rpt = 0, nt = 0;  // compact panel shape; nt = 0: the built-in rule
  int block = -1;               // second-level block width; -1: the built-in rule, 0: none
};

// size classes: boxes of at most kTuneClass[i] rows
constexpr int kTuneClasses = 6;
constexpr int kTuneClass[kTuneClasses] = {128, 256, 512, 1024, 2048, 4096};

// scalar: 0 float, 1 double, 2 complex float, 3 complex double
bool tuning_lookup(int scalar, int rows, TuneEntry& e);
void tuning_set(int scalar, int cls_rows, const TuneEntry& e);
void tuning_clear();
// reads the autotuner's JSON; returns the number of entries taken, throws Error on
// a malformed file
int tuning_load(const std::string& path);
// loads <directory of libhss.so>/tuning_gfx950.json (or $HSS_TUNING; empty: none)
// once per process, unless the table was already set, cleared or loaded by a call
void tuning_load_default();

}  // namespace hss
