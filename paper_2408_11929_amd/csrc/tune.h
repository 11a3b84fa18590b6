// Autotuner of the sweep's segment plan (tune.cpp).
#pragma once

#include <tuple>

#include "hh_internal.h"

namespace hh {

// Shape of a sweep launch as the autotuner keys it.
struct TuneKey {
  int prec, KP, P, kmax, n, N, chains;  // chains: rounded up to a power of two
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, KP, P, kmax, n, N, chains) <
           std::tie(o.prec, o.KP, o.P, o.kmax, o.n, o.N, o.chains);
  }
};

// The choice kept for a shape (a segment plan 0, 1, 2, or HH_PLAN_TILE) and
// the measured launch time of each choice (milliseconds; 0 where it did not fit).
struct TuneEntry {
  int plan = 0;
  double ms[HH_NCHOICE] = {0, 0, 0, 0};
};

int tune_bucket(int chains);
bool tune_enabled();
void tune_set_enabled(bool on);
bool tune_lookup(const TuneKey& k, int& plan);
void tune_store(const TuneKey& k, const TuneEntry& e);
bool tune_save(const char* path);
bool tune_load(const char* path);
void tune_clear();
size_t tune_entries();

}  // namespace hh
