// Tuning table lookup and storage (tuning_cache.cpp): keys, candidate lists, the user cache and
// the LTL_TILE override. Host-only.
#pragma once
#include <string>
#include <vector>

#include "ltl.h"

namespace ltl {
namespace host {

struct TuneKey {
    std::string method, elem, epi;   // "cat_i8"..., "i8"/"i8w"/"i8x"/"f16"/"f8"/"direct", "byte"/"win"/"half"/"decay"/"mixed"
    int r = 0;                       // radius (0 for a batch)
    int bucket = 0;                  // round(log2(sqrt(cells)))
    std::string boundary;            // "dead" / "periodic"
    int batched = 0;
};

int size_bucket(double cells);
TuneKey make_key(int H, int W, const ltl_rule_t &rule, int method, int boundary, int batched);
// Table entries of the key's class, nearest radius first, then nearest size bucket (user cache
// before the shipped table on ties). *exact: the first candidate has the key's r and bucket.
std::vector<ltl_tuning_t> tuning_candidates(const TuneKey &key, bool *exact);
// Insert or replace the key's entry in the user cache.
bool store_tuning(const TuneKey &key, const ltl_tuning_t &t, double ms_per_step, std::string *err);
// LTL_TILE override: 0 if unset, 1 with *t filled, -1 if malformed (message in *err).
int env_tile(ltl_tuning_t *t, std::string *err);
std::string user_cache_path();
std::string shipped_table_path();

}  // namespace host
}  // namespace ltl
