// Autotuning table of the product kernel and the batched kernel's tile: the
// host-side state behind sincosm_tune_* (the kernels and their configuration
// list live with the product kernel).
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace sc {
namespace {

// Tuning table: for (arith, launch class, padded order in [lo, hi]) use
// configuration idx. Launch classes:
//   0  one problem with at most one k-segment (a plain product);
//   1  several problems with equal k-work (the double-angle steps);
//   2  the rest: problems of unequal k-work, or one problem with several
//      k-segments (the reverse pass). A tile that is a good choice for two
//      equal problems can leave CUs idle here, so this class is tuned on its
//      own and falls back to the single-product entries.
// Classes 1 and 2 use class 0 entries when none of their own matches.
// Class 3 holds the batched kernel's product mode per padded order instead of
// a configuration of the product kernel (0: 64 x 64 output tiles, the
// default; 1: 32 x 32; 2: the LDS-resident kernel, padded orders up to 32 in
// float64 and 64 in float32 only, 64 x 64 above).
struct TuneEntry { int ar; int cls; int64_t lo, hi; int idx; };
std::mutex tune_mu;
std::vector<TuneEntry> tune_table;

constexpr int TUNE_FLAGS = SINCOSM_TUNE_MULTI | SINCOSM_TUNE_UNEVEN | SINCOSM_TUNE_BATCHED;
constexpr int BATCHED_CLASS = 3;
// Output tiles of the batched kernel, by configuration index (0: the whole
// matrix in LDS).
const int kBatchedTile[] = {64, 32, 0};
// Largest padded order the LDS-resident kernel holds: nine matrices of order
// + 1 row stride in 160 KB of LDS.
inline int lds_max_order(int ar) { return ar == (int)Arith::F64 ? 32 : 64; }

}  // namespace

int tuned_cfg(Arith ar, int cls, int64_t np) {
  std::lock_guard<std::mutex> g(tune_mu);
  const int order[2] = {cls, 0};
  const bool fallback = cls == 1 || cls == 2;   // the batched tile table has none
  for (int k = 0; k < (fallback ? 2 : 1); ++k)
    for (auto it = tune_table.rbegin(); it != tune_table.rend(); ++it)
      if (it->ar == (int)ar && it->cls == order[k] && np >= it->lo && np <= it->hi) return it->idx;
  return -1;
}

int batched_tile(Arith ar, int64_t np) {
  const int idx = tuned_cfg(ar, BATCHED_CLASS, np);
  const int count = (int)(sizeof(kBatchedTile) / sizeof(kBatchedTile[0]));
  if (idx < 0 || idx >= count) return 64;
  if (kBatchedTile[idx] == 0 && np > lds_max_order((int)ar)) return 64;
  return kBatchedTile[idx];
}

}  // namespace sc

extern "C" {

int sincosm_tune_num_configs(int arith) {
  int count = 0;
  sc::cfg_table((sc::Arith)(arith & ~sc::TUNE_FLAGS), count);
  if (count && (arith & SINCOSM_TUNE_BATCHED)) return (int)(sizeof(sc::kBatchedTile) / sizeof(int));
  return count;
}

sincosm_status sincosm_tune_config_info(int arith, int idx, int32_t* info) {
  int count = 0;
  const sc::KernelCfg* t = sc::cfg_table((sc::Arith)(arith & ~sc::TUNE_FLAGS), count);
  if (t && info && (arith & SINCOSM_TUNE_BATCHED)) {
    if (idx < 0 || idx >= sincosm_tune_num_configs(arith)) return SINCOSM_E_ARG;
    const int tb = sc::kBatchedTile[idx];   // four waves of tb/2 x tb/2, k depth 16, staged
    if (tb == 0) {
      // LDS-resident: one wave per 16 x 16 block up to the largest order it
      // holds (32 in float64, 64 in float32), k depth 4; "direct" = 2 marks
      // the mode, the wave grid is that of the largest order
      const int mo = sc::lds_max_order(arith & ~sc::TUNE_FLAGS);
      info[0] = mo; info[1] = mo; info[2] = 4; info[3] = mo / 16; info[4] = mo / 16;
      info[5] = mo / 16 == 2 ? 2 : 4; info[6] = 2; info[7] = 1;
      return SINCOSM_OK;
    }
    info[0] = tb; info[1] = tb; info[2] = 16; info[3] = 2; info[4] = 2; info[5] = 3;
    info[6] = 0; info[7] = 1;
    return SINCOSM_OK;
  }
  if (!t || !info || idx < 0 || idx >= count) return SINCOSM_E_ARG;
  info[0] = t[idx].bm; info[1] = t[idx].bn; info[2] = t[idx].bk;
  info[3] = t[idx].wgm; info[4] = t[idx].wgn; info[5] = t[idx].wpe; info[6] = t[idx].dl;
  info[7] = t[idx].ks;
  return SINCOSM_OK;
}

sincosm_status sincosm_tune_set(int arith, int64_t np_lo, int64_t np_hi, int idx) {
  const int flags = arith & sc::TUNE_FLAGS;
  if (flags & (flags - 1)) return SINCOSM_E_ARG;   // at most one table flag
  const int cls = (arith & SINCOSM_TUNE_BATCHED)  ? sc::BATCHED_CLASS
                  : (arith & SINCOSM_TUNE_UNEVEN) ? 2
                  : (arith & SINCOSM_TUNE_MULTI)  ? 1 : 0;
  const int ar = arith & ~sc::TUNE_FLAGS;
  int count = sincosm_tune_num_configs(arith);
  if (count == 0 || np_lo > np_hi) return SINCOSM_E_ARG;
  std::lock_guard<std::mutex> g(sc::tune_mu);
  if (idx < 0) {   // clear entries of this arithmetic and class overlapping the range
    std::vector<sc::TuneEntry> keep;
    for (auto& e : sc::tune_table)
      if (!(e.ar == ar && e.cls == cls && e.hi >= np_lo && e.lo <= np_hi)) keep.push_back(e);
    sc::tune_table.swap(keep);
    return SINCOSM_OK;
  }
  if (idx >= count) return SINCOSM_E_ARG;
  // an entry for exactly the same range replaces the earlier one, so that
  // installing a cache again does not grow the table
  auto& tt = sc::tune_table;
  tt.erase(std::remove_if(tt.begin(), tt.end(),
                          [&](const sc::TuneEntry& e) {
                            return e.ar == ar && e.cls == cls && e.lo == np_lo && e.hi == np_hi;
                          }),
           tt.end());
  tt.push_back(sc::TuneEntry{ar, cls, np_lo, np_hi, idx});
  return SINCOSM_OK;
}

int sincosm_tune_lookup(int arith, int64_t np) {
  const int flags = arith & sc::TUNE_FLAGS;
  if (flags & (flags - 1)) return -1;
  const int cls = (arith & SINCOSM_TUNE_BATCHED)  ? sc::BATCHED_CLASS
                  : (arith & SINCOSM_TUNE_UNEVEN) ? 2
                  : (arith & SINCOSM_TUNE_MULTI)  ? 1 : 0;
  if (sincosm_tune_num_configs(arith) == 0) return -1;
  return sc::tuned_cfg((sc::Arith)(arith & ~sc::TUNE_FLAGS), cls, np);
}

}  // extern "C"
