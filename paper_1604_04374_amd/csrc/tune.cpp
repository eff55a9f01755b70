// Tuning table: measured per-length variant choices for given workloads
// (written by the package's tuner, loaded through pc_tune_set), and the
// workload keys they are filed under.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/pc.h"
#include "pc_internal.hpp"

namespace pc {
namespace {
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

// FNV-1a over 64-bit words
uint64_t mix(uint64_t h, uint64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (v >> (8 * i)) & 0xffu;
    h *= 0x100000001b3ull;
  }
  return h;
}
constexpr uint64_t FNV0 = 0xcbf29ce484222325ull;
// plan description fields that decide the launches (not the window values)
uint64_t desc_words(uint64_t h, const pc_plan_desc& d) {
  h = mix(h, (uint64_t)d.ndim);
  h = mix(h, (uint64_t)d.m);
  h = mix(h, (uint64_t)d.n0);
  h = mix(h, (uint64_t)d.n1);
  h = mix(h, (uint64_t)d.batch);
  h = mix(h, (uint64_t)d.w_format);
  h = mix(h, (uint64_t)d.m_rows);
  h = mix(h, (uint64_t)d.m_cols);
  return mix(h, (uint64_t)d.flags);
}
}  // namespace

void tune_set(const std::vector<TuneEntry>& entries) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune = entries;
}

int tune_get(uint64_t key, int knob, int length, int rule) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const TuneEntry& e : g_tune)
    if (e.key == key && e.knob == knob && e.length == length) return e.value;
  return rule;
}

uint64_t tune_key(const pc_plan_desc& d) { return desc_words(FNV0, d); }

uint64_t tune_batch_key(const std::vector<pc_plan_desc>& ds) {
  // order-free: the sorted keys of the plans, then their count
  std::vector<uint64_t> ks;
  for (const pc_plan_desc& d : ds) ks.push_back(desc_words(FNV0, d));
  std::sort(ks.begin(), ks.end());
  uint64_t h = mix(FNV0, 0x62617463ull);  // domain separation from plan keys
  for (uint64_t k : ks) h = mix(h, k);
  return mix(h, (uint64_t)ks.size());
}

}  // namespace pc
