// qf_tune.hip -- autotuner of a filter set's launch parameters.
//
// The parameters (region size of the merge, tile and chunk of the radix sort,
// keys per lane of the lookups) only decide how the work is cut into
// work-groups; the results are the same for every choice.  The best choice
// depends on the mix of filter sizes (small filters have few regions, so
// smaller regions give the merge more work-groups), on the batch size (sort
// grid) and on the lookup batch (latency hiding), so it is measured: private
// filters of a sample of the requested sizes are filled and queried with
// synthetic keys under each candidate, one parameter at a time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "qf.h"
#include "qf_dev.h"
#include "qf_lib.h"

namespace {

constexpr uint64_t SAMPLE_SLOTS = 1ull << 26;  // quotients of the sample, at most

// a SplitMix64 stream on the host (synthetic keys for timing only)
uint64_t stream_key(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebull;
  z ^= z >> 31;
  return z;
}

struct Cached {
  qf_tuning_t t;
  double ms[2];
};
std::mutex g_mu;
std::map<std::vector<uint64_t>, Cached> g_cache;

// Everything one tuning run allocates; released by the destructor.
struct Bench {
  std::vector<qf_t *> fs;
  qf_set_t *set = nullptr;
  uint64_t *d_keys = nullptr, *d_qkeys = nullptr;
  uint32_t *d_fid = nullptr, *d_qfid = nullptr;
  uint8_t *d_out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  uint64_t n = 0, nq = 0;
  ~Bench() {
    (void)hipDeviceSynchronize();
    qf_set_destroy(set);
    for (qf_t *f : fs) qf_destroy(f);
    (void)hipFree(d_keys);
    (void)hipFree(d_qkeys);
    (void)hipFree(d_fid);
    (void)hipFree(d_qfid);
    (void)hipFree(d_out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  // every filter back to empty (both copies and the state words)
  bool reset() {
    for (qf_t *f : fs) {
      for (int c = 0; c < 2; ++c)
        if (hipMemsetAsync(f->blk[c], 0, f->nblocks * f->block_bytes, nullptr) != hipSuccess) return false;
      if (hipMemsetAsync(f->state, 0, qf::ST_WORDS * sizeof(uint64_t), nullptr) != hipSuccess) return false;
    }
    return hipDeviceSynchronize() == hipSuccess;
  }
  // milliseconds of one set insert of the fill batch into empty filters,
  // best of two runs; < 0 on failure
  double insert_ms() {
    double best = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
      if (!reset()) return -1;
      (void)hipEventRecord(e0, nullptr);
      if (qf_set_insert_batch(set, d_fid, d_keys, n, nullptr) != QF_OK) return -1;
      (void)hipEventRecord(e1, nullptr);
      if (hipEventSynchronize(e1) != hipSuccess) return -1;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (qf_set_sync(set, nullptr) != QF_OK) return -1;
      best = std::min(best, static_cast<double>(ms));
    }
    return best;
  }
  // milliseconds of one set query batch on the filled filters, best of three
  double query_ms() {
    double best = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(e0, nullptr);
      if (qf_set_query_batch(set, d_qfid, d_qkeys, nq, d_out, nullptr) != QF_OK) return -1;
      (void)hipEventRecord(e1, nullptr);
      if (hipEventSynchronize(e1) != hipSuccess) return -1;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, static_cast<double>(ms));
    }
    return best;
  }
};

// A candidate replaces the one in hand only when it is faster by more than
// this fraction: the defaults are measured first, and differences within
// run-to-run noise no longer move the pick.
constexpr double MARGIN = 0.03;

int tune(const uint32_t *qs, uint32_t nf, uint32_t r, double load, uint64_t n_query, qf_tuning_t *best,
         double *ms_out) {
  // the sample: every k-th filter, at most SAMPLE_SLOTS quotients in total
  uint64_t total = 0;
  for (uint32_t i = 0; i < nf; ++i) total += 1ull << qs[i];
  const uint64_t k = std::max<uint64_t>(1, (total + SAMPLE_SLOTS - 1) / SAMPLE_SLOTS);
  std::vector<uint32_t> sq;
  uint64_t stotal = 0;
  for (uint32_t i = 0; i < nf; i += static_cast<uint32_t>(k)) {
    sq.push_back(qs[i]);
    stotal += 1ull << qs[i];
  }
  Bench b;
  for (uint32_t q : sq) {
    qf_t *f = qf_create(q, r);
    if (!f) return qf_last_error();
    b.fs.push_back(f);
  }
  // the fill batch: floor(load 2^q) keys per filter
  std::vector<uint64_t> keys;
  std::vector<uint32_t> fid;
  std::vector<uint64_t> start(sq.size() + 1, 0);
  for (size_t j = 0; j < sq.size(); ++j) {
    const uint64_t nj = static_cast<uint64_t>(std::floor(load * static_cast<double>(1ull << sq[j])));
    for (uint64_t i = 0; i < nj; ++i) {
      keys.push_back(stream_key(0x51ED + j, i));
      fid.push_back(static_cast<uint32_t>(j));
    }
    start[j + 1] = keys.size();
  }
  b.n = keys.size();
  // the query batch, scaled to the sample: filters in proportion to 2^q,
  // even positions a key inserted into that filter, odd ones a fresh key
  b.nq = std::max<uint64_t>(1ull << 16, static_cast<uint64_t>(static_cast<double>(n_query) *
                                                             static_cast<double>(stotal) /
                                                             static_cast<double>(total)));
  std::vector<uint64_t> qkeys(b.nq);
  std::vector<uint32_t> qfid(b.nq);
  std::vector<uint64_t> cum(sq.size());
  uint64_t acc = 0;
  for (size_t j = 0; j < sq.size(); ++j) cum[j] = (acc += 1ull << sq[j]);
  for (uint64_t i = 0; i < b.nq; ++i) {
    const uint64_t u = stream_key(0x7E57, i) % acc;
    const size_t j = static_cast<size_t>(std::upper_bound(cum.begin(), cum.end(), u) - cum.begin());
    qfid[i] = static_cast<uint32_t>(j);
    const uint64_t nj = start[j + 1] - start[j];
    if ((i & 1) == 0 && nj > 0)
      qkeys[i] = keys[start[j] + stream_key(0xA11, i) % nj];
    else
      qkeys[i] = stream_key(0xAB5E47, i);
  }
  if (b.n == 0) return QF_ERR_ARG;
  if (hipMalloc(&b.d_keys, b.n * 8) != hipSuccess || hipMalloc(&b.d_fid, b.n * 4) != hipSuccess ||
      hipMalloc(&b.d_qkeys, b.nq * 8) != hipSuccess || hipMalloc(&b.d_qfid, b.nq * 4) != hipSuccess ||
      hipMalloc(&b.d_out, b.nq) != hipSuccess)
    return QF_ERR_OOM;
  if (hipMemcpy(b.d_keys, keys.data(), b.n * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b.d_fid, fid.data(), b.n * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b.d_qkeys, qkeys.data(), b.nq * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b.d_qfid, qfid.data(), b.nq * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreate(&b.e0) != hipSuccess || hipEventCreate(&b.e1) != hipSuccess)
    return QF_ERR_DEVICE;
  b.set = qf_set_create(b.fs.data(), static_cast<uint32_t>(b.fs.size()));
  if (!b.set) return qf_last_error();
  int rc = qf_set_reserve(b.set, b.n, nullptr);
  if (rc) return rc;

  qf_tuning_t cur{0, 4096, 4096, 1};
  double best_ins = 1e30;
  // 1. region size
  const uint32_t rmax = static_cast<uint32_t>(qf::max_region_log2(r));
  qf_tuning_t pick = cur;
  for (uint32_t rl = rmax; rl + 3 >= rmax && rl >= 6; --rl) {
    qf_tuning_t t = cur;
    t.region_log2 = rl;
    if ((rc = qf_set_tune(b.set, &t)) != QF_OK) return rc;
    const double ms = b.insert_ms();
    if (ms < 0) return QF_ERR_DEVICE;
    if (ms < best_ins * (1.0 - MARGIN)) {
      best_ins = ms;
      pick = t;
    }
  }
  cur = pick;
  // 2. sort tile and chunk
  const uint32_t sorts[4][2] = {{4096, 4096}, {2048, 4096}, {4096, 16384}, {2048, 16384}};
  for (int c = 1; c < 4; ++c) {
    qf_tuning_t t = cur;
    t.sort_tile = sorts[c][0];
    t.sort_chunk = sorts[c][1];
    if ((rc = qf_set_tune(b.set, &t)) != QF_OK) return rc;
    const double ms = b.insert_ms();
    if (ms < 0) return QF_ERR_DEVICE;
    if (ms < best_ins * (1.0 - MARGIN)) {
      best_ins = ms;
      pick = t;
    }
  }
  cur = pick;
  // 3. keys per lane of the lookups, on the table the chosen insert built
  if ((rc = qf_set_tune(b.set, &cur)) != QF_OK) return rc;
  if (b.insert_ms() < 0) return QF_ERR_DEVICE;
  double best_q = 1e30;
  for (uint32_t kpl : {1u, 2u, 4u}) {
    qf_tuning_t t = cur;
    t.lookup_keys_per_lane = kpl;
    if ((rc = qf_set_tune(b.set, &t)) != QF_OK) return rc;
    const double ms = b.query_ms();
    if (ms < 0) return QF_ERR_DEVICE;
    if (ms < best_q * (1.0 - MARGIN)) {
      best_q = ms;
      pick = t;
    }
  }
  *best = pick;
  if (ms_out) {
    ms_out[0] = best_ins;
    ms_out[1] = best_q;
  }
  return QF_OK;
}

}  // namespace

extern "C" int qf_autotune_set(const uint32_t *qs, uint32_t nf, uint32_t r, double load, uint64_t n_query,
                               qf_tuning_t *best, double *ms) {
  if (!qs || nf == 0 || !best || (r != 8 && r != 16) || !(load > 0.0 && load < 1.0)) return QF_ERR_ARG;
  for (uint32_t i = 0; i < nf; ++i)
    if (qs[i] < 6 || qs[i] > QF_Q_MAX) return QF_ERR_ARG;
  std::vector<uint64_t> key{r, static_cast<uint64_t>(load * 1e9), n_query};
  key.insert(key.end(), qs, qs + nf);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      *best = it->second.t;
      if (ms) {
        ms[0] = it->second.ms[0];
        ms[1] = it->second.ms[1];
      }
      return QF_OK;
    }
  }
  double m[2] = {0, 0};
  const int rc = tune(qs, nf, r, load, n_query, best, m);
  if (rc != QF_OK) return rc;
  if (ms) {
    ms[0] = m[0];
    ms[1] = m[1];
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key] = Cached{*best, {m[0], m[1]}};
  return QF_OK;
}
