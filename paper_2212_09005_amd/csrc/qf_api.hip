// qf_api.hip -- the C ABI declared in include/qf.h.
//
// A bulk update (Sec. 5.3-5.4, 6.4) enqueues, on the caller's stream:
//   hash -> radix sort of the fingerprints -> reduction to <fp, count> ->
//   region bounds (successor search) -> region merge into the other table copy.
// A bulk query / count (Sec. 6.2) enqueues one lookup kernel.
// Nothing waits for the device except qf_sync / qf_export / qf_import and the
// (rare) growth of the scratch area.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "qf.h"
#include "qf_dev.h"
#include "qf_lib.h"

// Batch scratch of qf_insert_batch_noalloc: batches of up to 2^19 keys, 64
// bytes per key (four uint64 arrays of the batch size, the merge's 32-byte
// per-entry area) plus the radix sort's counts (256 digit totals and 256
// counts per sort work-group of at least 4096 keys).  About 32 MiB per GPU.
constexpr uint64_t QF_NOALLOC_KEYS = 1ull << 19;
constexpr uint64_t QF_NOALLOC_HIST_WORDS = 256ull * (1 + (QF_NOALLOC_KEYS + 4095) / 4096);
constexpr uint64_t QF_NOALLOC_BYTES = 8 * QF_NOALLOC_KEYS * sizeof(uint64_t) + QF_NOALLOC_HIST_WORDS * sizeof(uint32_t);
static __device__ __align__(256) uint8_t scratch[QF_NOALLOC_BYTES];

namespace qf {
int max_region_log2(uint32_t r);
}

namespace {

thread_local int g_last_error = QF_OK;

int fail(int code) {
  g_last_error = code;
  return code;
}

#define QF_HIP(call)                                       \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return fail(QF_ERR_DEVICE);      \
  } while (0)

uint64_t isqrt_u64(uint64_t n) {
  uint64_t x = 0;
  for (uint64_t bit = 1ull << 62; bit; bit >>= 2) {
    if (n >= x + bit) {
      n -= x + bit;
      x = (x >> 1) + bit;
    } else {
      x >>= 1;
    }
  }
  return x;
}

// extra slots after slot 2^q - 1 where runs may still end (no wrap-around):
// 64 * ceil(10 * sqrt(2^q) / 64)
uint64_t extra_slots(uint32_t q) {
  const uint64_t e = 10ull * isqrt_u64(1ull << q);
  return (e + 63) / 64 * 64;
}

void free_scratch(qf::Pipe &p) {
  (void)hipFree(p.bufA);
  (void)hipFree(p.bufB);
  (void)hipFree(p.bufC);
  (void)hipFree(p.bufD);
  (void)hipFree(p.bufE);
  (void)hipFree(p.hist);
  p.bufA = p.bufB = p.bufC = p.bufD = p.bufE = nullptr;
  p.hist = nullptr;
  p.cap = 0;
  p.hist_words = 0;
}

int ensure_scratch(qf::Pipe &p, uint64_t n, hipStream_t s) {
  if (n <= p.cap) return QF_OK;
  uint64_t cap = 1ull << 16;
  while (cap < n) cap <<= 1;
  if (p.cap) QF_HIP(hipStreamSynchronize(s));
  p.device_bytes -= 8 * p.cap * sizeof(uint64_t) + p.hist_words * sizeof(uint32_t);
  free_scratch(p);
  const size_t bytes = cap * sizeof(uint64_t);
  const uint64_t hw = qf::sort_count_words(cap);
  if (hipMalloc(&p.bufA, bytes) != hipSuccess || hipMalloc(&p.bufB, bytes) != hipSuccess ||
      hipMalloc(&p.bufC, bytes) != hipSuccess || hipMalloc(&p.bufD, bytes) != hipSuccess ||
      hipMalloc(&p.bufE, 4 * bytes) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&p.hist), hw * sizeof(uint32_t)) != hipSuccess) {
    free_scratch(p);
    return fail(QF_ERR_OOM);
  }
  p.cap = cap;
  p.hist_words = hw;
  p.device_bytes += 8 * bytes + hw * sizeof(uint32_t);
  return QF_OK;
}

void pipe_free(qf::Pipe &p) {
  (void)hipFree(p.d_desc);
  (void)hipFree(p.d_rmap);
  (void)hipFree(p.rb);
  (void)hipFree(p.tags);
  (void)hipFree(p.pst);
  (void)hipFree(p.d_err);
  (void)hipFree(p.d_afil);
  (void)hipFree(p.d_areg);
  for (int i = 0; i < qf::Pipe::PIN_RING; ++i) {
    if (p.pin_ev[i]) (void)hipEventSynchronize(p.pin_ev[i]);
    (void)hipHostFree(p.h_pin[i]);
    if (p.pin_ev[i]) (void)hipEventDestroy(p.pin_ev[i]);
  }
  free_scratch(p);
  delete p.timer;
  p = qf::Pipe();
}

// region log2 of filter f in a pipeline that asks for `req` (0: the largest
// region the merge's LDS holds, and never more than the filter's quotients)
uint32_t rlog_for(const qf_filter *f, uint32_t req) {
  const uint32_t mx = std::min<uint32_t>(f->q, static_cast<uint32_t>(qf::max_region_log2(f->r)));
  return req == 0 ? mx : std::min(mx, std::max<uint32_t>(req, 6));
}

qf::FDesc desc_of(const qf_filter *f, uint32_t rbase, uint32_t rlog) {
  qf::FDesc d;
  std::memset(&d, 0, sizeof(d));
  d.blk[0] = f->blk[0];
  d.blk[1] = f->blk[1];
  d.state = f->state;
  d.N = static_cast<int64_t>(f->N);
  d.P = static_cast<int64_t>(f->P);
  d.nblocks = static_cast<int64_t>(f->nblocks);
  d.q = f->q;
  d.r = f->r;
  d.rlog = rlog;
  const uint64_t S = 1ull << rlog;
  d.nqregions = static_cast<uint32_t>(f->N / S);
  d.nregions = static_cast<uint32_t>((f->P + S - 1) / S);
  d.rbase = rbase;
  return d;
}

uint32_t bits_for(uint64_t v) {  // bits of the values 0..v
  uint32_t b = 0;
  while ((1ull << b) <= v) ++b;
  return b;
}

// The update pipeline of nf filters (same r): descriptors, region map, bounds,
// look-back words, statistics, old carries, histograms.  Synchronous.
int pipe_init(qf::Pipe &p, qf_filter *const *fs, uint32_t nf, const qf::Tune &tn) {
  p = qf::Pipe();
  p.tune = tn;
  p.nf = nf;
  p.r = fs[0]->r;
  (void)hipGetDevice(&p.device);
  std::vector<qf::FDesc> desc(nf);
  uint64_t G = 0;
  p.h_nreg.resize(nf);
  for (uint32_t i = 0; i < nf; ++i) {
    if (fs[i]->r != p.r) return fail(QF_ERR_ARG);
    const uint32_t rl = rlog_for(fs[i], tn.region_log2);
    p.RL = std::max(p.RL, rl);
    desc[i] = desc_of(fs[i], static_cast<uint32_t>(G), rl);
    p.h_nreg[i] = desc[i].nregions;
    G += desc[i].nregions;
    p.fin_slices = std::max(p.fin_slices, (desc[i].nregions + qf::FIN_REG - 1) / qf::FIN_REG);
  }
  if (G >= (1ull << 31)) return fail(QF_ERR_ARG);
  p.G = static_cast<uint32_t>(G);
  // region indices 0..G-1 stay below 2^gbits - 1, so no valid composite key
  // shares its sorted bits with the all-ones key of a dropped (bad index) key
  p.gbits = bits_for(G);
  if (nf > 1 && p.gbits + p.RL + p.r > 62) return fail(QF_ERR_ARG);
  std::vector<uint32_t> rmap(G);
  p.h_rbase.resize(nf);
  for (uint32_t i = 0; i < nf; ++i) {
    p.h_rbase[i] = desc[i].rbase;
    for (uint32_t k = 0; k < desc[i].nregions; ++k) rmap[desc[i].rbase + k] = i;
  }
  const uint64_t tag_words = 8ull * G + 8;        // 3 G tags, 4 G statistics, G carries
  bool ok = hipMalloc(reinterpret_cast<void **>(&p.d_desc), nf * sizeof(qf::FDesc)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void **>(&p.d_rmap), G * sizeof(uint32_t)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void **>(&p.rb), (G + 1) * sizeof(uint64_t)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void **>(&p.tags), tag_words * sizeof(uint64_t)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void **>(&p.pst), qf::ST_WORDS * sizeof(uint64_t)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void **>(&p.d_err), nf * sizeof(int64_t)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void **>(&p.d_afil), nf * sizeof(uint32_t)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void **>(&p.d_areg), G * sizeof(uint32_t)) == hipSuccess;
  ok = ok && hipMemcpy(p.d_desc, desc.data(), nf * sizeof(qf::FDesc), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(p.d_rmap, rmap.data(), G * sizeof(uint32_t), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(p.tags, 0, tag_words * sizeof(uint64_t)) == hipSuccess &&
       hipMemset(p.pst, 0, qf::ST_WORDS * sizeof(uint64_t)) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    pipe_free(p);
    return fail(QF_ERR_OOM);
  }
  p.one = desc[0];
  p.rstat = p.tags + ((3ull * G + 1) & ~1ull);  // 16-byte aligned (read as 16-byte vectors)
  p.cb = reinterpret_cast<int64_t *>(p.tags + 7ull * G + 2);
  p.device_bytes = nf * sizeof(qf::FDesc) + G * 4 + (G + 1) * 8 + tag_words * 8 + qf::ST_WORDS * 8;
  return QF_OK;
}

// true while `s` is being captured into a graph: nothing may allocate,
// synchronise or copy from pageable host memory then
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// hash -> radix sort -> reduction -> region bounds -> merge, on stream s.
// fid == nullptr: the pipeline has one filter and keys are its own.
// values != nullptr (one filter): value association, the fingerprints are
// the keys' q + r - vbits bit fingerprints followed by the values' low bits.
int pipe_update(qf::Pipe &p, const uint64_t *keys, const uint32_t *fid, uint64_t n, int del,
                uint64_t *not_found, hipStream_t s, uint32_t single_q, const qf_set *set = nullptr,
                const uint32_t *h_active = nullptr, uint32_t nactive = 0, const uint64_t *values = nullptr,
                uint32_t vbits = 0) {
  // under capture: scratch must be reserved, lists and timers are refused
  if (capturing(s) && (n > p.cap || h_active || p.timer)) return fail(QF_ERR_ARG);
  int rc = ensure_scratch(p, n, s);
  if (rc) return rc;
  // restrict the merge to the listed filters (their regions, in order); the
  // lists are copied from pageable host memory, which the runtime stages
  // before the call returns
  p.nafil = p.nareg = 0;
  if (set && h_active) {
    if (nactive == 0) return QF_OK;
    p.h_afil.assign(h_active, h_active + nactive);
    p.h_areg.clear();
    for (uint32_t k = 0; k < nactive; ++k) {
      const uint32_t f = h_active[k];
      if (f >= set->nf || (k && f <= h_active[k - 1])) return fail(QF_ERR_ARG);
      for (uint32_t R = 0; R < p.h_nreg[f]; ++R) p.h_areg.push_back(p.h_rbase[f] + R);
    }
    // both lists through the next pinned buffer (see Pipe::h_pin)
    const int i = p.pin_i;
    p.pin_i = (p.pin_i + 1) % qf::Pipe::PIN_RING;
    const uint64_t words = nactive + p.h_areg.size();
    if (p.pin_ev[i]) QF_HIP(hipEventSynchronize(p.pin_ev[i]));
    else QF_HIP(hipEventCreateWithFlags(&p.pin_ev[i], hipEventDisableTiming));
    if (words > p.h_pin_cap[i]) {
      // sized once for the longest lists (every filter and region), since
      // pinned allocations and frees cost the host up to a millisecond
      const uint64_t cap = std::max<uint64_t>(words, static_cast<uint64_t>(p.nf) + p.G);
      (void)hipHostFree(p.h_pin[i]);
      p.h_pin[i] = nullptr;
      p.h_pin_cap[i] = 0;
      if (hipHostMalloc(reinterpret_cast<void **>(&p.h_pin[i]), cap * sizeof(uint32_t), 0) != hipSuccess)
        return fail(QF_ERR_OOM);
      p.h_pin_cap[i] = cap;
    }
    std::copy(p.h_afil.begin(), p.h_afil.end(), p.h_pin[i]);
    std::copy(p.h_areg.begin(), p.h_areg.end(), p.h_pin[i] + nactive);
    QF_HIP(hipMemcpyAsync(p.d_afil, p.h_pin[i], nactive * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    QF_HIP(hipMemcpyAsync(p.d_areg, p.h_pin[i] + nactive, p.h_areg.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice, s));
    QF_HIP(hipEventRecord(p.pin_ev[i], s));
    p.nafil = nactive;
    p.nareg = static_cast<uint32_t>(p.h_areg.size());
  }
  // one filter: its composite key is the fingerprint itself, and the sort
  // hashes the keys on its first read
  const uint32_t bits = fid ? p.gbits + p.RL + p.r : single_q + p.r;
  const uint64_t pmask = bits >= 64 ? ~0ull : ((1ull << bits) - 1ull);
  // pre: the fingerprints (or composite keys) are computed into bufA first
  const bool pre = fid || values;
  if (fid) QF_HIP(qf::launch_hash_multi(keys, fid, n, p, p.bufA, s, p.timer));
  if (values) {
    const uint32_t kb = single_q + p.r - vbits;
    QF_HIP(qf::launch_kv_compose(keys, values, n, (1ull << kb) - 1ull, vbits, p.bufA, s, p.timer));
  }
  if (n <= qf::SMALL_KEYS) {
    // small batch: sort and reduction in one work-group
    QF_HIP(qf::launch_small_prep(pre ? p.bufA : keys, n, bits, pmask, !pre, p.bufC, p.bufD, p.pst, s, p.timer));
  } else {
    uint64_t *sorted = nullptr;
    if (pre)
      QF_HIP(qf::launch_sort(p.bufA, p.bufB, n, bits, p.hist, &sorted, s, p));
    else
      QF_HIP(qf::launch_sort(p.bufA, p.bufB, n, bits, p.hist, &sorted, s, p, keys, pmask));
    uint64_t *other = sorted == p.bufA ? p.bufB : p.bufA;
    QF_HIP(qf::launch_rle(sorted, n, other, p.bufC, p.bufD, p.hist + 256, p.pst, s, p));
  }
  QF_HIP(qf::launch_bounds(p.bufC, p, s));
  QF_HIP(qf::launch_merge(p, p.bufC, p.bufD, del, not_found, s));
  p.batches += 1;
  return QF_OK;
}

int check_filter(const qf_filter *f) { return f ? QF_OK : fail(QF_ERR_ARG); }

int update(qf_filter *f, const uint64_t *keys, uint64_t n, int del, uint64_t *not_found,
           void *stream) {
  if (!f || (n && !keys) || f->vbits) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  return pipe_update(f->pipe, keys, nullptr, n, del, not_found, static_cast<hipStream_t>(stream), f->q);
}

int read_clear_error(qf_filter *f) {
  uint64_t st[qf::ST_WORDS];
  QF_HIP(hipMemcpy(st, f->state, sizeof(st), hipMemcpyDeviceToHost));
  const int64_t e = static_cast<int64_t>(st[qf::ST_ERR]);
  if (e != 0) {
    const uint64_t zero = 0;
    QF_HIP(hipMemcpy(f->state + qf::ST_ERR, &zero, sizeof(zero), hipMemcpyHostToDevice));
    return fail(static_cast<int>(e));
  }
  return QF_OK;
}

// Launch timer: a pool of reusable events; pairs are resolved on read.
struct EventTimer : qf::Timer {
  std::vector<hipEvent_t> pool;
  struct Pair { int kind; hipEvent_t a, b; };
  std::vector<Pair> pending;
  hipEvent_t open_ev = nullptr;
  uint32_t mask = QF_PROF_ALL;  // kinds whose launches are bracketed
  double ms[QF_PROF_KINDS] = {};
  uint64_t n[QF_PROF_KINDS] = {};
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(int kind, hipStream_t s) override {
    if (!((mask >> kind) & 1u)) return;
    open_ev = take();
    (void)hipEventRecord(open_ev, s);
  }
  void end(int kind, hipStream_t s) override {
    if (!((mask >> kind) & 1u) || !open_ev) return;
    hipEvent_t e = take();
    (void)hipEventRecord(e, s);
    pending.push_back(Pair{kind, open_ev, e});
    open_ev = nullptr;
  }
  int collect() {
    for (const Pair &p : pending) {
      if (hipEventSynchronize(p.b) != hipSuccess) return QF_ERR_DEVICE;
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.a, p.b) != hipSuccess) return QF_ERR_DEVICE;
      ms[p.kind] += t;
      n[p.kind] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
    return QF_OK;
  }
  ~EventTimer() override {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    for (const Pair &p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
  }
};

bool tuning_from(const qf_tuning_t &t, qf::Tune *out) {
  qf::Tune d;
  if (t.region_log2 != 0 && (t.region_log2 < 6 || t.region_log2 > 13)) return false;
  if (t.sort_tile != 0 && t.sort_tile != 2048 && t.sort_tile != 4096) return false;
  if (t.sort_chunk != 0 && (t.sort_chunk < 4096 || t.sort_chunk > 65536 || (t.sort_chunk & (t.sort_chunk - 1))))
    return false;
  const uint32_t k = t.lookup_keys_per_lane;
  if (k != 0 && k != 1 && k != 2 && k != 4) return false;
  out->region_log2 = t.region_log2;
  out->sort_tile = t.sort_tile ? t.sort_tile : d.sort_tile;
  out->sort_chunk = t.sort_chunk ? t.sort_chunk : d.sort_chunk;
  out->lookup_kpl = k ? k : d.lookup_kpl;
  return true;
}

void tuning_to(const qf::Pipe &p, qf_tuning_t *t) {
  t->region_log2 = p.RL;
  t->sort_tile = p.tune.sort_tile;
  t->sort_chunk = p.tune.sort_chunk;
  t->lookup_keys_per_lane = p.tune.lookup_kpl;
}

// rebuild a pipeline with new launch parameters (waits for the device; keeps
// the scratch capacity, drops the launch timer)
int retune(qf::Pipe &p, qf_filter *const *fs, uint32_t nf, const qf::Tune &tn) {
  QF_HIP(hipDeviceSynchronize());
  const uint64_t cap = p.cap;
  pipe_free(p);
  int rc = pipe_init(p, fs, nf, tn);
  if (rc == QF_OK && cap) rc = ensure_scratch(p, cap, nullptr);
  return rc;
}

int profile_enable(qf::Pipe &p, int kinds) {
  const bool enable = (kinds & QF_PROF_ALL) != 0;
  if (enable && !p.timer) p.timer = new (std::nothrow) EventTimer();
  if (enable && !p.timer) return fail(QF_ERR_OOM);
  if (enable) static_cast<EventTimer *>(p.timer)->mask = static_cast<uint32_t>(kinds) & QF_PROF_ALL;
  if (!enable && p.timer) {
    (void)static_cast<EventTimer *>(p.timer)->collect();
    delete p.timer;
    p.timer = nullptr;
  }
  return QF_OK;
}

int profile_read(qf::Pipe &p, double *ms, uint64_t *n) {
  if (!p.timer) {
    for (int k = 0; k < QF_PROF_KINDS; ++k) {
      ms[k] = 0.0;
      n[k] = 0;
    }
    return QF_OK;
  }
  EventTimer *t = static_cast<EventTimer *>(p.timer);
  const int rc = t->collect();
  for (int k = 0; k < QF_PROF_KINDS; ++k) {
    ms[k] = t->ms[k];
    n[k] = t->n[k];
    t->ms[k] = 0.0;
    t->n[k] = 0;
  }
  return rc ? fail(rc) : QF_OK;
}


// ---- batch scratch that is never allocated ----------------------------------
// qf_insert_batch_noalloc runs the same pipeline as qf_insert_batch, with the
// batch scratch in the file-scope array `scratch` instead of the filter's
// grow-only area.  Each GPU the library runs on holds its own copy of the
// array until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address is looked up once per
// device with that device current (hipGetSymbolAddress) and only that address
// is handed to kernels.
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
uint8_t *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// the device address of `scratch` on device dev (looked up on first use)
int noalloc_scratch(int dev, uint8_t **out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(QF_ERR_ARG);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    int cur = -1;
    QF_HIP(hipGetDevice(&cur));
    if (cur != dev) QF_HIP(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) QF_HIP(hipSetDevice(cur));
    if (e != hipSuccess || p == nullptr) return fail(QF_ERR_DEVICE);
    g_noalloc_ptr[dev] = static_cast<uint8_t *>(p);
  }
  *out = g_noalloc_ptr[dev];
  return QF_OK;
}

// enumeration of f into fp / cnt (device, at least cap entries); *n gets the
// number of pairs; *big whether a count is 2^32 or more.  Synchronous.
int enumerate_into(qf_filter *f, uint64_t *fp, uint64_t *cnt, uint64_t cap, uint64_t *n, bool *big,
                   hipStream_t s) {
  void *scr = nullptr;
  if (hipMalloc(&scr, qf::enum_scratch_bytes(f)) != hipSuccess) return fail(QF_ERR_OOM);
  int rc = QF_OK;
  uint64_t words[2] = {0, 0};
  if (qf::launch_enum(f, scr, nullptr, nullptr, false, s) != hipSuccess ||
      hipMemcpyAsync(words, qf::enum_words(f, scr), sizeof(words), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    rc = fail(QF_ERR_DEVICE);
  } else {
    *n = words[0];
    if (cap == 0) {
      // (only the number of pairs was asked for)
    } else if (words[0] > cap) {
      rc = fail(QF_ERR_ARG);
    } else if (words[0]) {
      if (qf::launch_enum(f, scr, fp, cnt, true, s) != hipSuccess ||
          hipMemcpyAsync(words, qf::enum_words(f, scr), sizeof(words), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        rc = fail(QF_ERR_DEVICE);
      else if (big)
        *big = words[1] != 0;
    }
  }
  (void)hipFree(scr);
  return rc;
}

}  // namespace

namespace qf {
int record_error(int code) { return fail(code); }
}  // namespace qf

extern "C" {

qf_t *qf_create(uint32_t q, uint32_t r) {
  if (q < 6 || q > QF_Q_MAX || (r != 8 && r != 16)) {
    fail(QF_ERR_ARG);
    return nullptr;
  }
  qf_filter *f = new (std::nothrow) qf_filter();  // value-initialised: all zero
  if (!f) {
    fail(QF_ERR_OOM);
    return nullptr;
  }
  f->q = q;
  f->r = r;
  f->N = 1ull << q;
  f->E = extra_slots(q);
  f->P = f->N + f->E;
  f->nblocks = f->P / 64;
  f->block_bytes = static_cast<uint32_t>(qf::table_bytes(1, r));
  (void)hipGetDevice(&f->device);
  bool ok = true;
  for (int c = 0; c < 2 && ok; ++c) {
    ok = hipMalloc(&f->blk[c], f->nblocks * f->block_bytes) == hipSuccess &&
         hipMemset(f->blk[c], 0, f->nblocks * f->block_bytes) == hipSuccess;
  }
  ok = ok && hipMalloc(reinterpret_cast<void **>(&f->state), qf::ST_WORDS * sizeof(uint64_t)) == hipSuccess &&
       hipMemset(f->state, 0, qf::ST_WORDS * sizeof(uint64_t)) == hipSuccess;
  const uint64_t lock_bytes = qf::point_lock_words(f->P) * sizeof(uint32_t);
  ok = ok && hipMalloc(reinterpret_cast<void **>(&f->plocks), lock_bytes) == hipSuccess &&
       hipMemset(f->plocks, 0, lock_bytes) == hipSuccess;
  if (!ok) {
    qf_destroy(f);
    fail(QF_ERR_OOM);
    return nullptr;
  }
  qf_filter *self[1] = {f};
  if (pipe_init(f->pipe, self, 1, qf::Tune()) != QF_OK) {
    qf_destroy(f);
    fail(QF_ERR_OOM);
    return nullptr;
  }
  f->table_device_bytes = 2 * qf::table_bytes(f->nblocks, r) + qf::ST_WORDS * 8 + lock_bytes;
  return f;
}

void qf_destroy(qf_t *f) {
  if (!f) return;
  (void)hipDeviceSynchronize();
  for (int c = 0; c < 2; ++c) {
    (void)hipFree(f->blk[c]);
  }
  (void)hipFree(f->state);
  (void)hipFree(f->plocks);
  pipe_free(f->pipe);
  delete f;
}

int qf_insert_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, void *stream) {
  return update(f, d_keys, n, 0, nullptr, stream);
}

int qf_insert_batch_noalloc(qf_t *f, const uint64_t *d_keys, uint64_t n, void *stream) {
  if (!f || (n && !d_keys) || f->vbits) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > QF_NOALLOC_KEYS) return fail(QF_ERR_LIMIT);
  uint8_t *base = nullptr;
  const int rc0 = noalloc_scratch(f->device, &base);
  if (rc0) return rc0;
  // the filter's pipeline with its scratch pointers swapped for the static
  // area (capacity QF_NOALLOC_KEYS, so nothing grows) and no launch timer
  // (its events are created on demand); restored after the launches
  qf::Pipe &p = f->pipe;
  const uint64_t cap = p.cap, hw = p.hist_words;
  uint64_t *const bA = p.bufA, *const bB = p.bufB, *const bC = p.bufC, *const bD = p.bufD, *const bE = p.bufE;
  uint32_t *const hist = p.hist;
  qf::Timer *const timer = p.timer;
  const uint64_t K = QF_NOALLOC_KEYS;
  uint64_t *const w = reinterpret_cast<uint64_t *>(base);
  p.bufA = w;
  p.bufB = w + K;
  p.bufC = w + 2 * K;
  p.bufD = w + 3 * K;
  p.bufE = w + 4 * K;  // 4 K words: 32 bytes per key
  p.hist = reinterpret_cast<uint32_t *>(w + 8 * K);
  p.hist_words = QF_NOALLOC_HIST_WORDS;
  p.cap = K;
  p.timer = nullptr;
  const int rc = pipe_update(p, d_keys, nullptr, n, 0, nullptr, static_cast<hipStream_t>(stream), f->q);
  p.bufA = bA;
  p.bufB = bB;
  p.bufC = bC;
  p.bufD = bD;
  p.bufE = bE;
  p.hist = hist;
  p.hist_words = hw;
  p.cap = cap;
  p.timer = timer;
  return rc;
}

int qf_delete_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint64_t *d_not_found,
                    void *stream) {
  return update(f, d_keys, n, 1, d_not_found, stream);
}

int qf_point_insert(qf_t *f, const uint64_t *d_keys, uint64_t n, int32_t *d_status, void *stream) {
  if (!f || (n && !d_keys) || f->vbits) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  QF_HIP(qf::launch_point(f, d_keys, n, 0, d_status, nullptr, static_cast<hipStream_t>(stream)));
  return QF_OK;
}

int qf_point_delete(qf_t *f, const uint64_t *d_keys, uint64_t n, int32_t *d_status, uint64_t *d_not_found,
                    void *stream) {
  if (!f || (n && !d_keys) || f->vbits) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  QF_HIP(qf::launch_point(f, d_keys, n, 1, d_status, d_not_found, static_cast<hipStream_t>(stream)));
  return QF_OK;
}

int qf_query_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint8_t *d_out, void *stream) {
  if (!f || (n && (!d_keys || !d_out)) || f->vbits) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  QF_HIP(qf::launch_lookup(f, d_keys, n, d_out, nullptr, static_cast<hipStream_t>(stream)));
  return QF_OK;
}

int qf_count_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint64_t *d_out, void *stream) {
  if (!f || (n && (!d_keys || !d_out)) || f->vbits) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  QF_HIP(qf::launch_lookup(f, d_keys, n, nullptr, d_out, static_cast<hipStream_t>(stream)));
  return QF_OK;
}

qf_t *qf_create_kv(uint32_t q, uint32_t r, uint32_t vbits) {
  if (vbits < 1 || vbits >= r) {
    fail(QF_ERR_ARG);
    return nullptr;
  }
  qf_t *f = qf_create(q, r);
  if (f) f->vbits = vbits;
  return f;
}

int qf_kv_insert_batch(qf_t *f, const uint64_t *d_keys, const uint64_t *d_values, uint64_t n, void *stream) {
  if (!f || !f->vbits || (n && (!d_keys || !d_values))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  return pipe_update(f->pipe, d_keys, nullptr, n, 0, nullptr, static_cast<hipStream_t>(stream), f->q, nullptr,
                     nullptr, 0, d_values, f->vbits);
}

int qf_kv_delete_batch(qf_t *f, const uint64_t *d_keys, const uint64_t *d_values, uint64_t n,
                       uint64_t *d_not_found, void *stream) {
  if (!f || !f->vbits || (n && (!d_keys || !d_values))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  return pipe_update(f->pipe, d_keys, nullptr, n, 1, d_not_found, static_cast<hipStream_t>(stream), f->q, nullptr,
                     nullptr, 0, d_values, f->vbits);
}

int qf_kv_lookup_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint64_t *d_value, uint32_t *d_nvalues,
                       void *stream) {
  if (!f || !f->vbits || (n && (!d_keys || !d_value))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  QF_HIP(qf::launch_kv_lookup(f, d_keys, n, d_value, d_nvalues, static_cast<hipStream_t>(stream)));
  return QF_OK;
}

int qf_sync(qf_t *f, void *stream) {
  if (check_filter(f)) return QF_ERR_ARG;
  QF_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  return read_clear_error(f);
}

int qf_export(qf_t *f, qf_layout_t *out, void *stream) {
  if (!f || !out || !out->occ_words || !out->runend_words || !out->slots || !out->offsets)
    return fail(QF_ERR_ARG);
  hipStream_t s = static_cast<hipStream_t>(stream);
  QF_HIP(hipStreamSynchronize(s));
  const uint64_t nq = f->N / 64, nb = f->nblocks, P = f->P;
  uint64_t *d_occ = nullptr, *d_rend = nullptr;
  uint16_t *d_slots = nullptr;
  uint32_t *d_offs = nullptr;
  int rc = QF_OK;
  if (hipMalloc(&d_occ, nq * 8) != hipSuccess || hipMalloc(&d_rend, nb * 8) != hipSuccess ||
      hipMalloc(&d_slots, P * 2) != hipSuccess || hipMalloc(&d_offs, nb * 4) != hipSuccess) {
    rc = fail(QF_ERR_OOM);
  }
  uint64_t st[qf::ST_WORDS];
  if (rc == QF_OK) {
    if (qf::launch_export(f, d_occ, d_rend, d_slots, d_offs, s) != hipSuccess ||
        hipMemcpyAsync(out->occ_words, d_occ, nq * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(out->runend_words, d_rend, nb * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(out->slots, d_slots, P * 2, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(out->offsets, d_offs, nb * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(st, f->state, sizeof(st), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(QF_ERR_DEVICE);
    }
  }
  (void)hipFree(d_occ);
  (void)hipFree(d_rend);
  (void)hipFree(d_slots);
  (void)hipFree(d_offs);
  if (rc) return rc;
  out->header[0] = f->q;
  out->header[1] = f->r;
  out->header[2] = f->N;
  out->header[3] = f->E;
  out->header[4] = f->P;
  out->header[5] = st[qf::ST_USED];
  out->header[6] = st[qf::ST_DIST];
  out->header[7] = st[qf::ST_TOTAL];
  return read_clear_error(f);
}

int qf_import(qf_t *f, const qf_layout_t *in, void *stream) {
  if (!f || !in || !in->occ_words || !in->runend_words || !in->slots || !in->offsets)
    return fail(QF_ERR_ARG);
  if (in->header[0] != f->q || in->header[1] != f->r || in->header[4] != f->P)
    return fail(QF_ERR_ARG);
  hipStream_t s = static_cast<hipStream_t>(stream);
  QF_HIP(hipStreamSynchronize(s));
  const uint64_t nq = f->N / 64, nb = f->nblocks, P = f->P;
  uint64_t *d_occ = nullptr, *d_rend = nullptr;
  uint16_t *d_slots = nullptr;
  uint32_t *d_offs = nullptr;
  int rc = QF_OK;
  if (hipMalloc(&d_occ, nq * 8) != hipSuccess || hipMalloc(&d_rend, nb * 8) != hipSuccess ||
      hipMalloc(&d_slots, P * 2) != hipSuccess || hipMalloc(&d_offs, nb * 4) != hipSuccess) {
    rc = fail(QF_ERR_OOM);
  }
  uint64_t st[qf::ST_WORDS];
  if (rc == QF_OK) {
    if (hipMemcpyAsync(st, f->state, sizeof(st), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(QF_ERR_DEVICE);
    }
  }
  if (rc == QF_OK) {
    st[qf::ST_CUR] = 0;
    st[qf::ST_USED] = in->header[5];
    st[qf::ST_DIST] = in->header[6];
    st[qf::ST_TOTAL] = in->header[7];
    if (hipMemcpyAsync(d_occ, in->occ_words, nq * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_rend, in->runend_words, nb * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_slots, in->slots, P * 2, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_offs, in->offsets, nb * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(f->state, st, sizeof(st), hipMemcpyHostToDevice, s) != hipSuccess ||
        qf::launch_import(f, d_occ, d_rend, d_slots, d_offs, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(QF_ERR_DEVICE);
    }
  }
  (void)hipFree(d_occ);
  (void)hipFree(d_rend);
  (void)hipFree(d_slots);
  (void)hipFree(d_offs);
  return rc;
}

int qf_stats(qf_t *f, uint64_t *out, void *stream) {
  if (!f || !out) return fail(QF_ERR_ARG);
  QF_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  uint64_t st[qf::ST_WORDS];
  QF_HIP(hipMemcpy(st, f->state, sizeof(st), hipMemcpyDeviceToHost));
  out[0] = st[qf::ST_USED];
  out[1] = st[qf::ST_DIST];
  out[2] = st[qf::ST_TOTAL];
  return QF_OK;
}

int qf_enumerate(qf_t *f, uint64_t *d_fp, uint64_t *d_cnt, uint64_t cap, uint64_t *n, void *stream) {
  if (!f || !n || (cap && (!d_fp || !d_cnt))) return fail(QF_ERR_ARG);
  return enumerate_into(f, d_fp, d_cnt, cap, n, nullptr, static_cast<hipStream_t>(stream));
}

int qf_merge_into(qf_t *dst, qf_t *src, int subtract, uint64_t *d_not_found, void *stream) {
  if (!dst || !src || dst->q + dst->r != src->q + src->r || dst->vbits != src->vbits) return fail(QF_ERR_ARG);
  const hipStream_t s = static_cast<hipStream_t>(stream);
  uint64_t st[qf::ST_WORDS];
  QF_HIP(hipStreamSynchronize(s));
  QF_HIP(hipMemcpy(st, src->state, sizeof(st), hipMemcpyDeviceToHost));
  const uint64_t nsrc = st[qf::ST_DIST];
  if (nsrc == 0) return QF_OK;
  if (nsrc > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  qf::Pipe &p = dst->pipe;
  int rc = ensure_scratch(p, nsrc, s);
  if (rc) return rc;
  // the source's pairs are the reduced batch: sorted distinct fingerprints
  // (a single filter's merge key is the fingerprint) and their counts
  uint64_t n = 0;
  bool big = false;
  rc = enumerate_into(src, p.bufC, p.bufD, p.cap, &n, &big, s);
  if (rc) return rc;
  if (big) return fail(QF_ERR_ARG);  // counts of 2^32 or more per fingerprint
  if (n == 0) return QF_OK;
  QF_HIP(hipMemcpyAsync(p.pst + qf::ST_NUNIQ, &n, sizeof(n), hipMemcpyHostToDevice, s));
  p.nafil = p.nareg = 0;
  QF_HIP(qf::launch_bounds(p.bufC, p, s));
  QF_HIP(qf::launch_merge(p, p.bufC, p.bufD, subtract ? 1 : 0, d_not_found, s));
  QF_HIP(hipStreamSynchronize(s));  // (n lives on this host stack until the copy is done)
  p.batches += 1;
  return QF_OK;
}

qf_t *qf_resize(qf_t *src, uint32_t q, uint32_t r, void *stream) {
  if (!src || q + r != src->q + src->r || r <= src->vbits) {
    fail(QF_ERR_ARG);
    return nullptr;
  }
  qf_t *dst = qf_create(q, r);
  if (!dst) return nullptr;
  dst->vbits = src->vbits;
  const int rc = qf_merge_into(dst, src, 0, nullptr, stream);
  if (rc == QF_OK) {
    const int e = qf_sync(dst, stream);
    if (e == QF_OK) return dst;
    fail(e);
  }
  qf_destroy(dst);
  return nullptr;
}

int qf_last_error(void) { return g_last_error; }

int qf_reserve(qf_t *f, uint64_t n, void *stream) {
  if (!f || n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  return ensure_scratch(f->pipe, n, static_cast<hipStream_t>(stream));
}

int qf_set_reserve(qf_set_t *st, uint64_t n, void *stream) {
  if (!st || n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  return ensure_scratch(st->pipe, n, static_cast<hipStream_t>(stream));
}

qf_set_t *qf_set_create(qf_t *const *filters, uint32_t nf) {
  if (!filters || nf == 0) {
    fail(QF_ERR_ARG);
    return nullptr;
  }
  // NULL handles and the same handle twice are refused before any handle is
  // read: two descriptors of one filter would both write its other table
  // copy and flip its current copy twice in one merge launch
  std::vector<const qf_t *> seen(filters, filters + nf);
  std::sort(seen.begin(), seen.end());
  for (uint32_t i = 0; i < nf; ++i) {
    if (!seen[i] || (i > 0 && seen[i] == seen[i - 1])) {
      fail(QF_ERR_ARG);
      return nullptr;
    }
  }
  for (uint32_t i = 0; i < nf; ++i) {
    if (filters[i]->r != filters[0]->r || filters[i]->vbits) {
      fail(QF_ERR_ARG);
      return nullptr;
    }
  }
  qf_set *st = new (std::nothrow) qf_set();
  if (!st) {
    fail(QF_ERR_OOM);
    return nullptr;
  }
  st->nf = nf;
  st->fs = new (std::nothrow) qf_filter *[nf];
  if (!st->fs) {
    delete st;
    fail(QF_ERR_OOM);
    return nullptr;
  }
  for (uint32_t i = 0; i < nf; ++i) st->fs[i] = filters[i];
  int rc = pipe_init(st->pipe, st->fs, nf, qf::Tune());
  if (rc == QF_OK) {
    std::vector<uint32_t *> lk(nf);
    for (uint32_t i = 0; i < nf; ++i) lk[i] = st->fs[i]->plocks;
    if (hipMalloc(reinterpret_cast<void **>(&st->d_plocks), nf * sizeof(uint32_t *)) != hipSuccess)
      rc = QF_ERR_OOM;
    else if (hipMemcpy(st->d_plocks, lk.data(), nf * sizeof(uint32_t *), hipMemcpyHostToDevice) != hipSuccess)
      rc = QF_ERR_DEVICE;
    if (rc != QF_OK) pipe_free(st->pipe);
  }
  if (rc != QF_OK) {
    (void)hipFree(st->d_plocks);
    delete[] st->fs;
    delete st;
    fail(rc);
    return nullptr;
  }
  return st;
}

void qf_set_destroy(qf_set_t *st) {
  if (!st) return;
  (void)hipDeviceSynchronize();
  pipe_free(st->pipe);
  (void)hipFree(st->d_plocks);
  delete[] st->fs;
  delete st;
}

int qf_set_insert_batch(qf_set_t *st, const uint32_t *d_fid, const uint64_t *d_keys, uint64_t n,
                        void *stream) {
  if (!st || (n && (!d_keys || !d_fid))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  return pipe_update(st->pipe, d_keys, d_fid, n, 0, nullptr, static_cast<hipStream_t>(stream), 0);
}

int qf_set_delete_batch(qf_set_t *st, const uint32_t *d_fid, const uint64_t *d_keys, uint64_t n,
                        uint64_t *d_not_found, void *stream) {
  if (!st || (n && (!d_keys || !d_fid))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  return pipe_update(st->pipe, d_keys, d_fid, n, 1, d_not_found, static_cast<hipStream_t>(stream), 0);
}

int qf_set_insert_some(qf_set_t *st, const uint32_t *h_filters, uint32_t n_filters, const uint32_t *d_fid,
                       const uint64_t *d_keys, uint64_t n, void *stream) {
  if (!st || !h_filters || (n && (!d_keys || !d_fid))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  return pipe_update(st->pipe, d_keys, d_fid, n, 0, nullptr, static_cast<hipStream_t>(stream), 0, st, h_filters,
                     n_filters);
}

int qf_set_delete_some(qf_set_t *st, const uint32_t *h_filters, uint32_t n_filters, const uint32_t *d_fid,
                       const uint64_t *d_keys, uint64_t n, uint64_t *d_not_found, void *stream) {
  if (!st || !h_filters || (n && (!d_keys || !d_fid))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  return pipe_update(st->pipe, d_keys, d_fid, n, 1, d_not_found, static_cast<hipStream_t>(stream), 0, st,
                     h_filters, n_filters);
}

int qf_set_query_batch(qf_set_t *st, const uint32_t *d_fid, const uint64_t *d_keys, uint64_t n,
                       uint8_t *d_out, void *stream) {
  if (!st || (n && (!d_keys || !d_fid || !d_out))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  QF_HIP(qf::launch_lookup_multi(st->pipe, d_keys, d_fid, n, d_out, nullptr, static_cast<hipStream_t>(stream)));
  return QF_OK;
}

int qf_set_count_batch(qf_set_t *st, const uint32_t *d_fid, const uint64_t *d_keys, uint64_t n,
                       uint64_t *d_out, void *stream) {
  if (!st || (n && (!d_keys || !d_fid || !d_out))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  QF_HIP(qf::launch_lookup_multi(st->pipe, d_keys, d_fid, n, nullptr, d_out, static_cast<hipStream_t>(stream)));
  return QF_OK;
}

int qf_set_sync(qf_set_t *st, void *stream) {
  if (!st) return fail(QF_ERR_ARG);
  QF_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  // the set's own flag (a filter index out of range), then each filter's
  // deferred error; all are cleared, the first one is returned
  uint64_t w = 0;
  QF_HIP(hipMemcpy(&w, st->pipe.pst + qf::ST_ERR, sizeof(w), hipMemcpyDeviceToHost));
  int first = QF_OK;
  if (w != 0) {
    const uint64_t zero = 0;
    QF_HIP(hipMemcpy(st->pipe.pst + qf::ST_ERR, &zero, sizeof(zero), hipMemcpyHostToDevice));
    first = static_cast<int>(static_cast<int64_t>(w));
  }
  for (uint32_t i = 0; i < st->nf; ++i) {
    const int rc = read_clear_error(st->fs[i]);
    if (first == QF_OK && rc != QF_OK) first = rc;
  }
  return first == QF_OK ? QF_OK : fail(first);
}

int qf_set_errors(qf_set_t *st, int32_t *codes, void *stream) {
  if (!st || !codes) return fail(QF_ERR_ARG);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<int64_t> e(st->nf);
  QF_HIP(qf::launch_take_errors(st->pipe, st->pipe.d_err, s));
  QF_HIP(hipMemcpyAsync(e.data(), st->pipe.d_err, st->nf * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  QF_HIP(hipStreamSynchronize(s));
  int bad = 0;
  for (uint32_t i = 0; i < st->nf; ++i) {
    codes[i] = static_cast<int32_t>(e[i]);
    bad += e[i] != 0;
  }
  return bad;
}

int qf_set_info(const qf_set_t *st, uint64_t *info) {
  if (!st || !info) return fail(QF_ERR_ARG);
  info[0] = st->nf;
  info[1] = st->pipe.r;
  info[2] = st->pipe.G;
  info[3] = st->pipe.RL;
  info[4] = st->pipe.device_bytes;
  info[5] = st->pipe.batches;
  info[6] = st->pipe.gbits + st->pipe.RL + st->pipe.r;
  info[7] = 0;
  return QF_OK;
}

int qf_set_profile_enable(qf_set_t *st, int kinds) {
  if (!st) return fail(QF_ERR_ARG);
  return profile_enable(st->pipe, kinds);
}

int qf_set_profile_read(qf_set_t *st, double *ms, uint64_t *n) {
  if (!st || !ms || !n) return fail(QF_ERR_ARG);
  return profile_read(st->pipe, ms, n);
}

uint64_t qf_table_bytes(uint32_t q, uint32_t r) {
  if (q < 6 || q > QF_Q_MAX || (r != 8 && r != 16)) return 0;
  const uint64_t P = (1ull << q) + extra_slots(q);
  return qf::table_bytes(P / 64, r);
}

int qf_info(const qf_t *f, uint64_t *info) {
  if (!f || !info) return fail(QF_ERR_ARG);
  info[0] = f->q;
  info[1] = f->r;
  info[2] = f->N;
  info[3] = f->E;
  info[4] = f->P;
  info[5] = 1ull << f->pipe.one.rlog;
  info[6] = f->table_device_bytes + f->pipe.device_bytes;
  info[7] = f->pipe.batches;
  return QF_OK;
}

int qf_profile_enable(qf_t *f, int kinds) {
  if (!f) return fail(QF_ERR_ARG);
  return profile_enable(f->pipe, kinds);
}

int qf_profile_read(qf_t *f, double *ms, uint64_t *n) {
  if (!f || !ms || !n) return fail(QF_ERR_ARG);
  return profile_read(f->pipe, ms, n);
}

// ---- launch parameters -----------------------------------------------------

int qf_tune(qf_t *f, const qf_tuning_t *t) {
  if (!f || !t) return fail(QF_ERR_ARG);
  qf::Tune tn;
  if (!tuning_from(*t, &tn)) return fail(QF_ERR_ARG);
  qf_filter *self[1] = {f};
  return retune(f->pipe, self, 1, tn);
}

int qf_get_tuning(const qf_t *f, qf_tuning_t *t) {
  if (!f || !t) return fail(QF_ERR_ARG);
  tuning_to(f->pipe, t);
  return QF_OK;
}

int qf_set_tune(qf_set_t *st, const qf_tuning_t *t) {
  if (!st || !t) return fail(QF_ERR_ARG);
  qf::Tune tn;
  if (!tuning_from(*t, &tn)) return fail(QF_ERR_ARG);
  return retune(st->pipe, st->fs, st->nf, tn);
}

int qf_set_get_tuning(const qf_set_t *st, qf_tuning_t *t) {
  if (!st || !t) return fail(QF_ERR_ARG);
  tuning_to(st->pipe, t);
  return QF_OK;
}

// ---- stream capture ----------------------------------------------------------

struct qf_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int qf_graph_begin(void *stream) {
  if (!stream) return fail(QF_ERR_ARG);
  QF_HIP(hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal));
  return QF_OK;
}

qf_graph_t *qf_graph_end(void *stream) {
  if (!stream) {
    fail(QF_ERR_ARG);
    return nullptr;
  }
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(static_cast<hipStream_t>(stream), &g) != hipSuccess || !g) {
    (void)hipGetLastError();
    fail(QF_ERR_DEVICE);
    return nullptr;
  }
  qf_graph *q = new (std::nothrow) qf_graph();
  if (!q) {
    (void)hipGraphDestroy(g);
    fail(QF_ERR_OOM);
    return nullptr;
  }
  q->graph = g;
  if (hipGraphInstantiate(&q->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    qf_graph_destroy(q);
    fail(QF_ERR_DEVICE);
    return nullptr;
  }
  return q;
}

int qf_graph_launch(qf_graph_t *g, void *stream) {
  if (!g || !g->exec) return fail(QF_ERR_ARG);
  QF_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return QF_OK;
}

void qf_graph_destroy(qf_graph_t *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
