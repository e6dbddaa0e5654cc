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
#include <vector>

#include "qf.h"
#include "qf_dev.h"
#include "qf_lib.h"

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

void free_scratch(qf_filter *f) {
  (void)hipFree(f->bufA);
  (void)hipFree(f->bufB);
  (void)hipFree(f->bufC);
  (void)hipFree(f->bufD);
  f->bufA = f->bufB = f->bufC = f->bufD = nullptr;
  f->cap = 0;
}

int ensure_scratch(qf_filter *f, uint64_t n, hipStream_t s) {
  if (n <= f->cap) return QF_OK;
  uint64_t cap = 1ull << 16;
  while (cap < n) cap <<= 1;
  if (f->cap) QF_HIP(hipStreamSynchronize(s));
  f->device_bytes -= 4 * f->cap * sizeof(uint64_t);
  free_scratch(f);
  const size_t bytes = cap * sizeof(uint64_t);
  if (hipMalloc(&f->bufA, bytes) != hipSuccess || hipMalloc(&f->bufB, bytes) != hipSuccess ||
      hipMalloc(&f->bufC, bytes) != hipSuccess || hipMalloc(&f->bufD, bytes) != hipSuccess) {
    free_scratch(f);
    return fail(QF_ERR_OOM);
  }
  f->cap = cap;
  f->device_bytes += 4 * bytes;
  return QF_OK;
}

int check_filter(const qf_filter *f) { return f ? QF_OK : fail(QF_ERR_ARG); }

int update(qf_filter *f, const uint64_t *keys, uint64_t n, int del, uint64_t *not_found,
           void *stream) {
  if (!f || (n && !keys)) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return fail(QF_ERR_ARG);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = ensure_scratch(f, n, s);
  if (rc) return rc;
  const uint32_t p = f->q + f->r;
  const uint64_t pmask = p >= 64 ? ~0ull : ((1ull << p) - 1ull);
  QF_HIP(qf::launch_hash(keys, n, pmask, f->bufA, s, f->timer));
  uint64_t *sorted = nullptr;
  QF_HIP(qf::launch_sort(f->bufA, f->bufB, n, p, f->hist, &sorted, s, f->timer));
  uint64_t *other = sorted == f->bufA ? f->bufB : f->bufA;
  QF_HIP(qf::launch_rle(sorted, n, other, f->bufC, f->bufD, f->hist, f->state, s, f->timer));
  QF_HIP(qf::launch_bounds(f->bufC, f->state, f, s));
  if (f->epoch == 65535) {
    QF_HIP(qf::launch_fill_u64(f->tags, 3ull * f->nregions, 0, s));
    f->epoch = 0;
  }
  f->epoch += 1;
  QF_HIP(qf::launch_merge(f, f->bufC, f->bufD, del, not_found, s));
  f->batches += 1;
  return QF_OK;
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
  void begin(int, hipStream_t s) override {
    open_ev = take();
    (void)hipEventRecord(open_ev, s);
  }
  void end(int kind, hipStream_t s) override {
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

}  // namespace

extern "C" {

qf_t *qf_create(uint32_t q, uint32_t r) {
  if (q < 6 || q > 31 || (r != 8 && r != 16)) {
    fail(QF_ERR_ARG);
    return nullptr;
  }
  qf_filter *f = new (std::nothrow) qf_filter();
  if (!f) {
    fail(QF_ERR_OOM);
    return nullptr;
  }
  std::memset(f, 0, sizeof(*f));
  f->q = q;
  f->r = r;
  f->N = 1ull << q;
  f->E = extra_slots(q);
  f->P = f->N + f->E;
  f->nblocks = f->P / 64;
  f->rlog = std::min<uint32_t>(q, static_cast<uint32_t>(qf::max_region_log2(r)));
  const uint64_t S = 1ull << f->rlog;
  f->nqregions = static_cast<uint32_t>(f->N / S);
  f->nregions = static_cast<uint32_t>((f->P + S - 1) / S);
  f->block_bytes = r == 8 ? 80 : 144;
  (void)hipGetDevice(&f->device);
  bool ok = true;
  for (int c = 0; c < 2 && ok; ++c) {
    ok = hipMalloc(&f->blk[c], f->nblocks * f->block_bytes) == hipSuccess &&
         hipMalloc(reinterpret_cast<void **>(&f->off[c]), f->nblocks * sizeof(uint32_t)) == hipSuccess;
    if (ok) {
      ok = hipMemset(f->blk[c], 0, f->nblocks * f->block_bytes) == hipSuccess &&
           hipMemset(f->off[c], 0, f->nblocks * sizeof(uint32_t)) == hipSuccess;
    }
  }
  f->hist_words = 256ull * 1024ull + 256ull * 8;  // histograms + per-pass digit totals
  ok = ok && hipMalloc(reinterpret_cast<void **>(&f->state), qf::ST_WORDS * sizeof(uint64_t)) == hipSuccess &&
       hipMalloc(reinterpret_cast<void **>(&f->rb), (f->nregions + 1ull) * sizeof(uint64_t)) == hipSuccess &&
       hipMalloc(reinterpret_cast<void **>(&f->tags), (8ull * f->nregions + 8) * sizeof(uint64_t)) == hipSuccess &&
       hipMalloc(reinterpret_cast<void **>(&f->hist), f->hist_words * sizeof(uint32_t)) == hipSuccess;
  ok = ok && hipMemset(f->state, 0, qf::ST_WORDS * sizeof(uint64_t)) == hipSuccess &&
       hipMemset(f->tags, 0, (8ull * f->nregions + 8) * sizeof(uint64_t)) == hipSuccess &&
       hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    qf_destroy(f);
    fail(QF_ERR_OOM);
    return nullptr;
  }
  f->rstat = f->tags + 3ull * f->nregions;
  f->cb = reinterpret_cast<int64_t *>(f->tags + 7ull * f->nregions);
  f->device_bytes = 2 * qf::table_bytes(f->nblocks, r) + qf::ST_WORDS * 8 + (f->nregions + 1ull) * 8 +
                    (8ull * f->nregions + 8) * 8 + f->hist_words * 4;
  return f;
}

void qf_destroy(qf_t *f) {
  if (!f) return;
  (void)hipDeviceSynchronize();
  for (int c = 0; c < 2; ++c) {
    (void)hipFree(f->blk[c]);
    (void)hipFree(f->off[c]);
  }
  (void)hipFree(f->state);
  (void)hipFree(f->rb);
  (void)hipFree(f->tags);
  (void)hipFree(f->hist);
  free_scratch(f);
  delete f->timer;
  delete f;
}

int qf_insert_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, void *stream) {
  return update(f, d_keys, n, 0, nullptr, stream);
}

int qf_delete_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint64_t *d_not_found,
                    void *stream) {
  return update(f, d_keys, n, 1, d_not_found, stream);
}

int qf_query_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint8_t *d_out, void *stream) {
  if (!f || (n && (!d_keys || !d_out))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  QF_HIP(qf::launch_lookup(f, d_keys, n, d_out, nullptr, static_cast<hipStream_t>(stream)));
  return QF_OK;
}

int qf_count_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint64_t *d_out, void *stream) {
  if (!f || (n && (!d_keys || !d_out))) return fail(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  QF_HIP(qf::launch_lookup(f, d_keys, n, nullptr, d_out, static_cast<hipStream_t>(stream)));
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

int qf_last_error(void) { return g_last_error; }

uint64_t qf_table_bytes(uint32_t q, uint32_t r) {
  if (q < 6 || q > 31 || (r != 8 && r != 16)) return 0;
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
  info[5] = 1ull << f->rlog;
  info[6] = f->device_bytes;
  info[7] = f->batches;
  return QF_OK;
}

int qf_profile_enable(qf_t *f, int enable) {
  if (!f) return fail(QF_ERR_ARG);
  if (enable && !f->timer) f->timer = new (std::nothrow) EventTimer();
  if (enable && !f->timer) return fail(QF_ERR_OOM);
  if (!enable && f->timer) {
    (void)static_cast<EventTimer *>(f->timer)->collect();
    delete f->timer;
    f->timer = nullptr;
  }
  return QF_OK;
}

int qf_profile_read(qf_t *f, double *ms, uint64_t *n) {
  if (!f || !ms || !n) return fail(QF_ERR_ARG);
  if (!f->timer) {
    for (int k = 0; k < QF_PROF_KINDS; ++k) {
      ms[k] = 0.0;
      n[k] = 0;
    }
    return QF_OK;
  }
  EventTimer *t = static_cast<EventTimer *>(f->timer);
  const int rc = t->collect();
  for (int k = 0; k < QF_PROF_KINDS; ++k) {
    ms[k] = t->ms[k];
    n[k] = t->n[k];
    t->ms[k] = 0.0;
    t->n[k] = 0;
  }
  return rc ? fail(rc) : QF_OK;
}

}  // extern "C"
