// qf_serve.hip -- serving: device-resident filters answering a stream of mixed
// requests with continuous batching (declared in include/qf.h, qfs_*).
//
// A loop thread owns every HIP call of the server.  Requests are admitted in
// submission order; each round takes, per filter, the longest prefix of its
// waiting requests that share one operation (so per filter the effects follow
// admission order), packs the round's keys of each (r, operation) into pinned
// buffers and runs them as filter-set batches (one pipeline of launches for
// all filters with that r).  While the device runs round k the thread forms and
// launches round k + 1 on the same stream (two sets of pinned buffers), then
// completes round k: outputs are copied to the callers' buffers and each
// request's status is its filter's deferred error for that round, if any.
// Filters are admitted while the device bytes they need fit the budget; later
// ones wait (their requests too) until a close frees room.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "qf.h"
#include "qf_lib.h"

namespace {

enum { OP_INSERT = QFS_INSERT, OP_DELETE = QFS_DELETE, OP_QUERY = QFS_QUERY, OP_COUNT = QFS_COUNT, OP_CLOSE = 4,
       OP_EXPORT = 5 };

struct Req {
  uint64_t seq;  // submission order
  int op;
  int id;
  std::vector<uint64_t> keys;  // copied at submission
  void *out;
  uint64_t tag;
  int status;
};

struct Slot {
  uint32_t q, r;
  uint64_t bytes;  // device bytes reserved against the budget
  qf_t *f = nullptr;
  enum { PENDING, OPEN, CLOSED } state = PENDING;
  bool closing = false;  // a close was submitted: no further requests
};

// Pinned staging for one round: keys, filter indexes and outputs.
struct Stage {
  uint64_t cap = 0;
  uint64_t *keys = nullptr;
  uint32_t *fid = nullptr;
  uint64_t *out64 = nullptr;
  uint8_t *out8 = nullptr;
  uint64_t *d_keys = nullptr;
  uint32_t *d_fid = nullptr;
  uint64_t *d_out64 = nullptr;
  uint8_t *d_out8 = nullptr;
  hipEvent_t done = nullptr;
  hipEvent_t start = nullptr;                // the previous round's end, for the part streams
  hipEvent_t part_done[3] = {nullptr, nullptr, nullptr};
  // per-filter deferred errors of the round, gathered on the stream after
  // the round's launches (nerr words per set, sets in order of r)
  // and, behind them, each filter's used slots past its last quotient
  int64_t *d_err = nullptr, *h_err = nullptr;
  int64_t *d_tail = nullptr, *h_tail = nullptr;
  uint32_t nerr = 0;
  bool alloc_err(uint32_t n) {
    (void)hipFree(d_err);
    (void)hipHostFree(h_err);
    (void)hipFree(d_tail);
    (void)hipHostFree(h_tail);
    d_err = h_err = d_tail = h_tail = nullptr;
    nerr = n;
    return n == 0 || (hipMalloc(reinterpret_cast<void **>(&d_err), n * 8) == hipSuccess &&
                      hipHostMalloc(reinterpret_cast<void **>(&h_err), n * 8, 0) == hipSuccess &&
                      hipMalloc(reinterpret_cast<void **>(&d_tail), n * 8) == hipSuccess &&
                      hipHostMalloc(reinterpret_cast<void **>(&h_tail), n * 8, 0) == hipSuccess);
  }
  bool alloc(uint64_t n) {
    cap = n;
    return hipHostMalloc(reinterpret_cast<void **>(&keys), n * 8, 0) == hipSuccess &&
           hipHostMalloc(reinterpret_cast<void **>(&fid), n * 4, 0) == hipSuccess &&
           hipHostMalloc(reinterpret_cast<void **>(&out64), n * 8, 0) == hipSuccess &&
           hipHostMalloc(reinterpret_cast<void **>(&out8), n, 0) == hipSuccess &&
           hipMalloc(reinterpret_cast<void **>(&d_keys), n * 8) == hipSuccess &&
           hipMalloc(reinterpret_cast<void **>(&d_fid), n * 4) == hipSuccess &&
           hipMalloc(reinterpret_cast<void **>(&d_out64), n * 8) == hipSuccess &&
           hipMalloc(reinterpret_cast<void **>(&d_out8), n) == hipSuccess &&
           hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&start, hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&part_done[0], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&part_done[1], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&part_done[2], hipEventDisableTiming) == hipSuccess;
  }
  void release() {
    (void)hipHostFree(keys);
    (void)hipHostFree(fid);
    (void)hipHostFree(out64);
    (void)hipHostFree(out8);
    (void)hipFree(d_keys);
    (void)hipFree(d_fid);
    (void)hipFree(d_out64);
    (void)hipFree(d_out8);
    if (done) (void)hipEventDestroy(done);
    if (start) (void)hipEventDestroy(start);
    for (hipEvent_t e : part_done)
      if (e) (void)hipEventDestroy(e);
    (void)hipFree(d_err);
    (void)hipHostFree(h_err);
    (void)hipFree(d_tail);
    (void)hipHostFree(h_tail);
  }
};

// One (r, operation) batch of a round: the requests and their key offsets.
// An update part is ordered by path, then filter: first the filters updated
// in place (point updates), then those merged in bulk.
struct Part {
  uint32_t r;
  int op;
  std::vector<Req *> reqs;
  std::vector<uint64_t> off;  // offset of each request's keys in the stage
  uint64_t n = 0;
  std::vector<char> pt;       // update parts: the request is applied in place
  uint64_t n_point = 0;       // keys of the part updated in place (a prefix)
};

struct Round {
  std::vector<Part> parts;
  std::map<int, uint64_t> ins;  // keys inserted per filter id
  std::vector<Req *> closes;
  std::vector<Req *> exports;  // table copies to the caller, after the round
  bool empty() const { return parts.empty() && closes.empty() && exports.empty(); }
};

// A filter set per r over the open filters, rebuilt when membership changes.
struct SetOf {
  qf_set_t *set = nullptr;
  std::vector<int> ids;        // set index -> server id
  std::map<int, uint32_t> idx; // server id -> set index
};

}  // namespace

struct qf_server {
  uint64_t budget, used = 0, max_round;
  std::vector<Slot> slots;
  std::deque<Req *> queue;   // admitted requests, submission order
  std::vector<Req *> done;   // completed, not yet polled
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::thread loop;
  hipStream_t stream = nullptr;
  // a round's parts run on three streams (queries and counts; r = 8 updates;
  // r = 16 updates): they touch different filters or only read, and the two
  // update streams each keep their set's pipeline to one call at a time
  hipStream_t pstream[3] = {nullptr, nullptr, nullptr};
  Stage stage[2];
  std::map<uint32_t, SetOf> sets;  // by r
  bool sets_dirty = true;
  uint64_t rounds = 0, requests = 0, keys = 0, seq = 0;
  uint64_t upd_point = 0, upd_bulk = 0;  // update requests by path
  // loop thread's time (ns): forming rounds, launching them (host side),
  // waiting for the device, completing them (outputs, statuses, closes)
  std::atomic<uint64_t> ns_form{0}, ns_launch{0}, ns_wait{0}, ns_complete{0};
  std::atomic<uint64_t> ns_stage{0};  // of ns_launch: copying keys into the pinned stage
  // serving thread only: per filter id, a bound on its used slots past the
  // last quotient (measured after each update round, plus 3 per key
  // inserted since)
  std::map<int, uint64_t> tail_hi;
  int device = 0;
};

namespace {

// device bytes a filter holds: two table copies, its state words and its
// one-filter pipeline's per-region words (the server never uses that
// pipeline's scratch), plus a margin for its share of the filter sets
uint64_t filter_bytes(uint32_t q, uint32_t r) {
  const uint64_t regions = ((1ull << q) >> std::min<uint32_t>(q, r == 8 ? 13 : 12)) + 64;
  return 2 * qf_table_bytes(q, r) + regions * 72 + (1ull << 20) * 2;
}

void admit_locked(qf_server *s) {
  for (size_t i = 0; i < s->slots.size(); ++i) {
    Slot &sl = s->slots[i];
    if (sl.state != Slot::PENDING || sl.f) continue;
    if (s->used + sl.bytes > s->budget) break;  // admission in open order
    sl.f = qf_create(sl.q, sl.r);
    if (!sl.f) break;
    s->used += sl.bytes;
    sl.state = Slot::OPEN;
    s->sets_dirty = true;
  }
}

int rebuild_sets(qf_server *s) {
  for (auto &kv : s->sets) qf_set_destroy(kv.second.set);
  s->sets.clear();
  std::map<uint32_t, std::vector<qf_t *>> by_r;
  for (size_t i = 0; i < s->slots.size(); ++i) {
    const Slot &sl = s->slots[i];
    if (sl.state != Slot::OPEN) continue;
    SetOf &so = s->sets[sl.r];
    so.idx[static_cast<int>(i)] = static_cast<uint32_t>(so.ids.size());
    so.ids.push_back(static_cast<int>(i));
    by_r[sl.r].push_back(sl.f);
  }
  for (auto &kv : by_r) {
    SetOf &so = s->sets[kv.first];
    so.set = qf_set_create(kv.second.data(), static_cast<uint32_t>(kv.second.size()));
    if (!so.set) return qf_last_error();
    const int rc = qf_set_reserve(so.set, s->max_round, s->stream);
    if (rc) return rc;
  }
  uint32_t nopen = 0;
  for (auto &kv : s->sets) nopen += static_cast<uint32_t>(kv.second.ids.size());
  if (!s->stage[0].alloc_err(nopen) || !s->stage[1].alloc_err(nopen)) return QF_ERR_OOM;
  s->sets_dirty = false;
  return QF_OK;
}

// Take the next round from the queue (lock held): per filter the leading run
// of requests with one operation; a filter with a skipped request takes no
// later request in this round; requests of pending filters wait.
Round form_round_locked(qf_server *s) {
  Round rd;
  std::map<int, int> fop;        // id -> operation taken this round
  std::map<int, bool> blocked;   // id -> a request of it was skipped
  std::map<std::pair<uint32_t, int>, size_t> part_of;
  std::deque<Req *> rest;
  for (Req *q : s->queue) {
    Slot &sl = s->slots[q->id];
    bool take = false;
    if (q->op == OP_CLOSE) {
      // after every earlier request of the filter has completed
      take = !blocked[q->id] && fop.find(q->id) == fop.end();
      if (take) rd.closes.push_back(q);
      blocked[q->id] = true;
      if (!take) rest.push_back(q);
      continue;
    }
    if (q->op == OP_EXPORT) {
      // the same rule as a close, for an admitted filter; later requests of
      // the filter wait for the next round
      take = sl.state == Slot::OPEN && !blocked[q->id] && fop.find(q->id) == fop.end();
      if (take) rd.exports.push_back(q);
      blocked[q->id] = true;
      if (!take) rest.push_back(q);
      continue;
    }
    if (sl.state == Slot::OPEN && !blocked[q->id]) {
      auto it = fop.find(q->id);
      take = it == fop.end() || it->second == q->op;
      if (take) {
        const auto key = std::make_pair(sl.r, q->op);
        auto pit = part_of.find(key);
        if (pit == part_of.end()) {
          part_of[key] = rd.parts.size();
          Part p;
          p.r = sl.r;
          p.op = q->op;
          rd.parts.push_back(p);
          pit = part_of.find(key);
        }
        Part &p = rd.parts[pit->second];
        if (p.n + q->keys.size() > s->max_round) {
          take = false;  // round full for this batch
        } else {
          fop[q->id] = q->op;
          p.off.push_back(p.n);
          p.reqs.push_back(q);
          p.n += q->keys.size();
        }
      }
    }
    if (!take) {
      blocked[q->id] = true;
      rest.push_back(q);
    }
  }
  // a stage holds all parts of a round back to back
  uint64_t total = 0;
  for (Part &p : rd.parts) total += p.n;
  if (total > s->max_round) {
    // keep whole parts while they fit; the rest goes back in order
    uint64_t acc = 0;
    std::vector<Part> keep;
    std::vector<Req *> back;
    for (Part &p : rd.parts) {
      if (acc + p.n <= s->max_round) {
        acc += p.n;
        keep.push_back(p);
      } else {
        for (Req *q : p.reqs) back.push_back(q);
      }
    }
    rd.parts = keep;
    // requests put back keep their submission order relative to the rest
    std::deque<Req *> merged;
    std::vector<Req *> all(rest.begin(), rest.end());
    all.insert(all.end(), back.begin(), back.end());
    std::sort(all.begin(), all.end(), [](Req *a, Req *b) { return a->seq < b->seq; });
    rest.assign(all.begin(), all.end());
  }
  s->queue.swap(rest);
  // a round that closes filters is completed (and the sets rebuilt) before
  // the next one is formed
  if (!rd.closes.empty()) s->sets_dirty = true;
  return rd;
}

uint64_t ns_since(std::chrono::steady_clock::time_point t0) {
  return static_cast<uint64_t>(
      std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count());
}

constexpr unsigned STAGE_THREADS = 8;  // host threads that stage one large part

// Choose each update's path.  A filter's keys of the round are applied in
// place (point updates: one lane per key under region locks) when the filter
// has at least 2^INPLACE_MIN_Q quotients, there are at most
// INPLACE_PER_REGION of them per lock region, and, for inserts, they cannot
// run out of room.  A point update is a chain of dependent device-scope
// steps (lock, plan, shift, fences, unlock) of some 80 us, while the bulk
// merge costs about 5 ps per slot of the filter plus the batch pipeline's
// launches, shared by every filter of the part: measured with 4096 keys at
// load 0.5, in place took 87 us against 317 us merged at 2^26 quotients, but
// the merge won below about 2^23.  Few keys per region keep lanes from
// waiting for each other.  The room test: each key adds at most 3 used
// slots, and the used slots past the last quotient form one stretch whose
// length is bounded by tail_hi, so tail_hi + 3 n + 3 <= E keeps every shift
// inside the table and no key can fail for lack of room (the request stays
// all or nothing; deletes never need room).  The rest go through the bulk
// merge, which rewrites every block of the filter.  The part is reordered
// (in-place filters first, then by filter, each filter's requests in
// submission order) so that each filter's keys lie together.
constexpr uint64_t INPLACE_PER_REGION = 2;
constexpr uint32_t INPLACE_MIN_Q = 23;
void plan_updates(qf_server *s, Round &rd) {
  for (Part &p : rd.parts) {
    if (p.op != OP_INSERT && p.op != OP_DELETE) continue;
    SetOf &so = s->sets[p.r];
    std::map<int, uint64_t> nk;
    for (Req *q : p.reqs) nk[q->id] += q->keys.size();
    std::map<int, char> inplace;
    for (auto &kv : nk) {
      const qf_filter *f = so.set->fs[so.idx[kv.first]];
      const uint64_t n = kv.second, room = f->P - f->N;
      const uint64_t t = s->tail_hi[kv.first];
      inplace[kv.first] = n > 0 && f->q >= INPLACE_MIN_Q && n <= INPLACE_PER_REGION * qf::point_regions(f->P) &&
                          (p.op == OP_DELETE || t + 3 * n + 3 <= room);
      if (p.op == OP_INSERT) {
        rd.ins[kv.first] += n;
        s->tail_hi[kv.first] = t + 3 * n;
      }
    }
    std::stable_sort(p.reqs.begin(), p.reqs.end(), [&inplace](Req *a, Req *b) {
      const char pa = inplace.at(a->id), pb = inplace.at(b->id);
      if (pa != pb) return pa > pb;
      return a->id < b->id;
    });
    p.pt.assign(p.reqs.size(), 0);
    p.n_point = 0;
    uint64_t o = 0;
    for (size_t k = 0; k < p.reqs.size(); ++k) {
      p.off[k] = o;
      o += p.reqs[k]->keys.size();
      p.pt[k] = inplace.at(p.reqs[k]->id);
      if (p.pt[k]) p.n_point = o;
    }
  }
}

// Enqueue a round on the stream (no waiting).
// Copy a part's keys and filter indexes into the pinned stage at base.  A
// large part is split over a few threads by bytes (one core's copy rate
// left the device idle between rounds).
void stage_part(qf_server *s, const Part &p, Stage &st, uint64_t base) {
  const SetOf &so = s->sets.at(p.r);
  std::vector<uint32_t> fi(p.reqs.size());
  for (size_t k = 0; k < p.reqs.size(); ++k) fi[k] = so.idx.at(p.reqs[k]->id);
  auto copy = [&](size_t a, size_t b) {
    for (size_t k = a; k < b; ++k) {
      const Req *q = p.reqs[k];
      const uint64_t o = base + p.off[k];
      std::memcpy(st.keys + o, q->keys.data(), q->keys.size() * 8);
      std::fill(st.fid + o, st.fid + o + q->keys.size(), fi[k]);
    }
  };
  constexpr uint64_t PER_THREAD = 1ull << 16;  // keys (768 KB of staging)
  const unsigned nt = static_cast<unsigned>(std::min<uint64_t>(STAGE_THREADS, p.n / PER_THREAD));
  if (nt < 2 || p.reqs.size() < 2) {
    copy(0, p.reqs.size());
    return;
  }
  // request ranges of about p.n / nt keys each
  std::vector<size_t> cut{0};
  for (size_t k = 0; k < p.reqs.size() && cut.size() < nt; ++k)
    if (p.off[k] >= p.n / nt * cut.size()) cut.push_back(k);
  cut.push_back(p.reqs.size());
  std::vector<std::thread> th;
  for (size_t i = 1; i + 1 < cut.size(); ++i) th.emplace_back(copy, cut[i], cut[i + 1]);
  copy(cut[0], cut[1]);
  for (auto &t : th) t.join();
}

// Stage, send and launch one part on stream ps (stage offset base).
int launch_part(qf_server *s, Part &p, Stage &st, uint64_t base, hipStream_t ps) {
  // each part is staged and sent on its own, so the device starts on the
  // first part while the host stages the next
  const auto t0 = std::chrono::steady_clock::now();
  stage_part(s, p, st, base);
  s->ns_stage += ns_since(t0);
  if (p.n && (hipMemcpyAsync(st.d_keys + base, st.keys + base, p.n * 8, hipMemcpyHostToDevice, ps) != hipSuccess ||
              hipMemcpyAsync(st.d_fid + base, st.fid + base, p.n * 4, hipMemcpyHostToDevice, ps) != hipSuccess))
    return QF_ERR_DEVICE;
  const SetOf &so = s->sets.at(p.r);
  qf_set_t *set = so.set;
  const uint64_t *k = st.d_keys + base;
  const uint32_t *f = st.d_fid + base;
  int rc = QF_OK;
  if (p.op == OP_INSERT || p.op == OP_DELETE) {
    // in place: one launch over the keys of every such filter (errors go
    // to each filter's error word, as a merge's do)
    if (p.n_point &&
        qf::launch_point_multi(set->pipe, set->d_plocks, f, k, p.n_point, p.op == OP_DELETE, ps) != hipSuccess)
      rc = QF_ERR_DEVICE;
    // in bulk: merge only the filters of the rest of the part
    std::vector<uint32_t> act;
    for (size_t a = 0; a < p.reqs.size(); ++a)
      if (!p.pt[a] && !p.reqs[a]->keys.empty()) act.push_back(so.idx.at(p.reqs[a]->id));
    std::sort(act.begin(), act.end());
    act.erase(std::unique(act.begin(), act.end()), act.end());
    const uint64_t np = p.n_point, nb = p.n - p.n_point;
    if (!rc && !act.empty()) {
      if (p.op == OP_INSERT)
        rc = qf_set_insert_some(set, act.data(), static_cast<uint32_t>(act.size()), f + np, k + np, nb, ps);
      else
        rc = qf_set_delete_some(set, act.data(), static_cast<uint32_t>(act.size()), f + np, k + np, nb, nullptr, ps);
    }
  }
  if (p.op == OP_QUERY) {
    rc = qf_set_query_batch(set, f, k, p.n, st.d_out8 + base, ps);
    if (!rc && hipMemcpyAsync(st.out8 + base, st.d_out8 + base, p.n, hipMemcpyDeviceToHost, ps))
      rc = QF_ERR_DEVICE;
  }
  if (p.op == OP_COUNT) {
    rc = qf_set_count_batch(set, f, k, p.n, st.d_out64 + base, ps);
    if (!rc && hipMemcpyAsync(st.out64 + base, st.d_out64 + base, p.n * 8, hipMemcpyDeviceToHost, ps))
      rc = QF_ERR_DEVICE;
  }
  return rc;
}

int launch_round(qf_server *s, Round &rd, Stage &st) {
  plan_updates(s, rd);
  // the part streams start behind everything the main stream holds: the
  // previous round, whose queries may read filters this round updates
  int rc = hipEventRecord(st.start, s->stream) == hipSuccess ? QF_OK : QF_ERR_DEVICE;
  for (hipStream_t ps : s->pstream)
    if (!rc && hipStreamWaitEvent(ps, st.start, 0) != hipSuccess) rc = QF_ERR_DEVICE;
  // the parts of each stream, with their stage offsets (round order)
  std::vector<std::pair<Part *, uint64_t>> by[3];
  uint64_t base = 0;
  for (Part &p : rd.parts) {
    const int si = (p.op == OP_QUERY || p.op == OP_COUNT) ? 0 : (p.r == 8 ? 1 : 2);
    by[si].emplace_back(&p, base);
    base += p.n;
  }
  bool used[3];
  for (int i = 0; i < 3; ++i) {
    used[i] = !by[i].empty();
    for (auto &pb : by[i]) {
      if (!rc) rc = launch_part(s, *pb.first, st, pb.second, s->pstream[i]);
    }
  }
  // the main stream waits for every part stream that took work
  for (int i = 0; i < 3; ++i)
    if (used[i] && (hipEventRecord(st.part_done[i], s->pstream[i]) != hipSuccess ||
                    hipStreamWaitEvent(s->stream, st.part_done[i], 0) != hipSuccess) && !rc)
      rc = QF_ERR_DEVICE;
  // this round's per-filter errors, taken on the stream behind its updates
  bool updates = false;
  for (Part &p : rd.parts) updates |= p.op == OP_INSERT || p.op == OP_DELETE;
  if (!rc && updates && st.nerr) {
    uint32_t o = 0;
    for (auto &kv : s->sets) {
      if (qf::launch_take_errors(kv.second.set->pipe, st.d_err + o, s->stream) != hipSuccess ||
          qf::launch_take_tails(kv.second.set->pipe, st.d_tail + o, s->stream) != hipSuccess)
        rc = QF_ERR_DEVICE;
      o += static_cast<uint32_t>(kv.second.ids.size());
    }
    if (!rc && (hipMemcpyAsync(st.h_err, st.d_err, st.nerr * 8, hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
                hipMemcpyAsync(st.h_tail, st.d_tail, st.nerr * 8, hipMemcpyDeviceToHost, s->stream) != hipSuccess))
      rc = QF_ERR_DEVICE;
  }
  if (hipEventRecord(st.done, s->stream) != hipSuccess && !rc) rc = QF_ERR_DEVICE;
  return rc;
}

// Wait for a launched round, copy outputs, set statuses, run its closes.
// next: the round launched after it, if any (its inserts count against the
// room measured at the end of this one).
void complete_round(qf_server *s, Round &rd, Stage &st, int launch_rc, const Round *next) {
  if (!rd.parts.empty()) {
    const auto t0 = std::chrono::steady_clock::now();
    (void)hipEventSynchronize(st.done);
    s->ns_wait += static_cast<uint64_t>(
        std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count());
  }
  // per-filter errors of this round (updates only)
  std::map<int, int> err;
  bool updates = false;
  for (Part &p : rd.parts) updates |= p.op == OP_INSERT || p.op == OP_DELETE;
  if (updates && launch_rc == QF_OK && st.nerr) {
    uint32_t o = 0;
    for (auto &kv : s->sets) {
      for (size_t i = 0; i < kv.second.ids.size(); ++i) {
        const int id = kv.second.ids[i];
        if (st.h_err[o + i]) err[id] = static_cast<int>(st.h_err[o + i]);
        uint64_t t = static_cast<uint64_t>(st.h_tail[o + i]);
        if (next) {
          auto it = next->ins.find(id);
          if (it != next->ins.end()) t += 3 * it->second;
        }
        s->tail_hi[id] = t;
      }
      o += static_cast<uint32_t>(kv.second.ids.size());
    }
  }
  uint64_t base = 0;
  for (Part &p : rd.parts) {
    for (size_t k = 0; k < p.reqs.size(); ++k) {
      Req *q = p.reqs[k];
      const uint64_t o = base + p.off[k];
      if (q->out && p.op == OP_QUERY) std::memcpy(q->out, st.out8 + o, q->keys.size());
      if (q->out && p.op == OP_COUNT) std::memcpy(q->out, st.out64 + o, q->keys.size() * 8);
      auto e = err.find(q->id);
      q->status = launch_rc ? launch_rc : (e != err.end() && (p.op == OP_INSERT || p.op == OP_DELETE) ? e->second : QF_OK);
    }
    base += p.n;
  }
  // exports read the table as this round left it (the round launched after
  // it holds no request of an exported filter)
  for (Req *e : rd.exports) {
    qf_t *f = s->slots[e->id].f;
    e->status = f ? qf_export(f, static_cast<qf_layout_t *>(e->out), s->stream) : QF_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  for (Req *c : rd.closes) {
    Slot &sl = s->slots[c->id];
    if (sl.f) {
      qf_destroy(sl.f);
      sl.f = nullptr;
      s->used -= sl.bytes;
    }
    sl.state = Slot::CLOSED;
    c->status = QF_OK;
    s->sets_dirty = true;
  }
  if (!rd.closes.empty()) admit_locked(s);
  for (Part &p : rd.parts)
    for (size_t k = 0; k < p.reqs.size(); ++k) {
      s->done.push_back(p.reqs[k]);
      s->keys += p.reqs[k]->keys.size();
      if (p.op == OP_INSERT || p.op == OP_DELETE) ++(p.pt[k] ? s->upd_point : s->upd_bulk);
    }
  for (Req *c : rd.closes) s->done.push_back(c);
  for (Req *e : rd.exports) s->done.push_back(e);
  s->requests += rd.closes.size() + rd.exports.size();
  for (Part &p : rd.parts) s->requests += p.reqs.size();
  s->rounds += 1;
  s->cv_done.notify_all();
}


void serve(qf_server *s) {
  (void)hipSetDevice(s->device);
  Round inflight;
  int inflight_rc = QF_OK;
  int cur = 0;
  bool have = false;
  for (;;) {
    Round rd;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (!have)
        s->cv_work.wait_for(lk, std::chrono::milliseconds(50), [s] { return s->stop || !s->queue.empty(); });
      if (s->stop && s->queue.empty() && !have) break;
      admit_locked(s);
      if (s->sets_dirty && !have) {
        lk.unlock();
        (void)hipStreamSynchronize(s->stream);
        (void)rebuild_sets(s);
        lk.lock();
      }
      if (!s->sets_dirty) {
        const auto t0 = std::chrono::steady_clock::now();
        rd = form_round_locked(s);
        s->ns_form += ns_since(t0);
      }
    }
    int rc = QF_OK;
    if (!rd.parts.empty()) {
      const auto t0 = std::chrono::steady_clock::now();
      rc = launch_round(s, rd, s->stage[cur]);
      s->ns_launch += ns_since(t0);
    }
    if (have) {
      const auto t0 = std::chrono::steady_clock::now();
      const uint64_t w0 = s->ns_wait;
      complete_round(s, inflight, s->stage[cur ^ 1], inflight_rc, rd.empty() ? nullptr : &rd);
      s->ns_complete += ns_since(t0) - (s->ns_wait - w0);
    }
    have = !rd.empty();
    if (have) {
      inflight = rd;
      inflight_rc = rc;
      cur ^= 1;
    }
  }
  (void)hipStreamSynchronize(s->stream);
}

}  // namespace

extern "C" {

qfs_t *qfs_create(uint64_t budget_bytes, uint64_t max_round_keys) {
  if (max_round_keys == 0 || max_round_keys > (1ull << 31)) return nullptr;
  qf_server *s = new (std::nothrow) qf_server();
  if (!s) return nullptr;
  s->budget = budget_bytes;
  s->max_round = max_round_keys;
  (void)hipGetDevice(&s->device);
  bool ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess &&
            s->stage[0].alloc(max_round_keys) && s->stage[1].alloc(max_round_keys);
  for (hipStream_t &ps : s->pstream) ok = ok && hipStreamCreateWithFlags(&ps, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    s->stage[0].release();
    s->stage[1].release();
    if (s->stream) (void)hipStreamDestroy(s->stream);
    for (hipStream_t ps : s->pstream)
      if (ps) (void)hipStreamDestroy(ps);
    delete s;
    return nullptr;
  }
  // the two stages and the sets' scratch (64 B per key, up to two sets)
  s->used = 2 * max_round_keys * 21 + 2 * 64 * max_round_keys;
  s->loop = std::thread(serve, s);
  return s;
}

void qfs_destroy(qfs_t *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->loop.join();
  for (auto &kv : s->sets) qf_set_destroy(kv.second.set);
  for (Slot &sl : s->slots)
    if (sl.f) qf_destroy(sl.f);
  for (Req *q : s->queue) delete q;
  for (Req *q : s->done) delete q;
  s->stage[0].release();
  s->stage[1].release();
  (void)hipStreamDestroy(s->stream);
  for (hipStream_t ps : s->pstream) (void)hipStreamDestroy(ps);
  delete s;
}

int qfs_open(qfs_t *s, uint32_t q, uint32_t r) {
  if (!s || q < 6 || q > QF_Q_MAX || (r != 8 && r != 16)) return QF_ERR_ARG;
  const uint64_t b = filter_bytes(q, r);
  std::lock_guard<std::mutex> lk(s->mu);
  if (b > s->budget) return QF_ERR_BUDGET;
  Slot sl;
  sl.q = q;
  sl.r = r;
  sl.bytes = b;
  s->slots.push_back(sl);
  s->cv_work.notify_all();
  return static_cast<int>(s->slots.size() - 1);
}

int qfs_submit(qfs_t *s, int op, int id, const uint64_t *h_keys, uint64_t n, void *h_out, uint64_t tag) {
  if (!s || op < QFS_INSERT || op > QFS_COUNT || (n && !h_keys)) return QF_ERR_ARG;
  if ((op == QFS_QUERY || op == QFS_COUNT) && n && !h_out) return QF_ERR_ARG;
  Req *q = new (std::nothrow) Req();
  if (!q) return QF_ERR_OOM;
  q->op = op;
  q->id = id;
  q->out = h_out;
  q->tag = tag;
  q->status = QF_OK;
  if (n > s->max_round) {
    delete q;
    return QF_ERR_ARG;
  }
  q->keys.assign(h_keys, h_keys + n);  // (outside the lock: the loop thread waits for it)
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (id < 0 || static_cast<size_t>(id) >= s->slots.size() || s->slots[id].state == Slot::CLOSED ||
        s->slots[id].closing) {
      delete q;
      return QF_ERR_ARG;
    }
    q->seq = s->seq++;
    s->queue.push_back(q);
  }
  s->cv_work.notify_all();
  return QF_OK;
}

int qfs_close(qfs_t *s, int id, uint64_t tag) {
  if (!s) return QF_ERR_ARG;
  Req *q = new (std::nothrow) Req();
  if (!q) return QF_ERR_OOM;
  q->op = OP_CLOSE;
  q->id = id;
  q->out = nullptr;
  q->tag = tag;
  q->status = QF_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (id < 0 || static_cast<size_t>(id) >= s->slots.size() || s->slots[id].closing ||
        s->slots[id].state == Slot::CLOSED) {
      delete q;
      return QF_ERR_ARG;
    }
    s->slots[id].closing = true;
    q->seq = s->seq++;
    s->queue.push_back(q);
  }
  s->cv_work.notify_all();
  return QF_OK;
}

int qfs_export(qfs_t *s, int id, qf_layout_t *out, uint64_t tag) {
  if (!s || !out || !out->occ_words || !out->runend_words || !out->slots || !out->offsets) return QF_ERR_ARG;
  Req *q = new (std::nothrow) Req();
  if (!q) return QF_ERR_OOM;
  q->op = OP_EXPORT;
  q->id = id;
  q->out = out;
  q->tag = tag;
  q->status = QF_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (id < 0 || static_cast<size_t>(id) >= s->slots.size() || s->slots[id].closing ||
        s->slots[id].state == Slot::CLOSED) {
      delete q;
      return QF_ERR_ARG;
    }
    q->seq = s->seq++;
    s->queue.push_back(q);
  }
  s->cv_work.notify_all();
  return QF_OK;
}

int qfs_poll(qfs_t *s, uint64_t *tags, int32_t *status, uint32_t max, int wait_us) {
  if (!s || (max && (!tags || !status))) return QF_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [s] { return !s->done.empty(); });
  uint32_t k = 0;
  while (k < max && !s->done.empty()) {
    Req *q = s->done.front();
    s->done.erase(s->done.begin());
    tags[k] = q->tag;
    status[k] = q->status;
    delete q;
    ++k;
  }
  return static_cast<int>(k);
}

int qfs_stats(qfs_t *s, uint64_t *st) {
  if (!s || !st) return QF_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  uint64_t open = 0, pending = 0;
  for (const Slot &sl : s->slots) {
    open += sl.state == Slot::OPEN;
    pending += sl.state == Slot::PENDING;
  }
  st[0] = s->rounds;
  st[1] = s->requests;
  st[2] = s->keys;
  st[3] = open;
  st[4] = pending;
  st[5] = s->used;
  st[6] = s->budget;
  st[7] = s->queue.size();
  st[8] = s->upd_point;
  st[9] = s->upd_bulk;
  st[10] = s->ns_form;
  st[11] = s->ns_launch;
  st[12] = s->ns_wait;
  st[13] = s->ns_complete;
  st[14] = s->ns_stage;
  return QF_OK;
}

}  // extern "C"
