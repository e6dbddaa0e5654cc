// qf_point.hip -- point updates: insert and delete of one key at a time, in
// place on the current table, from many lanes at once in any order.
//
// What is computed (Sec. 5.2; the point rows of the API table of Sec. 6): each
// operation has exactly the effect of the same key's bulk operation (Sec. 5.1,
// 6.4), so the table is the canonical table of the multiset after all of
// them, whatever the order in which concurrent keys land.  The paper's point
// GQF locks 8192-slot regions (the key's region and the next one) and moves
// slots with its own memmove.  Point queries and counts need no new code: the
// bulk query and count already look each key up on its own (one lane per key,
// no sort), and like the paper's they run in a phase of their own, not beside
// point updates.
//
// How (MI355X design):
//   * Lock regions of 4096 slots, one 32-bit word each (64 bytes apart, so
//     lanes spinning on one lock do not slow the others).  At most one lane
//     per two lock regions is in flight; the other keys wait their turn in a
//     grid-stride loop.  An update locks the region of its quotient and plans
//     its change from the held regions only; where the change (or the plan)
//     needs a slot after them, it takes the next region's lock, in
//     increasing order and keeping what it holds, and plans again.  Nothing
//     after the held regions is read (it may be another lane's update half
//     done), and everything an update reads or writes lies at or after the
//     first slot of its quotient's 64-slot block (runs never start before
//     their quotient), so the held regions cover it.
//   * Insert: the fingerprint's run grows by g slots (a new run or entry: 1;
//     a counter that needs more digits: 1, or 3 for remainder 0 going from
//     count 2 to 3).  Each slot of growth moves the slots from the growth point
//     up to the first empty slot one place right; the run-end bits move with
//     them.  Delete: the run shrinks by d slots, the following runs of the
//     cluster move left, each at most down to its own quotient, until one
//     does not move; freed slots are cleared to 0.  The offsets of the blocks
//     that start inside the changed stretch are recomputed by a walk over its
//     runs.
//   * Table words are plain loads and stores; taking a lock is followed by an
//     agent-scope acquire fence and releasing one preceded by an agent-scope
//     release fence (L2 invalidate / write-back), which makes the holder's
//     writes visible on every XCD.
#include "qf_dev.h"
#include "qf.h"
#include "qf_lib.h"

namespace qf {

constexpr uint32_t PLOCK_LOG = 12;     // slots per lock region, log2
constexpr uint32_t PLOCK_STRIDE = 16;  // lock words are 64 bytes apart (one line each)
constexpr uint32_t PLOCKS_PER_LANE = 2;  // lock regions per lane in flight
// A lane gives up (QF_ERR_STALLED, nothing changed for its key) after this
// many failed tries of a lock: a safety bound that lane counts sized to the
// lock count keep far away.
constexpr uint32_t PMAX_TRIES = 1u << 20;

namespace {

constexpr int NT = 256;

template <typename T>
struct PT {
  Block<T> *b;  // the current table copy
  int64_t N, P, nb;
  uint32_t r;
  uint64_t *state;
  uint32_t *locks;

  __device__ bool occ(int64_t x) const { return (b[x >> 6].occ >> (x & 63)) & 1ull; }
  __device__ uint64_t slot(int64_t j) const { return b[j >> 6].s[j & 63]; }
  __device__ void set_slot(int64_t j, uint64_t v) const { b[j >> 6].s[j & 63] = static_cast<T>(v); }
  __device__ void set_re(int64_t j, bool v) const {
    uint64_t &w = b[j >> 6].rend;
    w = v ? (w | (1ull << (j & 63))) : (w & ~(1ull << (j & 63)));
  }
  __device__ void set_occ(int64_t x, bool v) const {
    uint64_t &w = b[x >> 6].occ;
    w = v ? (w | (1ull << (x & 63))) : (w & ~(1ull << (x & 63)));
  }
  // first occupied quotient in [from, lim] (lim clipped to N - 1), or -1.
  // Every caller bounds the scan by the position that matters: an unbounded
  // scan of a sparse table walks millions of words.
  __device__ int64_t next_occ_le(int64_t from, int64_t lim) const {
    if (lim > N - 1) lim = N - 1;
    if (from > lim) return -1;
    int64_t w = from >> 6;
    const int64_t wl = lim >> 6;
    uint64_t m = b[w].occ & (~0ull << (from & 63));
    for (;;) {
      if (w == wl) m &= ~0ull >> (63 - (lim & 63));
      if (m) return (w << 6) + ctz64(m);
      if (w == wl) return -1;
      m = b[++w].occ;
    }
  }
  // first run end in [from, lim] (lim clipped to P - 1), or -1
  __device__ int64_t next_re_le(int64_t from, int64_t lim) const {
    if (lim > P - 1) lim = P - 1;
    if (from > lim) return -1;
    int64_t w = from >> 6;
    const int64_t wl = lim >> 6;
    uint64_t m = b[w].rend & (~0ull << (from & 63));
    for (;;) {
      if (w == wl) m &= ~0ull >> (63 - (lim & 63));
      if (m) return (w << 6) + ctz64(m);
      if (w == wl) return -1;
      m = b[++w].rend;
    }
  }
  // last run end in [lo, hi], or -1 (0 <= lo <= hi)
  __device__ int64_t prev_re(int64_t lo, int64_t hi) const {
    int64_t w = hi >> 6;
    uint64_t m = b[w].rend & (~0ull >> (63 - (hi & 63)));
    const int64_t wl = lo >> 6;
    for (;;) {
      if (w == wl) m &= ~0ull << (lo & 63);
      if (m) return (w << 6) + msb64(m);
      if (w == wl) return -1;
      m = b[--w].rend;
    }
  }
  // The end of the runs of all quotients below x when it is at or after the
  // first slot i of x's block, else some value in [that end, i - 1]: a run of
  // x starts at max(x, end_before(x) + 1) either way.  From the block offset
  // (which locates the run of the last occupied quotient <= i) and the runs
  // of the block's occupied quotients below x.  hend + 1 when the answer
  // needs slots after hend (then x's run starts after hend too).
  __device__ int64_t end_before(int64_t x, int64_t hend) const {
    const int64_t bi = x >> 6, i = bi << 6;
    const uint64_t ow = b[bi].occ;
    const int64_t O = b[bi].off;
    int64_t c;
    if (!(ow & 1ull)) {
      // the last occupied quotient <= i lies below i: its run ends at i + O
      // when O > 0, at i when O == 0 and slot i ends a run, else before i
      c = (O > 0 || ((b[bi].rend & 1ull) != 0)) ? i + O : i - 1;
    } else {
      // quotient i's run ends at i + O; run ends before that in the block
      // belong to quotients below i
      if (i + O > hend) return hend + 1;
      c = O > 0 ? prev_re(i, i + O - 1) : -1;
      if (c < 0) c = i - 1;
    }
    if (c > hend) return hend + 1;
    uint64_t m = x > i ? (ow & ((1ull << (x - i)) - 1ull)) : 0ull;
    while (m) {
      const int64_t y = i + ctz64(m);
      m &= m - 1;
      c = next_re_le(max(y, c + 1), hend);
      if (c < 0) return hend + 1;
    }
    return c;
  }
  // run-end bits of [sh, z] move one place up: bit j takes bit j - 1 for j in
  // (sh, z], bit sh becomes 0; words from high to low
  __device__ void shift_re_up(int64_t sh, int64_t z) const {
    for (int64_t w = z >> 6; w >= (sh >> 6); --w) {
      const int64_t lo = max(sh, w << 6), hi = min(z, (w << 6) + 63);
      const uint64_t old = b[w].rend;
      const uint64_t below = (w << 6) <= sh ? 0ull : (w > 0 ? (b[w - 1].rend >> 63) : 0ull);
      uint64_t up = (old << 1) | below;
      const uint64_t mask = (~0ull >> (63 - (hi & 63))) & (~0ull << (lo & 63));
      if (lo == sh) up &= ~(1ull << (sh & 63));
      b[w].rend = (old & ~mask) | (up & mask);
    }
  }
};

template <typename T>
struct PSlots {
  const PT<T> *t;
  __device__ uint64_t slot(int64_t j) const { return t->slot(j); }
};
template <typename T>
struct PEmit {
  const PT<T> *t;
  __device__ void emit(int64_t j, uint64_t v) const { t->set_slot(j, v); }
};

__device__ __forceinline__ bool try_lock(uint32_t *l) {
  // (a load first: a taken lock costs no read-modify-write at the line)
  if (__hip_atomic_load(l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
  if (atomicCAS(l, 0u, 1u) != 0u) return false;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the previous holder's writes are visible
  return true;
}
__device__ __forceinline__ void unlock_range(uint32_t *locks, int64_t lo, int64_t hi) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this holder's writes before the lock words
  for (int64_t k = lo; k <= hi; ++k) atomicExch(&locks[k * PLOCK_STRIDE], 0u);
}

// The entry of remainder rem in the run [s, e]: its first slot, slot count
// and count (true), or the slot where a new entry goes (false).
template <typename T>
__device__ bool find_entry(const PT<T> &t, int64_t s, int64_t e, uint64_t rem, int64_t *pos, int64_t *len,
                           uint64_t *cnt) {
  PSlots<T> g{&t};
  int64_t p = s;
  while (p <= e) {
    uint64_t xr, c;
    const int64_t nx = dec_entry(g, p, e, t.r, xr, c);
    if (xr == rem) {
      *pos = p;
      *len = nx - p;
      *cnt = c;
      return true;
    }
    if (xr > rem) break;
    p = nx;
  }
  *pos = p;
  *len = 0;
  *cnt = 0;
  return false;
}

// Offsets of the blocks that start in [from, last] (definition: the end of
// the run of the last occupied quotient <= the block start, minus the start,
// floored at 0).  y0 is the first occupied quotient >= from (or -1) and e0 its
// run end; blocks before y0 take the end eprev of the runs of quotients below
// from.
template <typename T>
__device__ void fix_offsets(const PT<T> &t, int64_t from, int64_t last, int64_t eprev, int64_t y0, int64_t e0) {
  int64_t i = (from + 63) & ~static_cast<int64_t>(63);
  while (i <= last && (y0 < 0 || i < y0)) {
    t.b[i >> 6].off = static_cast<uint32_t>(max(eprev - i, static_cast<int64_t>(0)));
    i += 64;
  }
  int64_t y = y0, ey = e0;
  while (i <= last) {
    const int64_t ny = t.next_occ_le(y + 1, last);  // (only quotients <= last matter)
    while (i <= last && (ny < 0 || i < ny)) {
      t.b[i >> 6].off = static_cast<uint32_t>(max(ey - i, static_cast<int64_t>(0)));
      i += 64;
    }
    if (i > last) break;
    y = ny;
    ey = t.next_re_le(max(ny, ey + 1), last);
  }
}

enum { PT_OK = 0, PT_MORE = 1, PT_FULL = 2, PT_ABSENT = 3, PT_OVF = 4 };

// A lane's changes of the used-slot, distinct and total counts, added to the
// filter's state words once per wave at the end of the launch (one atomic
// per update on three shared words would queue every lane of the chip).
struct Delta {
  int64_t used = 0, dist = 0, total = 0, absent = 0;
};

// One insert of fingerprint (x, rem), with the locks of regions [x's region,
// hi] held: the change, or PT_MORE with *need = the last region the change
// reaches (or read to plan it) when that lies after hi.
template <typename T>
__device__ int insert_step(const PT<T> &t, int64_t x, uint64_t rem, int64_t hi, int64_t *need, Delta &dl) {
  // The plan reads nothing after the held regions' last slot hend: where it
  // would, it asks for the next region (PT_MORE) and is made again.  (What
  // lies after hend may be another lane's update half done; a walk over it
  // can run far past the cluster's true end.)  With the table's last region
  // held, running past it means the table is full.
  const int64_t hend = min(((hi + 1) << PLOCK_LOG) - 1, t.P - 1);
  const bool at_end = hend == t.P - 1;
  const int beyond = at_end ? PT_FULL : PT_MORE;
  *need = hi + 1;
  const bool has = t.occ(x);
  const int64_t eb = t.end_before(x, hend);
  if (eb >= hend) return beyond;
  const int64_t s = max(x, eb + 1);  // where x's run starts (or will)
  int64_t e = s - 1, epos = s, elen = 0;
  uint64_t c = 0;
  bool found = false;
  if (has) {
    e = t.next_re_le(s, hend);
    if (e < 0) return beyond;
    found = find_entry(t, s, e, rem, &epos, &elen, &c);
    if (found && c == ~0ull) return PT_OVF;
  }
  const int64_t sh = found ? epos + elen : epos;  // the growth point
  const int g = found ? static_cast<int>(enc_len(rem, c + 1, t.r)) - static_cast<int>(elen) : 1;
  // z[k]: the (k+1)-th empty slot at or after sh.  The run of the next
  // occupied quotient y after ylast starts at pe + 1 when y <= pe + 1 (the
  // cluster goes on), else slot pe + 1 is empty.
  int64_t z[3] = {0, 0, 0};
  if (g > 0) {
    int64_t pe = e, ylast = x;
    for (int k = 0; k < g; ++k) {
      for (;;) {
        if (pe + 1 > hend) return beyond;
        const int64_t y = t.next_occ_le(ylast + 1, pe + 1);
        if (y < 0) break;
        const int64_t ne = t.next_re_le(pe + 1, hend);
        if (ne < 0) return beyond;
        pe = ne;
        ylast = y;
      }
      z[k] = pe + 1;
      pe = z[k];
    }
  }
  const int64_t last = g > 0 ? z[g - 1] : e;  // (<= hend)
  // the change
  for (int k = 0; k < g; ++k) {
    for (int64_t j = z[k] - 1; j >= sh; --j) t.set_slot(j + 1, t.slot(j));
    t.shift_re_up(sh, z[k]);
  }
  int64_t xe;  // x's run end afterwards
  if (has) {
    xe = e + g;
    if (sh == e + 1 && g > 0) {  // the run grew at its end
      t.set_re(e, false);
      t.set_re(xe, true);
    }
    if (found) {
      PEmit<T> out{&t};
      enc_put(out, epos, rem, c + 1, t.r);
    } else {
      t.set_slot(sh, rem);
    }
  } else {
    t.set_slot(sh, rem);
    t.set_re(sh, true);
    t.set_occ(x, true);
    xe = sh;
  }
  if (g > 0) fix_offsets(t, x, last, eb, x, xe);
  dl.used += g;
  dl.dist += found ? 0 : 1;
  dl.total += 1;
  return PT_OK;
}

// One delete of fingerprint (x, rem), like insert_step.
template <typename T>
__device__ int delete_step(const PT<T> &t, int64_t x, uint64_t rem, int64_t hi, int64_t *need, Delta &dl) {
  // the plan (reads bounded by hend as for insert_step)
  const int64_t hend = min(((hi + 1) << PLOCK_LOG) - 1, t.P - 1);
  const bool at_end = hend == t.P - 1;
  *need = hi + 1;
  if (!t.occ(x)) return PT_ABSENT;
  const int64_t eb = t.end_before(x, hend);
  if (eb >= hend) return at_end ? PT_ABSENT : PT_MORE;  // (at the end: not in a consistent table)
  const int64_t s = max(x, eb + 1);
  const int64_t e = t.next_re_le(s, hend);
  if (e < 0) return at_end ? PT_ABSENT : PT_MORE;
  int64_t epos, elen;
  uint64_t c;
  if (!find_entry(t, s, e, rem, &epos, &elen, &c)) return PT_ABSENT;
  const int64_t nlen = c > 1 ? static_cast<int64_t>(enc_len(rem, c - 1, t.r)) : 0;
  const int64_t d = elen - nlen;                     // slots the run loses
  const bool gone = nlen == 0 && e - s + 1 == elen;  // the run goes
  int64_t last = e;
  if (d > 0) {
    // each following run of the cluster starts at pe_old + 1 and moves to
    // max(its quotient, pe_new + 1); the first that stays ends the walk
    int64_t pe_new = gone ? eb : e - d, pe_old = e, ylast = x;
    for (;;) {
      if (pe_old + 1 > hend) {
        if (at_end) break;  // no slot after the last one
        return PT_MORE;
      }
      const int64_t y = t.next_occ_le(ylast + 1, pe_old + 1);
      if (y < 0) break;
      const int64_t so = pe_old + 1, sn = max(y, pe_new + 1);
      if (sn == so) break;
      const int64_t eo = t.next_re_le(so, hend);
      if (eo < 0) {
        if (at_end) break;  // (not in a consistent table)
        return PT_MORE;
      }
      pe_new = sn + (eo - so);
      pe_old = eo;
      ylast = y;
    }
    last = pe_old;
  }
  // the change: the entry (shorter, or gone) and the rest of x's run
  if (nlen > 0) {
    PEmit<T> out{&t};
    enc_put(out, epos, rem, c - 1, t.r);
  }
  if (d > 0) {
    for (int64_t j = epos + elen; j <= e; ++j) t.set_slot(j - d, t.slot(j));
    t.set_re(e, false);
    if (gone)
      t.set_occ(x, false);
    else
      t.set_re(e - d, true);
    // the following runs, moved left in order; the gap a run leaves before
    // the next one's new start is cleared
    int64_t pn = gone ? eb : e - d, po = e, ylast = x, e1 = -1;
    for (;;) {
      const int64_t y = t.next_occ_le(ylast + 1, po + 1);
      if (y < 0) break;
      const int64_t so = po + 1, sn = max(y, pn + 1);
      if (sn == so) break;
      const int64_t eo = t.next_re_le(so, last);
      if (eo < 0) break;
      for (int64_t j = pn + 1; j < sn; ++j) t.set_slot(j, 0);
      for (int64_t j = so; j <= eo; ++j) t.set_slot(sn + (j - so), t.slot(j));
      const int64_t en = sn + (eo - so);
      t.set_re(eo, false);
      t.set_re(en, true);
      if (e1 < 0) e1 = en;
      pn = en;
      po = eo;
      ylast = y;
    }
    for (int64_t j = pn + 1; j <= po; ++j) t.set_slot(j, 0);
    if (gone)
      fix_offsets(t, x, po, eb, t.next_occ_le(x + 1, po), e1);
    else
      fix_offsets(t, x, po, eb, x, e - d);
    dl.used -= d;
  }
  dl.dist -= nlen == 0 ? 1 : 0;
  dl.total -= 1;
  return PT_OK;
}

// One update of key: QF_OK, QF_ERR_FULL, QF_ERR_COUNT_OVERFLOW or
// QF_ERR_STALLED (nothing changed), or 1 for a delete of a fingerprint that is
// not stored.
template <typename T>
__device__ int point_update(const PT<T> &t, uint32_t q, uint64_t key, bool del, Delta &dl) {
  const uint32_t p = q + t.r;
  const uint64_t fp = mix64(key) & (p >= 64 ? ~0ull : ((1ull << p) - 1ull));
  const int64_t x = static_cast<int64_t>(fp >> t.r);
  const uint64_t rem = fp & ((1ull << t.r) - 1ull);
  const int64_t R0 = x >> PLOCK_LOG;
  // Locks are taken in increasing region order and kept until the update is
  // done: a lane waits only for the lock after the ones it holds, so no
  // chain of waiting lanes closes a cycle.  The loop has one back edge and
  // every lane takes one step per trip (try the next lock; or plan, and
  // apply and release if nothing more is needed): a lane that waits never
  // keeps a lane of its own wave that holds that lock from finishing.  (A
  // loop that spun on one lock by itself could.)
  int64_t hi = R0 - 1, want = R0;
  uint32_t backoff = 0, tries = 0;
  int rc = PT_MORE;
  do {
    bool blocked = false;
    while (hi < want) {
      if (!try_lock(&t.locks[(hi + 1) * PLOCK_STRIDE])) {
        blocked = true;
        break;
      }
      ++hi;
    }
    if (!blocked) {
      int64_t need = want;
      rc = del ? delete_step(t, x, rem, hi, &need, dl) : insert_step(t, x, rem, hi, &need, dl);
      // one more region per plan: the plan is exact up to the held regions'
      // end, and what it read beyond may be another lane's update half done
      // (taking every lock such a plan asks for could hold most of the table)
      if (rc == PT_MORE)
        want = hi + 1;
      else
        unlock_range(t.locks, R0, hi);
      backoff = 0;
    } else {
      if (++tries >= PMAX_TRIES) {
        if (hi >= R0) unlock_range(t.locks, R0, hi);
        return QF_ERR_STALLED;
      }
      for (uint32_t k = 0; k <= backoff; ++k) __builtin_amdgcn_s_sleep(2);
      backoff = min(2 * backoff + 1, 63u);
    }
  } while (rc == PT_MORE);
  if (rc == PT_FULL) return QF_ERR_FULL;
  if (rc == PT_OVF) return QF_ERR_COUNT_OVERFLOW;
  if (rc == PT_ABSENT) return 1;
  return QF_OK;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_point(Block<T> *b0, Block<T> *b1, PT<T> t, uint32_t q,
                                              const uint64_t *__restrict__ keys, uint64_t n, int del,
                                              int32_t *status, uint64_t *not_found) {
  t.b = (t.state[ST_CUR] & 1ull) ? b1 : b0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  Delta dl;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride) {
    const int rc = point_update(t, q, keys[i], del != 0, dl);
    if (rc == 1) {
      ++dl.absent;
    } else if (rc != QF_OK) {
      atomicCAS(reinterpret_cast<ull *>(&t.state[ST_ERR]), 0ull, static_cast<ull>(static_cast<int64_t>(rc)));
    }
    if (status) status[i] = rc;
  }
  // every lane of the (full) work-group gets here: sum over the wave
  for (int m = 32; m >= 1; m >>= 1) {
    dl.used += __shfl_xor(dl.used, m);
    dl.dist += __shfl_xor(dl.dist, m);
    dl.total += __shfl_xor(dl.total, m);
    dl.absent += __shfl_xor(dl.absent, m);
  }
  if ((threadIdx.x & 63) == 0) {
    if (dl.used) atomic_add_u64(&t.state[ST_USED], static_cast<uint64_t>(dl.used));
    if (dl.dist) atomic_add_u64(&t.state[ST_DIST], static_cast<uint64_t>(dl.dist));
    if (dl.total) atomic_add_u64(&t.state[ST_TOTAL], static_cast<uint64_t>(dl.total));
    if (not_found && dl.absent) atomic_add_u64(not_found, static_cast<uint64_t>(dl.absent));
  }
}

// Point updates over a filter set: key i goes to filter fid[i], one lane per
// key.  A filter's keys lie together, so a wave's lanes mostly share one
// filter: the statistics are summed per filter over the wave (one atomic
// per filter and word) rather than per lane.
template <typename T>
__global__ __launch_bounds__(NT) void k_point_multi(const FDesc *__restrict__ desc, uint32_t *const *__restrict__ locks,
                                                    const uint32_t *__restrict__ fid,
                                                    const uint64_t *__restrict__ keys, uint64_t n, int del) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x;
  const bool valid = i < n;
  uint32_t f = 0;
  Delta dl;
  if (valid) {
    f = fid[i];
    const FDesc &d = desc[f];
    PT<T> t;
    t.b = static_cast<Block<T> *>(d.blk[d.state[ST_CUR] & 1ull]);
    t.N = d.N;
    t.P = d.P;
    t.nb = d.nblocks;
    t.r = d.r;
    t.state = d.state;
    t.locks = locks[f];
    const int rc = point_update(t, d.q, keys[i], del != 0, dl);
    if (rc != QF_OK && rc != 1)
      atomicCAS(reinterpret_cast<ull *>(&d.state[ST_ERR]), 0ull, static_cast<ull>(static_cast<int64_t>(rc)));
  }
  // per filter present in the wave: its lanes' sums, added by its first lane
  const int lane = threadIdx.x & 63;
  uint64_t left = __ballot(valid);
  while (left) {
    const int lead = __builtin_ctzll(left);
    const uint32_t f0 = static_cast<uint32_t>(__shfl(static_cast<int>(f), lead));
    const bool mine = valid && f == f0;
    const uint64_t grp = __ballot(mine);
    int64_t u = mine ? dl.used : 0, c = mine ? dl.dist : 0, tt = mine ? dl.total : 0;
    for (int m = 32; m >= 1; m >>= 1) {
      u += __shfl_xor(u, m);
      c += __shfl_xor(c, m);
      tt += __shfl_xor(tt, m);
    }
    if (lane == lead) {
      uint64_t *st = desc[f0].state;
      if (u) atomic_add_u64(&st[ST_USED], static_cast<uint64_t>(u));
      if (c) atomic_add_u64(&st[ST_DIST], static_cast<uint64_t>(c));
      if (tt) atomic_add_u64(&st[ST_TOTAL], static_cast<uint64_t>(tt));
    }
    left &= ~grp;
  }
}

template <typename T>
hipError_t point_t(qf_filter *f, const uint64_t *keys, uint64_t n, int del, int32_t *status, uint64_t *not_found,
                   hipStream_t s) {
  PT<T> t;
  t.b = nullptr;
  t.N = static_cast<int64_t>(f->N);
  t.P = static_cast<int64_t>(f->P);
  t.nb = static_cast<int64_t>(f->nblocks);
  t.r = f->r;
  t.state = f->state;
  t.locks = f->plocks;
  // One lane per key, but no more lanes in flight than one per two lock
  // regions (keys beyond go round again): at most one update per region runs
  // at a time, and a wave's lanes that took locks in one trip share its
  // fences, so fewer lanes, each more likely to find its lock free, measured
  // faster than more (2^28 slots, fill to 0.9) at any fill.
  const uint64_t regions = (f->P >> PLOCK_LOG) + 1;
  const uint64_t cap = max((regions / PLOCKS_PER_LANE + NT - 1) / NT, static_cast<uint64_t>(1));
  const uint64_t g = (n + NT - 1) / NT;
  const uint32_t grid = static_cast<uint32_t>(g < cap ? g : cap);
  k_point<T><<<grid, NT, 0, s>>>(static_cast<Block<T> *>(f->blk[0]), static_cast<Block<T> *>(f->blk[1]), t, f->q,
                                 keys, n, del, status, not_found);
  return hipGetLastError();
}

}  // namespace

uint64_t point_lock_words(uint64_t P) { return ((P >> PLOCK_LOG) + 2) * PLOCK_STRIDE; }

uint64_t point_regions(uint64_t P) { return (P >> PLOCK_LOG) + 1; }

hipError_t launch_point_multi(const Pipe &p, uint32_t *const *locks, const uint32_t *fid, const uint64_t *keys,
                              uint64_t n, int del, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = static_cast<uint32_t>((n + NT - 1) / NT);
  if (p.r == 8)
    k_point_multi<uint8_t><<<grid, NT, 0, s>>>(p.d_desc, locks, fid, keys, n, del);
  else
    k_point_multi<uint16_t><<<grid, NT, 0, s>>>(p.d_desc, locks, fid, keys, n, del);
  return hipGetLastError();
}

hipError_t launch_point(qf_filter *f, const uint64_t *keys, uint64_t n, int del, int32_t *status,
                        uint64_t *not_found, hipStream_t s) {
  if (f->r == 8) return point_t<uint8_t>(f, keys, n, del, status, not_found, s);
  return point_t<uint16_t>(f, keys, n, del, status, not_found, s);
}

}  // namespace qf
