// tcf.hip -- the two-choice filter (Sec. 4): the point form (Algorithm 1 with
// the shortcut and the backing table of Sec. 4.1) and the bulk form
// (Sec. 4.2), behind the C ABI of include/tcf.h.
//
// MI355X design:
//   * Point: one lane per key, 64 keys in flight per wave, instead of a
//     cooperative group per key.  A 32-byte block is two 16-byte loads into
//     registers and its 16 tags are tested four at a time with exact SWAR
//     tests on 64-bit words, so no cross-lane ballot is needed.  A slot is
//     taken with a 64-bit compare-and-swap of the word that holds it; a failed
//     swap means another lane's write to that word succeeded, so the lane
//     takes the word the swap returned and tries again (lock-free, and no
//     lane ever waits on another).
//   * Bulk: the batch is sorted by (primary block, tag, secondary block) with
//     the library's radix sort; one lane per block plans its shortcut count;
//     the other items (none while every block is below 3/4) choose a block,
//     are packed, and are sorted again by (chosen block, tag, other block); one wave per block merges its three sorted lists
//     (tags held, shortcut items, chosen items) by ranks -- each element's
//     output index is its own index plus its rank in the other two lists,
//     found by binary search in LDS -- and writes the 256-byte block back with
//     coalesced stores.  Items a block cannot take go to the end of the
//     backing array, which is then sorted again.
#include "qf.h"
#include "qf_dev.h"
#include "qf_lib.h"
#include "tcf.h"

#include <new>
#include <utility>

namespace tcf {
namespace {

using qf::ctz64;
using qf::mix64;
using qf::popc64;
typedef unsigned long long ull;

constexpr int NT = 256;
constexpr uint32_t PB = 16, BB = 128;          // tags per point / bulk block
constexpr uint32_t SHORT_P = 12, SHORT_B = 96;  // 3/4 of a block
constexpr uint32_t MAX_PROBES = 20;
constexpr uint64_t GOLD = 0x9E3779B97F4A7C15ull;
constexpr uint64_t BK_TOMB = ~0ull;
constexpr uint64_t SENT = ~0ull;  // sorts after every real key
constexpr uint16_t EMPTY_B = 0xFFFF;

// device state words
enum { TS_ERR = 0, TS_HELD = 1, TS_BACK = 2, TS_OVER = 3, TS_OVPOS = 4, TS_REMOVED = 5, TS_CHOSEN = 6, TS_WORDS = 8 };

// ---- hash ------------------------------------------------------------------
struct TK {
  uint32_t b1, b2, tag;
  uint64_t h2;
};
__device__ __forceinline__ TK key_of(uint64_t key, uint64_t nb) {
  const uint64_t h = mix64(key);
  uint32_t tag = static_cast<uint32_t>(h & 0xFFFFull);
  tag = tag == 0 ? 1u : (tag == 0xFFFFu ? 0xFFFEu : tag);
  TK k;
  k.tag = tag;
  k.b1 = static_cast<uint32_t>(((h >> 32) * nb) >> 32);
  k.h2 = mix64(h ^ GOLD);
  k.b2 = static_cast<uint32_t>(((k.h2 >> 32) * nb) >> 32);
  return k;
}
__device__ __forceinline__ uint64_t pair_of(uint32_t a, uint32_t b, uint32_t tag) {
  const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
  return (lo << 40) | (static_cast<uint64_t>(tag) << 24) | hi;
}
__device__ __forceinline__ uint64_t comp_of(uint32_t b1, uint32_t tag, uint32_t b2) {
  return (static_cast<uint64_t>(b1) << 40) | (static_cast<uint64_t>(tag) << 24) | b2;
}

// ---- 16-bit lanes of a 64-bit word (exact: no carry crosses a lane) --------
constexpr uint64_t L16 = 0x0001000100010001ull, H16 = 0x8000800080008000ull, M15 = 0x7FFF7FFF7FFF7FFFull;
__device__ __forceinline__ uint64_t nz16(uint64_t x) { return (((x & M15) + M15) | x) & H16; }
// lanes holding a tag (neither 0 nor 0xFFFF)
__device__ __forceinline__ uint64_t used16(uint64_t x) { return nz16(x) & nz16(~x); }
__device__ __forceinline__ uint64_t free16(uint64_t x) { return ~used16(x) & H16; }
__device__ __forceinline__ uint64_t eq16(uint64_t x, uint32_t tag) { return ~nz16(x ^ (tag * L16)) & H16; }

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}
// Sum over the work-group (every thread of it must call), valid in thread 0:
// statistics go to shared words with one atomic per work-group, since
// millions of same-address atomics (one per wave) queue for milliseconds.
__device__ __forceinline__ int64_t group_sum(int64_t v) {
  __shared__ int64_t part[NT / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) t += part[w];
  __syncthreads();
  return t;
}

// ---- point form --------------------------------------------------------------
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

struct Blk {
  uint64_t w0, w1, w2, w3;
};
__device__ __forceinline__ Blk load_blk(const uint64_t *p) {
  const u64x2 x = reinterpret_cast<const u64x2 *>(p)[0], y = reinterpret_cast<const u64x2 *>(p)[1];
  return Blk{x.x, x.y, y.x, y.y};
}
__device__ __forceinline__ int held_of(const Blk &b) {
  return popc64(used16(b.w0)) + popc64(used16(b.w1)) + popc64(used16(b.w2)) + popc64(used16(b.w3));
}
__device__ __forceinline__ void set_word(Blk &b, int k, uint64_t v) {
  if (k == 0) b.w0 = v;
  else if (k == 1) b.w1 = v;
  else if (k == 2) b.w2 = v;
  else b.w3 = v;
}

// Takes the lowest free slot (empty or tombstone) of the block at p for tag;
// false when it has none.
__device__ bool put_tag(uint64_t *p, Blk &b, uint32_t tag) {
  for (;;) {
    const uint64_t f0 = free16(b.w0), f1 = free16(b.w1), f2 = free16(b.w2), f3 = free16(b.w3);
    int k;
    uint64_t wk, fk;
    if (f0) {
      k = 0, wk = b.w0, fk = f0;
    } else if (f1) {
      k = 1, wk = b.w1, fk = f1;
    } else if (f2) {
      k = 2, wk = b.w2, fk = f2;
    } else if (f3) {
      k = 3, wk = b.w3, fk = f3;
    } else {
      return false;
    }
    const int sh = ctz64(fk) - 15;  // lane j's flag is bit 16 j + 15
    const uint64_t nv = (wk & ~(0xFFFFull << sh)) | (static_cast<uint64_t>(tag) << sh);
    const uint64_t old = atomicCAS(reinterpret_cast<ull *>(p + k), static_cast<ull>(wk), static_cast<ull>(nv));
    if (old == wk) return true;
    set_word(b, k, old);
  }
}

// Overwrites the lowest slot holding tag with a tombstone; false if none.
__device__ bool drop_tag(uint64_t *p, Blk &b, uint32_t tag) {
  for (;;) {
    const uint64_t e0 = eq16(b.w0, tag), e1 = eq16(b.w1, tag), e2 = eq16(b.w2, tag), e3 = eq16(b.w3, tag);
    int k;
    uint64_t wk, ek;
    if (e0) {
      k = 0, wk = b.w0, ek = e0;
    } else if (e1) {
      k = 1, wk = b.w1, ek = e1;
    } else if (e2) {
      k = 2, wk = b.w2, ek = e2;
    } else if (e3) {
      k = 3, wk = b.w3, ek = e3;
    } else {
      return false;
    }
    const int sh = ctz64(ek) - 15;
    const uint64_t nv = wk | (0xFFFFull << sh);
    const uint64_t old = atomicCAS(reinterpret_cast<ull *>(p + k), static_cast<ull>(wk), static_cast<ull>(nv));
    if (old == wk) return true;
    set_word(b, k, old);
  }
}

__device__ __forceinline__ bool has_tag(const Blk &b, uint32_t tag) {
  return (eq16(b.w0, tag) | eq16(b.w1, tag) | eq16(b.w2, tag) | eq16(b.w3, tag)) != 0;
}

// backing table (point): probe j at (a + j s) mod nbt
__device__ bool bk_put(uint64_t *bk, uint64_t nbt, const TK &k) {
  const uint64_t pk = pair_of(k.b1, k.b2, k.tag), m = nbt - 1;
  const uint64_t a = k.h2 & m, s = ((k.h2 >> 16) & m) | 1ull;
  for (uint32_t j = 0; j < MAX_PROBES; ++j) {
    ull *e = reinterpret_cast<ull *>(bk + ((a + j * s) & m));
    uint64_t v = *e;
    while (v == 0 || v == BK_TOMB) {
      const uint64_t old = atomicCAS(e, static_cast<ull>(v), static_cast<ull>(pk));
      if (old == v) return true;
      v = old;
    }
  }
  return false;
}
__device__ bool bk_find(const uint64_t *bk, uint64_t nbt, const TK &k) {
  const uint64_t pk = pair_of(k.b1, k.b2, k.tag), m = nbt - 1;
  const uint64_t a = k.h2 & m, s = ((k.h2 >> 16) & m) | 1ull;
  for (uint32_t j = 0; j < MAX_PROBES; ++j) {
    const uint64_t v = bk[(a + j * s) & m];
    if (v == 0) return false;
    if (v == pk) return true;
  }
  return false;
}
__device__ bool bk_drop(uint64_t *bk, uint64_t nbt, const TK &k) {
  const uint64_t pk = pair_of(k.b1, k.b2, k.tag), m = nbt - 1;
  const uint64_t a = k.h2 & m, s = ((k.h2 >> 16) & m) | 1ull;
  for (uint32_t j = 0; j < MAX_PROBES; ++j) {
    ull *e = reinterpret_cast<ull *>(bk + ((a + j * s) & m));
    uint64_t v = *e;
    if (v == 0) return false;
    while (v == pk) {
      const uint64_t old = atomicCAS(e, static_cast<ull>(pk), static_cast<ull>(BK_TOMB));
      if (old == pk) return true;
      v = old;
    }
  }
  return false;
}

__global__ __launch_bounds__(NT) void k_point_insert(uint64_t *tbl, uint64_t nb, uint64_t *bk, uint64_t nbt,
                                                     const uint64_t *__restrict__ keys, uint64_t n,
                                                     int32_t *status, uint64_t *state) {
  int64_t dheld = 0, dback = 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride) {
    const TK k = key_of(keys[i], nb);
    uint64_t *p1 = tbl + 4ull * k.b1, *p2 = tbl + 4ull * k.b2;
    Blk x = load_blk(p1), y{0, 0, 0, 0};
    bool have_y = false, primary_first = true;
    if (held_of(x) >= static_cast<int>(SHORT_P)) {  // no shortcut: the emptier candidate
      y = load_blk(p2);
      have_y = true;
      primary_first = held_of(x) <= held_of(y);
    }
    bool done;
    if (primary_first) {
      done = put_tag(p1, x, k.tag);
      if (!done) {
        if (!have_y) y = load_blk(p2);
        done = put_tag(p2, y, k.tag);
      }
    } else {
      done = put_tag(p2, y, k.tag) || put_tag(p1, x, k.tag);
    }
    int rc = QF_OK;
    if (done) {
      ++dheld;
    } else if (bk_put(bk, nbt, k)) {
      ++dback;
    } else {
      rc = QF_ERR_FULL;
      atomicCAS(reinterpret_cast<ull *>(&state[TS_ERR]), 0ull, static_cast<ull>(static_cast<int64_t>(rc)));
    }
    if (status) status[i] = rc;
  }
  dheld = group_sum(dheld);
  dback = group_sum(dback);
  if (threadIdx.x == 0) {
    if (dheld) qf::atomic_add_u64(&state[TS_HELD], static_cast<uint64_t>(dheld));
    if (dback) qf::atomic_add_u64(&state[TS_BACK], static_cast<uint64_t>(dback));
  }
}

__global__ __launch_bounds__(NT) void k_point_query(const uint64_t *tbl, uint64_t nb, const uint64_t *bk,
                                                    uint64_t nbt, const uint64_t *__restrict__ keys, uint64_t n,
                                                    uint8_t *__restrict__ out) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride) {
    const TK k = key_of(keys[i], nb);
    const Blk x = load_blk(tbl + 4ull * k.b1), y = load_blk(tbl + 4ull * k.b2);
    bool hit = has_tag(x, k.tag) || has_tag(y, k.tag);
    if (!hit) hit = bk_find(bk, nbt, k);
    out[i] = hit ? 1 : 0;
  }
}

__global__ __launch_bounds__(NT) void k_point_delete(uint64_t *tbl, uint64_t nb, uint64_t *bk, uint64_t nbt,
                                                     const uint64_t *__restrict__ keys, uint64_t n,
                                                     uint64_t *not_found, uint64_t *state) {
  int64_t dheld = 0, dback = 0, absent = 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride) {
    const TK k = key_of(keys[i], nb);
    uint64_t *p1 = tbl + 4ull * k.b1, *p2 = tbl + 4ull * k.b2;
    Blk x = load_blk(p1);
    if (drop_tag(p1, x, k.tag)) {
      ++dheld;
      continue;
    }
    Blk y = load_blk(p2);
    if (k.b2 != k.b1 && drop_tag(p2, y, k.tag)) {
      ++dheld;
      continue;
    }
    if (bk_drop(bk, nbt, k))
      ++dback;
    else
      ++absent;
  }
  dheld = group_sum(dheld);
  dback = group_sum(dback);
  absent = group_sum(absent);
  if (threadIdx.x == 0) {
    if (dheld) qf::atomic_add_u64(&state[TS_HELD], static_cast<uint64_t>(-dheld));
    if (dback) qf::atomic_add_u64(&state[TS_BACK], static_cast<uint64_t>(-dback));
    if (absent && not_found) qf::atomic_add_u64(not_found, static_cast<uint64_t>(absent));
  }
}

// ---- bulk form ---------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_compose(const uint64_t *__restrict__ keys, uint64_t n, uint64_t nb,
                                                uint64_t *__restrict__ out) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x;
  if (i >= n) return;
  const TK k = key_of(keys[i], nb);
  out[i] = comp_of(k.b1, k.tag, k.b2);
}

// first index in a[0, n) whose value is >= v
__device__ __forceinline__ uint64_t lower_bound(const uint64_t *a, uint64_t n, uint64_t v) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}
template <typename T>
__device__ __forceinline__ uint32_t lb16(const T *a, uint32_t n, uint32_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}
template <typename T>
__device__ __forceinline__ uint32_t ub16(const T *a, uint32_t n, uint32_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// gs[b] = first index of the sorted keys (block in the top 24 bits; SENT
// entries last) whose block is >= b, for b in [0, nb]
__global__ __launch_bounds__(NT) void k_gbounds(const uint64_t *__restrict__ s, uint64_t n, uint64_t nb,
                                                uint32_t *__restrict__ gs) {
  const uint64_t b = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x;
  if (b > nb) return;
  gs[b] = static_cast<uint32_t>(lower_bound(s, n, b == nb ? SENT : (b << 40)));
}

// the same bounds from the other side, for batches at least as large as the
// block count: entry i (i in [0, n]) writes gs[b] = i for every block b in
// (block of entry i - 1, block of entry i], SENT and the end counting as nb
__global__ __launch_bounds__(NT) void k_gbounds_scatter(const uint64_t *__restrict__ s, uint64_t n, uint64_t nb,
                                                        uint32_t *__restrict__ gs) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x;
  if (i > n) return;
  const auto blk = [&](uint64_t j) -> uint64_t { return s[j] == SENT ? nb : (s[j] >> 40); };
  const uint64_t lo = i == 0 ? 0 : blk(i - 1) + 1, hi = i == n ? nb : blk(i);
  for (uint64_t b = lo; b <= hi; ++b) gs[b] = static_cast<uint32_t>(i);
}

// per block: shortcut count s and f = held + s
// (16 lanes per block: each counts the tags among 8 slots with one 16-byte
// load, so a block's count takes one round trip, not a chain of
// binary-search probes; a block's tags are sorted with the empty slots
// last, so the count is also the first empty position)
__global__ __launch_bounds__(NT) void k_plan(const uint16_t *__restrict__ slots, uint64_t nb,
                                             const uint32_t *__restrict__ gs, uint32_t *__restrict__ ps,
                                             uint32_t *__restrict__ pf) {
  const uint64_t t = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x;
  const uint64_t b = t / 16;
  const uint32_t l = static_cast<uint32_t>(t % 16);
  uint32_t c = 0;
  if (b < nb) {
    const u64x2 v = reinterpret_cast<const u64x2 *>(slots + b * BB)[l];
    c = static_cast<uint32_t>(popc64(nz16(~v.x)) + popc64(nz16(~v.y)));
  }
  for (int m = 8; m >= 1; m >>= 1) c += __shfl_xor(c, m);  // (all lanes: the groups are aligned)
  if (b >= nb || l != 0) return;
  const uint32_t held = c;
  const uint32_t cnt = gs[b + 1] - gs[b];
  const uint32_t room = held < SHORT_B ? SHORT_B - held : 0;
  const uint32_t s = cnt < room ? cnt : room;
  ps[b] = s;
  pf[b] = held + s;
}

// The items not shortcut, with their keys for the second sort
// (chosen << 40 | tag << 24 | other), packed at out[0, state[TS_CHOSEN]) in
// no particular order (the sort orders them): one range per work-group.
// (CHOOSE_K items per lane, so that a work-group's one reservation in the
// output covers NT * CHOOSE_K items: same-address atomics from every
// work-group serialise at about 12 ns each, which bounded the kernel when
// each work-group took NT items)
constexpr int CHOOSE_K = 8;
__global__ __launch_bounds__(NT) void k_choose(const uint64_t *__restrict__ s1, uint64_t n,
                                               const uint32_t *__restrict__ gs, const uint32_t *__restrict__ ps,
                                               const uint32_t *__restrict__ pf, uint64_t *__restrict__ out,
                                               uint64_t *state) {
  __shared__ uint32_t wc[NT / 64];
  __shared__ uint64_t base;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * NT * CHOOSE_K + threadIdx.x;
  bool chosen[CHOOSE_K];
  uint64_t key[CHOOSE_K];
  uint32_t mine = 0;  // the wave's chosen items
  uint64_t bal[CHOOSE_K];
#pragma unroll
  for (int k = 0; k < CHOOSE_K; ++k) {
    const uint64_t i = i0 + static_cast<uint64_t>(k) * NT;
    chosen[k] = false;
    key[k] = 0;
    if (i < n) {
      const uint64_t c = s1[i];
      const uint32_t b1 = static_cast<uint32_t>(c >> 40), tag = static_cast<uint32_t>((c >> 24) & 0xFFFF);
      const uint32_t b2 = static_cast<uint32_t>(c & 0xFFFFFF);
      if (i - gs[b1] >= ps[b1]) {
        chosen[k] = true;
        key[k] = pf[b1] <= pf[b2] ? comp_of(b1, tag, b2) : comp_of(b2, tag, b1);
      }
    }
    bal[k] = __ballot(chosen[k]);
    mine += static_cast<uint32_t>(popc64(bal[k]));
  }
  if (lane == 0) wc[w] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int k = 0; k < NT / 64; ++k) {
      const uint32_t c = wc[k];
      wc[k] = tot;
      tot += c;
    }
    base = tot ? qf::atomic_add_u64(&state[TS_CHOSEN], tot) : 0;
  }
  __syncthreads();
  uint64_t at = base + wc[w];
#pragma unroll
  for (int k = 0; k < CHOOSE_K; ++k) {
    if (chosen[k]) out[at + popc64(bal[k] & ((1ull << lane) - 1ull))] = key[k];
    at += static_cast<uint64_t>(popc64(bal[k]));
  }
}

// items beyond each block's free slots: their total in state[TS_OVER]
__global__ __launch_bounds__(NT) void k_over(uint64_t nb, const uint32_t *__restrict__ gs2,
                                             const uint32_t *__restrict__ pf, uint64_t *state) {
  const uint64_t b = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x;
  int64_t over = 0;
  if (b < nb) {
    const uint32_t got = gs2[b + 1] - gs2[b], room = BB - pf[b];
    over = got > room ? got - room : 0;
  }
  over = group_sum(over);
  if (threadIdx.x == 0 && over) qf::atomic_add_u64(&state[TS_OVER], static_cast<uint64_t>(over));
}

// One wave per block: the sorted union of the tags held, the shortcut items
// and the chosen items that fit; chosen items that do not fit go to the
// backing array after its bn entries.
__global__ __launch_bounds__(NT) void k_merge_blocks(uint16_t *slots, uint64_t nb, const uint64_t *__restrict__ s1,
                                                     const uint32_t *__restrict__ gs1, const uint64_t *__restrict__ s2,
                                                     const uint32_t *__restrict__ gs2,
                                                     const uint32_t *__restrict__ ps,
                                                     const uint32_t *__restrict__ pf, uint64_t *bk, uint64_t bn,
                                                     uint64_t *state) {
  __shared__ uint16_t A[4][BB], S[4][BB], C[4][BB], O[4][BB];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t b = static_cast<uint64_t>(blockIdx.x) * 4 + w;
  uint32_t ha = 0, ns = 0, nc = 0;
  // the block's plan and list bounds, all requested together (then the
  // block and its two lists in one more round trip)
  uint32_t p_s = 0, p_f = 0, g1 = 0, g2 = 0, g2e = 0;
  if (b < nb) {
    p_s = ps[b];
    p_f = pf[b];
    g1 = gs1[b];
    g2 = gs2[b];
    g2e = gs2[b + 1];
  }
  // (a block that receives nothing is neither read nor written)
  const bool touched = b < nb && (p_s != 0 || g2e != g2);
  if (touched) {
    ns = p_s;
    ha = p_f - ns;
    const uint32_t got = g2e - g2, room = BB - p_f;
    nc = got < room ? got : room;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(slots + b * BB);
    const uint32_t v = src[lane];
    A[w][2 * lane] = static_cast<uint16_t>(v & 0xFFFF);
    A[w][2 * lane + 1] = static_cast<uint16_t>(v >> 16);
    for (uint32_t j = lane; j < ns; j += 64) S[w][j] = static_cast<uint16_t>((s1[g1 + j] >> 24) & 0xFFFF);
    for (uint32_t j = lane; j < nc; j += 64) C[w][j] = static_cast<uint16_t>((s2[g2 + j] >> 24) & 0xFFFF);
    for (uint32_t j = nc + lane; j < got; j += 64) {
      const uint64_t e = s2[g2 + j];
      const uint64_t pos = qf::atomic_add_u64(&state[TS_OVPOS], 1ull);
      bk[bn + pos] = pair_of(static_cast<uint32_t>(e >> 40), static_cast<uint32_t>(e & 0xFFFFFF),
                             static_cast<uint32_t>((e >> 24) & 0xFFFF));
    }
  }
  __syncthreads();
  const uint32_t tot = ha + ns + nc;
  if (touched) {
    for (uint32_t j = lane; j < tot; j += 64) {
      uint32_t x, pos;
      if (j < ha) {
        x = A[w][j];
        pos = j + lb16(S[w], ns, x) + lb16(C[w], nc, x);
      } else if (j < ha + ns) {
        const uint32_t i = j - ha;
        x = S[w][i];
        pos = i + ub16(A[w], ha, x) + lb16(C[w], nc, x);
      } else {
        const uint32_t i = j - ha - ns;
        x = C[w][i];
        pos = i + ub16(A[w], ha, x) + ub16(S[w], ns, x);
      }
      O[w][pos] = static_cast<uint16_t>(x);
    }
  }
  __syncthreads();
  if (touched) {
    const uint32_t i0 = 2 * lane, i1 = 2 * lane + 1;
    const uint32_t lo = i0 < tot ? O[w][i0] : EMPTY_B, hi = i1 < tot ? O[w][i1] : EMPTY_B;
    reinterpret_cast<uint32_t *>(slots + b * BB)[lane] = lo | (hi << 16);
  }
}

// Bulk delete, one step (phase 1: in the primary block of the sorted keys;
// phase 2: in the secondary).  One wave per block b: in each run of equal
// tags among the keys of block b, the first k succeed (k = copies held) and
// those copies leave the block; next[i] = SENT for a success, else the key
// for the next step (phase 1: secondary << 40 | tag << 24 | primary; phase 2:
// the backing-table identity).  Entries of L past the last block are SENT.
template <int PHASE>
__global__ __launch_bounds__(NT) void k_del_step(uint16_t *slots, uint64_t nb, const uint64_t *__restrict__ L,
                                                 uint64_t n, const uint32_t *__restrict__ gs,
                                                 uint64_t *__restrict__ next, uint64_t *state) {
  __shared__ uint16_t A[4][BB], O[4][BB];
  __shared__ uint8_t R[4][BB];  // copies removed
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t b = static_cast<uint64_t>(blockIdx.x) * 4 + w;  // (uniform over the wave)
  int64_t done = 0;
  uint32_t tot = 0, held = 0;
  // (a block with no keys in this step is neither read nor written)
  const bool touched = b < nb && gs[b + 1] != gs[b];
  if (touched) {
    const uint32_t v = reinterpret_cast<const uint32_t *>(slots + b * BB)[lane];
    A[w][2 * lane] = static_cast<uint16_t>(v & 0xFFFF);
    A[w][2 * lane + 1] = static_cast<uint16_t>(v >> 16);
    R[w][2 * lane] = 0;
    R[w][2 * lane + 1] = 0;
  }
  __syncthreads();
  if (touched) {
    held = lb16(A[w], BB, EMPTY_B);
    const uint64_t *grp = L + gs[b];
    const uint64_t gn = gs[b + 1] - gs[b];
    // the r-th key of a run of tag t (r = its index minus the run's first)
    // takes the r-th copy of t in the block, if there is one
    for (uint64_t j = lane; j < gn; j += 64) {
      const uint64_t e = grp[j];
      const uint32_t tag = static_cast<uint32_t>((e >> 24) & 0xFFFF), other = static_cast<uint32_t>(e & 0xFFFFFF);
      const uint64_t r = j - lower_bound(grp, gn, (b << 40) | (static_cast<uint64_t>(tag) << 24));
      const uint32_t lo = lb16(A[w], held, tag), copies = ub16(A[w], held, tag) - lo;
      const bool ok = r < copies;
      if (ok) R[w][lo + r] = 1;
      done += ok ? 1 : 0;
      next[gs[b] + j] = ok ? SENT
                           : (PHASE == 1 ? comp_of(other, tag, static_cast<uint32_t>(b))
                                         : pair_of(static_cast<uint32_t>(b), other, tag));
    }
  }
  __syncthreads();
  if (touched) {
    // the kept tags, in order: exclusive scan of the per-lane counts
    const uint32_t i0 = 2 * lane, i1 = 2 * lane + 1;
    const uint32_t keep0 = i0 < held && !R[w][i0] ? 1u : 0u, keep1 = i1 < held && !R[w][i1] ? 1u : 0u;
    const uint32_t c = keep0 + keep1;
    uint32_t inc = c;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t x = __shfl_up(inc, d);
      if (lane >= d) inc += x;
    }
    tot = __shfl(inc, 63);
    uint32_t pos = inc - c;
    if (keep0) O[w][pos++] = A[w][i0];
    if (keep1) O[w][pos] = A[w][i1];
  }
  __syncthreads();
  if (touched) {
    const uint32_t i0 = 2 * lane, i1 = 2 * lane + 1;
    const uint32_t lo = i0 < tot ? O[w][i0] : EMPTY_B, hi = i1 < tot ? O[w][i1] : EMPTY_B;
    reinterpret_cast<uint32_t *>(slots + b * BB)[lane] = lo | (hi << 16);
  }
  // entries past the last block's keys (SENT from an earlier step)
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t i = gs[nb] + static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride) next[i] = SENT;
  (void)done;
  (void)state;
}

// Bulk delete, last step: the identities in d[0, n) (sorted, SENT last)
// against the sorted backing array bk[0, bn): per run of equal identities
// the first (copies in the backing array) succeed; the others are counted
// not found.  tmp[i] = bk[i], or SENT for an entry that goes.
__global__ __launch_bounds__(NT) void k_del_backing(const uint64_t *__restrict__ d, uint64_t n,
                                                    const uint64_t *__restrict__ bk, uint64_t bn,
                                                    uint64_t *__restrict__ tmp, uint64_t *not_found,
                                                    uint64_t *state) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x;
  int64_t absent = 0, removed = 0;
  if (i < n) {
    const uint64_t v = d[i];
    if (v != SENT) {
      const uint64_t first = lower_bound(d, n, v);
      const uint64_t have = bn ? lower_bound(bk, bn, v + 1) - lower_bound(bk, bn, v) : 0;
      absent = i - first >= have ? 1 : 0;
    }
  }
  if (i < bn) {
    const uint64_t v = bk[i];
    const uint64_t lo = lower_bound(bk, bn, v), cp = lower_bound(bk, bn, v + 1) - lo;
    const uint64_t kd = lower_bound(d, n, v + 1) - lower_bound(d, n, v);
    const bool gone = i - lo < (kd < cp ? kd : cp);
    tmp[i] = gone ? SENT : v;
    removed = gone ? 1 : 0;
  }
  absent = group_sum(absent);
  removed = group_sum(removed);
  if (threadIdx.x == 0) {
    if (absent && not_found) qf::atomic_add_u64(not_found, static_cast<uint64_t>(absent));
    if (removed) qf::atomic_add_u64(&state[TS_REMOVED], static_cast<uint64_t>(removed));
  }
}

// Directory of the bulk form's sorted backing array: dir[d] = the first
// entry whose smaller block index is at least d << DIR_LOG (an entry's key
// starts with that index), for d in [0, nd); dir[nd - 1] = bn.
constexpr uint32_t DIR_LOG = 6;
__global__ __launch_bounds__(NT) void k_dir(const uint64_t *__restrict__ bk, uint64_t bn, uint32_t *__restrict__ dir,
                                            uint64_t nd) {
  const uint64_t d = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x;
  if (d >= nd) return;
  dir[d] = static_cast<uint32_t>(d + 1 == nd ? bn : lower_bound(bk, bn, (d << DIR_LOG) << 40));
}

// lookups of the bulk form: 16 lanes per key, each testing 8 tags of each
// candidate block (one 16-byte load per block and lane, so a key's two
// 256-byte blocks arrive in one round trip instead of a chain of dependent
// binary-search probes); a miss in both blocks then searches the part of
// the sorted backing array that the directory gives for the key's smaller
// block (a few entries) for the key's identity
__global__ __launch_bounds__(NT) void k_bulk_query(const uint16_t *__restrict__ slots, uint64_t nb,
                                                   const uint64_t *__restrict__ bk, uint64_t bn,
                                                   const uint32_t *__restrict__ dir,
                                                   const uint64_t *__restrict__ keys, uint64_t n,
                                                   uint8_t *__restrict__ out) {
  constexpr uint32_t LPK = 16;  // lanes per key: LPK x 16 bytes = one block of BB tags
  static_assert(LPK * 8 == BB, "16 lanes of 8 tags cover a block");
  const int lane = threadIdx.x & 63, g = lane / LPK, l = lane % LPK;
  const uint64_t per_grid = static_cast<uint64_t>(gridDim.x) * (NT / LPK);
  // (the loop bound is the wave's first key, so every lane of a wave takes
  // every trip and the ballot sees the whole wave)
  for (uint64_t i0 = (static_cast<uint64_t>(blockIdx.x) * NT + (threadIdx.x & ~63u)) / LPK; i0 < n; i0 += per_grid) {
    const uint64_t i = i0 + static_cast<uint64_t>(g);
    const bool valid = i < n;
    TK k{0, 0, 0, 0};
    bool m = false;
    if (valid) {
      k = key_of(keys[i], nb);
      const u64x2 vx = reinterpret_cast<const u64x2 *>(slots + static_cast<uint64_t>(k.b1) * BB)[l];
      const u64x2 vy = reinterpret_cast<const u64x2 *>(slots + static_cast<uint64_t>(k.b2) * BB)[l];
      m = (eq16(vx.x, k.tag) | eq16(vx.y, k.tag) | eq16(vy.x, k.tag) | eq16(vy.y, k.tag)) != 0;
    }
    const uint64_t bal = __ballot(m);
    bool hit = ((bal >> (g * LPK)) & 0xFFFFull) != 0;
    if (valid && l == 0) {
      if (!hit && bn) {
        const uint64_t pk = pair_of(k.b1, k.b2, k.tag);
        const uint32_t d = (k.b1 < k.b2 ? k.b1 : k.b2) >> DIR_LOG;
        const uint64_t a = dir[d], e = dir[d + 1];
        const uint64_t p = a + lower_bound(bk + a, e - a, pk);
        hit = p < e && bk[p] == pk;
      }
      out[i] = hit ? 1 : 0;
    }
  }
}

// after the last sort of a bulk delete: the keys still unmatched are the
// entries before the first SENT; the others left the blocks
__global__ void k_held_after_delete(const uint64_t *__restrict__ d, uint64_t n, uint64_t *state) {
  if (threadIdx.x == 0 && blockIdx.x == 0) state[TS_HELD] -= n - lower_bound(d, n, SENT);
}
__global__ void k_add_word(uint64_t *state, int idx, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) state[idx] += v;
}
__global__ void k_set_words(uint64_t *state, int idx, int cnt, uint64_t v) {
  if (threadIdx.x < static_cast<unsigned>(cnt) && blockIdx.x == 0) state[idx + threadIdx.x] = v;
}

uint32_t grid_for(uint64_t n) {
  const uint64_t g = (n + NT - 1) / NT;
  return static_cast<uint32_t>(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}
uint32_t blocks_for(uint64_t n) { return static_cast<uint32_t>((n + NT - 1) / NT); }
// grids of the point updates, which end with a same-address atomic per
// work-group (about 12 ns each, serialised): 4096 work-groups of 256 lanes
// still fill the chip twice over
uint32_t grid_for_updates(uint64_t n) {
  const uint32_t g = grid_for(n);
  return g > 4096 ? 4096 : g;
}

}  // namespace
}  // namespace tcf

struct tcf_filter {
  int kind = 0;
  uint32_t B = 0;
  uint64_t nb = 0, nbt = 0;
  uint16_t *slots = nullptr;
  uint64_t *backing = nullptr;
  uint64_t *state = nullptr;
  uint64_t bn = 0;  // bulk: backing entries in use
  uint32_t *dir = nullptr;  // bulk: directory of the backing array (nd words)
  uint64_t nd = 0;
  int device = 0;
  uint64_t bytes = 0;
  // bulk scratch
  uint32_t *gs1 = nullptr, *gs2 = nullptr, *ps = nullptr, *pf = nullptr;
  uint64_t *bk_tmp = nullptr;
  uint64_t cap = 0, hist_words = 0;
  uint64_t *bufA = nullptr, *bufB = nullptr, *bufC = nullptr;
  uint32_t *hist = nullptr;
  uint64_t *h_words = nullptr;  // pinned
  qf::Pipe pipe;                // the sort's launch parameters
};

namespace {

#define TCF_HIP(call)                                              \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return qf::record_error(QF_ERR_DEVICE);  \
  } while (0)

uint64_t backing_entries(uint64_t slots) {
  uint64_t need = (slots + 99) / 100;
  if (need < 64) need = 64;
  uint64_t n = 1;
  while (n < need) n <<= 1;
  return n;
}

void free_batch(tcf_filter *t) {
  (void)hipFree(t->bufA);
  (void)hipFree(t->bufB);
  (void)hipFree(t->bufC);
  (void)hipFree(t->hist);
  t->bufA = t->bufB = t->bufC = nullptr;
  t->hist = nullptr;
  t->bytes -= 3 * t->cap * 8 + t->hist_words * 4;
  t->cap = t->hist_words = 0;
}

int ensure_batch(tcf_filter *t, uint64_t n, hipStream_t s) {
  if (n <= t->cap) return QF_OK;
  uint64_t cap = 1ull << 16;
  while (cap < n) cap <<= 1;
  if (t->cap) TCF_HIP(hipStreamSynchronize(s));
  free_batch(t);
  const uint64_t hw = qf::sort_count_words(cap > t->nbt ? cap : t->nbt);
  if (hipMalloc(&t->bufA, cap * 8) != hipSuccess || hipMalloc(&t->bufB, cap * 8) != hipSuccess ||
      hipMalloc(&t->bufC, cap * 8) != hipSuccess || hipMalloc(&t->hist, hw * 4) != hipSuccess) {
    free_batch(t);
    return qf::record_error(QF_ERR_OOM);
  }
  t->cap = cap;
  t->hist_words = hw;
  t->bytes += 3 * cap * 8 + hw * 4;
  return QF_OK;
}

// sorts a[0, n) (64-bit keys) with b as the other buffer; the result is left in a
int sort64(tcf_filter *t, uint64_t *a, uint64_t *b, uint64_t n, hipStream_t s) {
  if (n == 0) return QF_OK;
  uint64_t *res = nullptr;
  TCF_HIP(qf::launch_sort(a, b, n, 64, t->hist, &res, s, t->pipe));
  if (res != a) TCF_HIP(hipMemcpyAsync(a, res, n * 8, hipMemcpyDeviceToDevice, s));
  return QF_OK;
}

// group bounds of sorted keys s[0, n): a scatter from the keys when they are
// dense (no SENT entries and at least one per block on average: every thread
// then writes a few entries), else a binary search per block (a scatter over
// a sparse list would leave one thread to fill the long gaps)
void group_bounds(tcf_filter *t, const uint64_t *s_, uint64_t n, uint32_t *gs, hipStream_t s, bool dense) {
  using namespace tcf;
  if (dense && n >= t->nb)
    k_gbounds_scatter<<<blocks_for(n + 1), NT, 0, s>>>(s_, n, t->nb, gs);
  else
    k_gbounds<<<blocks_for(t->nb + 1), NT, 0, s>>>(s_, n, t->nb, gs);
}

int bulk_insert(tcf_filter *t, const uint64_t *keys, uint64_t n, hipStream_t s) {
  using namespace tcf;
  if (int rc = ensure_batch(t, n, s)) return rc;
  k_compose<<<blocks_for(n), NT, 0, s>>>(keys, n, t->nb, t->bufA);
  if (int rc = sort64(t, t->bufA, t->bufB, n, s)) return rc;
  group_bounds(t, t->bufA, n, t->gs1, s, true);
  k_plan<<<blocks_for(t->nb * 16), NT, 0, s>>>(t->slots, t->nb, t->gs1, t->ps, t->pf);
  k_set_words<<<1, 64, 0, s>>>(t->state, TS_OVER, 4, 0ull);  // TS_OVER .. TS_CHOSEN
  k_choose<<<blocks_for((n + CHOOSE_K - 1) / CHOOSE_K), NT, 0, s>>>(t->bufA, n, t->gs1, t->ps, t->pf, t->bufC,
                                                                     t->state);
  TCF_HIP(hipMemcpyAsync(t->h_words, t->state + TS_CHOSEN, 8, hipMemcpyDeviceToHost, s));
  TCF_HIP(hipStreamSynchronize(s));
  // only the items that did not take the shortcut are sorted again (none
  // while every block is below 3/4 of its slots)
  const uint64_t m = t->h_words[0];
  uint64_t over = 0;
  if (m) {
    if (int rc = sort64(t, t->bufC, t->bufB, m, s)) return rc;
    group_bounds(t, t->bufC, m, t->gs2, s, true);
    k_over<<<blocks_for(t->nb), NT, 0, s>>>(t->nb, t->gs2, t->pf, t->state);
    TCF_HIP(hipMemcpyAsync(t->h_words, t->state + TS_OVER, 8, hipMemcpyDeviceToHost, s));
    TCF_HIP(hipStreamSynchronize(s));
    over = t->h_words[0];
    if (t->bn + over > t->nbt) return qf::record_error(QF_ERR_FULL);
  } else {
    group_bounds(t, t->bufC, 0, t->gs2, s, false);  // all zero: no chosen items
  }
  k_merge_blocks<<<static_cast<uint32_t>((t->nb + 3) / 4), NT, 0, s>>>(
      t->slots, t->nb, t->bufA, t->gs1, t->bufC, t->gs2, t->ps, t->pf, t->backing, t->bn, t->state);
  if (over) {
    if (int rc = sort64(t, t->backing, t->bk_tmp, t->bn + over, s)) return rc;
    t->bn += over;
    k_set_words<<<1, 64, 0, s>>>(t->state, TS_BACK, 1, t->bn);
    k_dir<<<blocks_for(t->nd), NT, 0, s>>>(t->backing, t->bn, t->dir, t->nd);
  }
  k_add_word<<<1, 64, 0, s>>>(t->state, TS_HELD, n - over);
  TCF_HIP(hipGetLastError());
  return QF_OK;
}

int bulk_delete(tcf_filter *t, const uint64_t *keys, uint64_t n, uint64_t *not_found, hipStream_t s) {
  using namespace tcf;
  if (int rc = ensure_batch(t, n, s)) return rc;
  const uint32_t mb = static_cast<uint32_t>((t->nb + 3) / 4);
  k_compose<<<blocks_for(n), NT, 0, s>>>(keys, n, t->nb, t->bufA);
  if (int rc = sort64(t, t->bufA, t->bufB, n, s)) return rc;
  group_bounds(t, t->bufA, n, t->gs1, s, true);
  k_del_step<1><<<mb, NT, 0, s>>>(t->slots, t->nb, t->bufA, n, t->gs1, t->bufC, t->state);
  if (int rc = sort64(t, t->bufC, t->bufB, n, s)) return rc;
  group_bounds(t, t->bufC, n, t->gs2, s, false);
  k_del_step<2><<<mb, NT, 0, s>>>(t->slots, t->nb, t->bufC, n, t->gs2, t->bufA, t->state);
  if (int rc = sort64(t, t->bufA, t->bufB, n, s)) return rc;
  k_held_after_delete<<<1, 64, 0, s>>>(t->bufA, n, t->state);
  k_set_words<<<1, 64, 0, s>>>(t->state, TS_REMOVED, 1, 0ull);
  const uint64_t m = n > t->bn ? n : t->bn;
  k_del_backing<<<blocks_for(m), NT, 0, s>>>(t->bufA, n, t->backing, t->bn, t->bk_tmp, not_found, t->state);
  if (t->bn) {
    TCF_HIP(hipMemcpyAsync(t->h_words, t->state + TS_REMOVED, 8, hipMemcpyDeviceToHost, s));
    TCF_HIP(hipStreamSynchronize(s));
    const uint64_t removed = t->h_words[0];
    if (removed) {
      // the kept entries of bk_tmp sorted (gone ones are SENT and sort
      // last); the old array serves as the sort's other buffer, then the two
      // arrays trade places
      if (int rc = sort64(t, t->bk_tmp, t->backing, t->bn, s)) return rc;
      std::swap(t->backing, t->bk_tmp);
      t->bn -= removed;
      k_set_words<<<1, 64, 0, s>>>(t->state, TS_BACK, 1, t->bn);
      k_dir<<<blocks_for(t->nd), NT, 0, s>>>(t->backing, t->bn, t->dir, t->nd);
    }
  }
  TCF_HIP(hipGetLastError());
  return QF_OK;
}

}  // namespace

extern "C" {

tcf_t *tcf_create(uint64_t nblocks, int kind) {
  if (nblocks < 1 || nblocks > (1ull << 24) || (kind != TCF_POINT && kind != TCF_BULK)) {
    qf::record_error(QF_ERR_ARG);
    return nullptr;
  }
  tcf_filter *t = new (std::nothrow) tcf_filter();
  if (!t) {
    qf::record_error(QF_ERR_OOM);
    return nullptr;
  }
  t->kind = kind;
  t->B = kind == TCF_POINT ? tcf::PB : tcf::BB;
  t->nb = nblocks;
  t->nbt = backing_entries(nblocks * t->B);
  (void)hipGetDevice(&t->device);
  const uint64_t sbytes = nblocks * t->B * 2;
  bool ok = hipMalloc(&t->slots, sbytes) == hipSuccess &&
            hipMemset(t->slots, kind == TCF_POINT ? 0 : 0xFF, sbytes) == hipSuccess &&
            hipMalloc(&t->backing, t->nbt * 8) == hipSuccess && hipMemset(t->backing, 0, t->nbt * 8) == hipSuccess &&
            hipMalloc(&t->state, tcf::TS_WORDS * 8) == hipSuccess &&
            hipMemset(t->state, 0, tcf::TS_WORDS * 8) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void **>(&t->h_words), 64) == hipSuccess;
  t->bytes = sbytes + t->nbt * 8 + tcf::TS_WORDS * 8;
  if (ok && kind == TCF_BULK) {
    ok = hipMalloc(&t->gs1, (nblocks + 1) * 4) == hipSuccess && hipMalloc(&t->gs2, (nblocks + 1) * 4) == hipSuccess &&
         hipMalloc(&t->ps, nblocks * 4) == hipSuccess && hipMalloc(&t->pf, nblocks * 4) == hipSuccess &&
         hipMalloc(&t->bk_tmp, t->nbt * 8) == hipSuccess;
    t->nd = (nblocks >> tcf::DIR_LOG) + 2;
    ok = ok && hipMalloc(&t->dir, t->nd * 4) == hipSuccess && hipMemset(t->dir, 0, t->nd * 4) == hipSuccess;
    t->bytes += 4 * (nblocks + 1) * 4 + t->nbt * 8 + t->nd * 4;
  }
  if (!ok) {
    tcf_destroy(t);
    qf::record_error(QF_ERR_OOM);
    return nullptr;
  }
  return t;
}

void tcf_destroy(tcf_t *t) {
  if (!t) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(t->slots);
  (void)hipFree(t->backing);
  (void)hipFree(t->state);
  (void)hipFree(t->gs1);
  (void)hipFree(t->gs2);
  (void)hipFree(t->ps);
  (void)hipFree(t->pf);
  (void)hipFree(t->bk_tmp);
  (void)hipFree(t->dir);
  free_batch(t);
  if (t->h_words) (void)hipHostFree(t->h_words);
  delete t;
}

int tcf_insert(tcf_t *t, const uint64_t *d_keys, uint64_t n, int32_t *d_status, void *stream) {
  if (!t || (n && !d_keys)) return qf::record_error(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return qf::record_error(QF_ERR_ARG);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (t->kind == TCF_POINT) {
    // At most one lane in flight per four blocks (at least one work-group),
    // further keys going round the grid-stride loop: a lane chooses its block
    // from the fills it reads, and lanes that all read an emptier table than
    // the one they fill spill far more items to the backing table (a 4096-slot
    // table at load 0.9 with every key in flight at once loses items that one
    // key at a time never does).  Large tables never have that many lanes.
    const uint64_t lanes = t->nb / 4 > static_cast<uint64_t>(tcf::NT) ? t->nb / 4 : tcf::NT;
    const uint32_t g = tcf::grid_for_updates(n), gmax = static_cast<uint32_t>((lanes + tcf::NT - 1) / tcf::NT);
    tcf::k_point_insert<<<g < gmax ? g : gmax, tcf::NT, 0, s>>>(reinterpret_cast<uint64_t *>(t->slots), t->nb,
                                                                t->backing, t->nbt, d_keys, n, d_status, t->state);
    TCF_HIP(hipGetLastError());
    return QF_OK;
  }
  if (d_status) return qf::record_error(QF_ERR_ARG);
  return bulk_insert(t, d_keys, n, s);
}

int tcf_query(tcf_t *t, const uint64_t *d_keys, uint64_t n, uint8_t *d_out, void *stream) {
  if (!t || (n && (!d_keys || !d_out))) return qf::record_error(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (t->kind == TCF_POINT)
    tcf::k_point_query<<<tcf::grid_for(n), tcf::NT, 0, s>>>(reinterpret_cast<const uint64_t *>(t->slots), t->nb,
                                                            t->backing, t->nbt, d_keys, n, d_out);
  else
    tcf::k_bulk_query<<<tcf::grid_for(n * 16), tcf::NT, 0, s>>>(t->slots, t->nb, t->backing, t->bn, t->dir, d_keys,
                                                                n, d_out);
  TCF_HIP(hipGetLastError());
  return QF_OK;
}

int tcf_delete(tcf_t *t, const uint64_t *d_keys, uint64_t n, uint64_t *d_not_found, void *stream) {
  if (!t || (n && !d_keys)) return qf::record_error(QF_ERR_ARG);
  if (n == 0) return QF_OK;
  if (n > 0xFFFFFFFFull) return qf::record_error(QF_ERR_ARG);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (t->kind == TCF_POINT) {
    tcf::k_point_delete<<<tcf::grid_for_updates(n), tcf::NT, 0, s>>>(reinterpret_cast<uint64_t *>(t->slots), t->nb,
                                                             t->backing, t->nbt, d_keys, n, d_not_found, t->state);
    TCF_HIP(hipGetLastError());
    return QF_OK;
  }
  return bulk_delete(t, d_keys, n, d_not_found, s);
}

int tcf_sync(tcf_t *t, void *stream) {
  if (!t) return qf::record_error(QF_ERR_ARG);
  hipStream_t s = static_cast<hipStream_t>(stream);
  TCF_HIP(hipStreamSynchronize(s));
  uint64_t e = 0;
  TCF_HIP(hipMemcpy(&e, t->state + tcf::TS_ERR, 8, hipMemcpyDeviceToHost));
  if (e) {
    const uint64_t zero = 0;
    TCF_HIP(hipMemcpy(t->state + tcf::TS_ERR, &zero, 8, hipMemcpyHostToDevice));
    return qf::record_error(static_cast<int>(static_cast<int64_t>(e)));
  }
  return QF_OK;
}

int tcf_info(tcf_t *t, uint64_t *info, void *stream) {
  if (!t || !info) return qf::record_error(QF_ERR_ARG);
  TCF_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  uint64_t st[tcf::TS_WORDS];
  TCF_HIP(hipMemcpy(st, t->state, sizeof(st), hipMemcpyDeviceToHost));
  info[0] = static_cast<uint64_t>(t->kind);
  info[1] = t->nb;
  info[2] = t->B;
  info[3] = t->nbt;
  info[4] = t->kind == TCF_POINT ? st[tcf::TS_BACK] : t->bn;
  info[5] = st[tcf::TS_HELD];
  info[6] = t->bytes;
  return QF_OK;
}

int tcf_export(tcf_t *t, uint16_t *h_slots, uint64_t *h_backing, void *stream) {
  if (!t || !h_slots || !h_backing) return qf::record_error(QF_ERR_ARG);
  TCF_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  TCF_HIP(hipMemcpy(h_slots, t->slots, t->nb * t->B * 2, hipMemcpyDeviceToHost));
  if (t->kind == TCF_POINT) {
    TCF_HIP(hipMemcpy(h_backing, t->backing, t->nbt * 8, hipMemcpyDeviceToHost));
  } else {
    if (t->bn) TCF_HIP(hipMemcpy(h_backing, t->backing, t->bn * 8, hipMemcpyDeviceToHost));
    for (uint64_t i = t->bn; i < t->nbt; ++i) h_backing[i] = 0;
  }
  return QF_OK;
}

}  // extern "C"
