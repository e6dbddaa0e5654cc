// qf_dev.h -- device-side building blocks of the MI355X counting quotient filter.
//
// Physical table (one of the two copies the library alternates between):
//   blocks[b] : 64 slots = { uint64 occupieds; uint64 runends; uint32 offset;
//               padding; T slot[64] } (128 B for r = 8: one 128-byte line, so
//               a lookup usually reads one line; 160 B for r = 16), where the
//               offset is the distance from slot 64b to the end of the run of
//               the last occupied quotient <= 64b (0 if that end lies before
//               64b).
// Quotient x's occupied bit is bit x%64 of blocks[x/64].occupieds, slot j's
// run-end bit is bit j%64 of blocks[j/64].runends (Sec. 5.1: runs, clusters;
// the rank/select metadata is this library's reading of the paper's CQF).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qf {

template <typename T>
struct Block {
  uint64_t occ;
  uint64_t rend;
  uint32_t off;
  uint32_t pad[sizeof(T) == 1 ? 11 : 3];
  T s[64];
};
// r = 8: one 128-byte line per block (metadata and offset in the first 64
// bytes, slots in the second); r = 16: 32 bytes of metadata + 128 of slots.
static_assert(sizeof(Block<uint8_t>) == 128, "r = 8 block is one 128-byte line");
static_assert(sizeof(Block<uint16_t>) == 160, "r = 16 block is 160 bytes");

// the block offsets seen as an array (offset of block i = blocks[i].off)
template <typename T>
struct OffRef {
  Block<T> *b;
  __device__ uint32_t &operator[](int64_t i) const { return b[i].off; }
};

// Device state words of one filter.
enum : int {
  ST_CUR = 0,     // which table copy is current (0/1)
  ST_ERR = 1,     // first deferred error code (as int64), 0 = none
  ST_USED = 2,    // used slots of the current table
  ST_DIST = 3,    // distinct fingerprints
  ST_TOTAL = 4,   // total count (mod 2^64)
  ST_ACC = 5,     // 5..8: the merge launch's statistics, summed over work-groups
  ST_TICKET = 9,  // work-groups of the launch's finish that are done
  ST_BATCH = 10,  // error bits of the running batch
  ST_NUNIQ = 11,  // distinct fingerprints in the running batch
  ST_BATCHES = 12,
  ST_SCRATCH = 13,  // sink for a NULL not-found pointer
  ST_EPOCH = 14,    // (pipeline words) epoch of the last merge launch, 1..65535
  ST_WORDS = 16
};
enum : uint64_t { BATCH_FULL = 1, BATCH_OVF = 2, BATCH_STALL = 4 };

typedef unsigned long long ull;

__device__ __forceinline__ uint64_t atomic_add_u64(uint64_t* p, uint64_t v) {
  return atomicAdd(reinterpret_cast<ull*>(p), static_cast<ull>(v));
}
__device__ __forceinline__ void atomic_or_u64(uint64_t* p, uint64_t v) {
  atomicOr(reinterpret_cast<ull*>(p), static_cast<ull>(v));
}
__device__ __forceinline__ void atomic_and_u64(uint64_t* p, uint64_t v) {
  atomicAnd(reinterpret_cast<ull*>(p), static_cast<ull>(v));
}

// SplitMix64 finalizer (Steele, Lea, Flood 2014; Stafford's "Mix13"
// constants): the key hash.  A bijection on 64-bit words.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ int popc64(uint64_t v) { return __popcll(v); }
__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }
__device__ __forceinline__ int msb64(uint64_t v) { return 63 - __builtin_clzll(v); }
// index of the k-th (0-based) set bit of v; v has more than k set bits
__device__ __forceinline__ int select64(uint64_t v, int k) {
  for (; k > 0; --k) v &= v - 1;
  return ctz64(v);
}

// ---- run placement as a max-plus map --------------------------------------
// A run of quotient x and length L placed after a previous end e ends at
// max(x, e + 1) + L - 1 = max(x + L - 1, e + L): a map c -> max(A, c + B).
// Such maps compose associatively, so the end of every run (and the carry
// across regions) is a prefix scan over them.  Ends are >= -1, -1 = "none".
struct Fn {
  int64_t A, B;
};
__device__ __forceinline__ Fn fn_id() { return Fn{-1, 0}; }
// g first, then h
__device__ __forceinline__ Fn fn_then(Fn g, Fn h) {
  return Fn{max(h.A, g.A + h.B), g.B + h.B};
}
__device__ __forceinline__ int64_t fn_apply(Fn f, int64_t c) { return max(f.A, c + f.B); }

// ---- tagged words for the merge's look-back ---------------------------------
// 16-bit launch epoch | 48-bit value + 1.  Each word is written once per
// launch with one agent-scope atomic store, so a reader that sees the current
// epoch sees the value; no fences are needed.
__device__ __forceinline__ void tag_store(uint64_t* p, uint32_t epoch, int64_t v) {
  const uint64_t w = (static_cast<uint64_t>(epoch) << 48) | static_cast<uint64_t>(v + 1);
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the epoch of the next merge launch after one that used e (0 = none yet)
__device__ __forceinline__ uint32_t next_epoch(uint64_t e) {
  return e >= 65535 ? 1u : static_cast<uint32_t>(e) + 1u;
}
__device__ __forceinline__ bool tag_load(const uint64_t* p, uint32_t epoch, int64_t* v) {
  const uint64_t w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((w >> 48) != epoch) return false;
  *v = static_cast<int64_t>(w & ((1ull << 48) - 1)) - 1;
  return true;
}

// ---- counter encoding --------------------------------------------------------
// One (remainder x, count c) entry in r-bit slots, digit base B = 2^r - 1:
//   c = 1: [x];  c = 2: [x, x];
//   c >= 3, x > 0: [x, (0), digits of c-3 (MSB first, d >= x stored d+1), x],
//                  the 0 present when the first stored digit would exceed x;
//   c >= 3, x = 0: [0, 0, 0, digits + 1, 0].
// (Sec. 2 and Sec. 6.7 only say that counters are variable-size and embedded
// in the slots; this is the library's reading, shared by the export format.)
// v / (2^r - 1) and the remainder, without a divide: the sum of v >> (r k),
// k >= 1, never exceeds the quotient and misses it by at most 64 / r + 1.
__device__ __forceinline__ uint64_t div_base(uint64_t v, uint32_t r, uint64_t *rem) {
  const uint64_t base = (1ull << r) - 1;
  uint64_t q = 0;
  for (uint32_t s = r; s < 64; s += r) q += v >> s;
  uint64_t m = v - q * base;
  while (m >= base) {
    m -= base;
    ++q;
  }
  *rem = m;
  return q;
}

// digits of v in base 2^r - 1 (at least one) and the most significant one
__device__ __forceinline__ uint32_t base_digits(uint64_t v, uint32_t r, uint64_t *msd) {
  const uint64_t base = (1ull << r) - 1;
  uint32_t nd = 1;
  while (v >= base) {
    uint64_t d;
    v = div_base(v, r, &d);
    ++nd;
  }
  *msd = v;
  return nd;
}

__device__ __forceinline__ uint32_t enc_len(uint64_t x, uint64_t c, uint32_t r) {
  if (c <= 2) return static_cast<uint32_t>(c);
  uint64_t msd;
  const uint32_t nd = base_digits(c - 3, r, &msd);
  if (x > 0) return 2 + nd + (msd >= x ? 1u : 0u);
  return 4 + nd;
}

// Writes the entry's slots at [pos, pos + enc_len); digits are produced least
// significant first and written back to front.
template <class Out, typename P>
__device__ __forceinline__ P enc_put(Out &out, P pos, uint64_t x, uint64_t c, uint32_t r) {
  if (c <= 2) {
    out.emit(pos++, x);
    if (c == 2) out.emit(pos++, x);
    return pos;
  }
  uint64_t msd;
  const uint32_t nd = base_digits(c - 3, r, &msd);
  P p0;  // first digit slot
  if (x > 0) {
    out.emit(pos, x);
    p0 = pos + 1;
    if (msd >= x) out.emit(p0++, 0);
  } else {
    out.emit(pos, 0);
    out.emit(pos + 1, 0);
    out.emit(pos + 2, 0);
    p0 = pos + 3;
  }
  uint64_t v = c - 3;
  for (uint32_t k = 0; k < nd; ++k) {
    uint64_t d;
    v = div_base(v, r, &d);
    out.emit(p0 + static_cast<P>(nd - 1 - k), x > 0 ? (d < x ? d : d + 1) : d + 1);
  }
  out.emit(p0 + static_cast<P>(nd), x);
  return p0 + static_cast<P>(nd) + 1;
}

// Decode the entry that starts at slot p of a run ending at slot e; returns the
// slot after it.  `Old` provides slot(j).
template <class Old, typename P>
__device__ __forceinline__ P dec_entry(const Old& o, P p, P e, uint32_t r, uint64_t& x, uint64_t& c) {
  const uint64_t base = (1ull << r) - 1;
  x = o.slot(p);
  if (x > 0) {
    if (p == e) { c = 1; return p + 1; }
    const uint64_t s1 = o.slot(p + 1);
    if (s1 > x) { c = 1; return p + 1; }
    if (s1 == x) { c = 2; return p + 2; }
    uint64_t v = 0;
    P q = p + 1;
    for (; q <= e; ++q) {
      const uint64_t s = o.slot(q);
      if (s == x) break;
      v = v * base + (s < x ? s : s - 1);
    }
    c = v + 3;
    return q + 1;
  }
  if (p == e || o.slot(p + 1) != 0) { c = 1; return p + 1; }
  if (p + 1 == e || o.slot(p + 2) != 0) { c = 2; return p + 2; }
  uint64_t v = 0;
  P q = p + 3;
  for (; q <= e; ++q) {
    const uint64_t s = o.slot(q);
    if (s == 0) break;
    v = v * base + (s - 1);
  }
  c = v + 3;
  return q + 1;
}

}  // namespace qf
