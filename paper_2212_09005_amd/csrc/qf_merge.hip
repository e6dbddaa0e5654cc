// qf_merge.hip -- bulk insert / delete: one work-group per region.
//
// What is computed (Sec. 5.1, 5.3, 5.4, 6.4): every region of S slots takes
// the sorted, reduced <fingerprint, count> entries whose quotients fall in it,
// merges them with the entries already stored there (summing counts, or
// subtracting them for a delete), and writes its runs back in quotient order,
// each run starting at max(quotient, end of previous run + 1), remainders
// sorted, counters re-encoded.
//
// How (MI355X design, differs from the paper's even/odd phases):
//   * The paper makes regions exclusive with two phases and a spill limit of
//     one region.  Here a run's end is a max-plus map of the previous end,
//     c -> max(A, c + B), and maps compose; each region publishes the
//     composition of its runs, a wave-parallel decoupled look-back gives every
//     region the exact end of all earlier runs (its carry-in), and there is no
//     spill limit.
//   * The table has two device copies; a batch reads the current one and
//     writes the other, so no region reads what another region writes.  The
//     last region to finish flips the current copy -- unless a run ran past
//     the last slot or a count overflowed, which leaves the old copy current
//     (all-or-nothing without a host round trip).
//   * Inside a region: the old blocks and the region's new entries are staged
//     in LDS with 16-byte loads; each of the 256 lanes owns a contiguous chunk
//     of quotients and works in int32 positions relative to the region.  Pass
//     1 walks the chunk once: runs that receive no new entry keep their
//     length (read off the run-end bits without decoding) and are composed
//     into max-plus maps, cut at each changed run, whose old extent is
//     recorded.  Then one lane per changed run decodes, merges and sizes it;
//     the lane maps are finished, block-scanned and chained across regions.
//     Pass 2 walks the chunk again from its carry: unchanged runs are copied
//     to their new place, changed runs get their slots reserved and are then
//     re-encoded one per lane.  The output buffers start zeroed, so gaps cost
//     nothing; the region's extent leaves LDS in 16-byte stores.
//     Regions whose runs or entries do not fit in LDS are done by one lane
//     straight from and to global memory.
#include "qf.h"
#include "qf_dev.h"
#include "qf_lib.h"

namespace qf {
namespace {

constexpr int NT = 256;
constexpr int64_t INF = INT64_MAX / 4;

// pointer to global memory (address space 1): loads and stores through it
// compile to global_* instructions instead of generic flat ones
template <typename U>
using GPtr = __attribute__((address_space(1))) U *;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // 16 bytes, no class methods
template <typename U>
__device__ __forceinline__ GPtr<U> to_global(U *p) {
  return (GPtr<U>)p;  // (a cast between address spaces; no reinterpret_cast for it)
}

template <typename T>
struct Cfg {
  // largest region: 8192 slots (r = 8), 4096 (r = 16); the LDS buffers hold
  // 1.125 regions of slots: a region's runs plus what spills past its end
  // (at load 0.95 a region's runs end at most ~80 slots past it)
  static constexpr int SMAXLOG = sizeof(T) == 1 ? 13 : 12;
  static constexpr int SMAX = 1 << SMAXLOG;
  static constexpr int CAP = SMAX + SMAX / 8;
  static constexpr int CAPW = CAP / 64;
  static constexpr int OW = SMAX / 64;
  static constexpr int NCAP = 304;  // distinct new entries staged in LDS (<= 2 per lane)
  static constexpr int CH = 64 * static_cast<int>(sizeof(T)) / 16;  // 16-byte chunks per block
  static constexpr int PER = 16 / static_cast<int>(sizeof(T));      // slots per chunk
};

// max-plus maps relative to a region's first quotient (-1 = "none")
struct Fn32 {
  int32_t A, B;
};
__device__ __forceinline__ Fn32 f32_id() { return Fn32{-1, 0}; }
__device__ __forceinline__ Fn32 f32_then(Fn32 g, Fn32 h) { return Fn32{max(h.A, g.A + h.B), g.B + h.B}; }

// One merge launch over the G regions of a pipeline (all filters of a set, or
// one filter); a work-group finds its filter through rmap and desc.
struct MergeArgs {
  FDesc one;  // the filter of a one-filter pipeline (read from the kernel arguments)
  const FDesc *desc;
  const uint32_t *rmap;
  const uint64_t *ufp, *ucnt, *rb;  // composite keys, counts, region bounds
  uint64_t *tags;                   // 3 G look-back words
  uint64_t *rstat;                  // 4 words per region: used, distinct, total, shortfall
  const int64_t *cb;                // old carries at region boundaries
  const uint64_t *pst;               // pipeline words: the epoch of the last launch
  uint32_t G;
  int del;
  const uint32_t *areg;  // the launch's regions (nullptr: all G, in order)
  // per-entry scratch (indexed like the reduced batch) for regions with more
  // entries than the LDS holds: region-relative fingerprints and counts, and
  // the changed-run arrays (a region has at most as many changed runs as
  // entries, so run c of the region starting at entry rb0 sits at rb0 + c)
  uint32_t *g_fp, *g_cnt, *g_head, *g_L;
  uint16_t *g_xr, *g_op, *g_oe, *g_st;
  Fn32 *g_gaf;
};

// ---- readers of the current (old) table -------------------------------------
template <typename T>
struct OldGlb {
  const Block<T> *blk;
  int64_t nblocks;
  __device__ uint64_t slot(int64_t j) const { return blk[j >> 6].s[j & 63]; }
  __device__ int64_t next_end(int64_t from) const {
    int64_t w = from >> 6;
    uint64_t m = blk[w].rend & (~0ull << (from & 63));
    while (!m) {
      if (++w >= nblocks) return nblocks * 64 - 1;
      m = blk[w].rend;
    }
    return (w << 6) + ctz64(m);
  }
};

// ---- the region's new <fingerprint, count> entries --------------------------
// staged in LDS: (quotient - region start) << r | remainder, and the count
struct NewRel {
  const uint32_t *fp;
  const uint32_t *cnt;
  __device__ uint64_t f(uint32_t i) const { return fp[i]; }
  __device__ uint64_t c(uint32_t i) const { return cnt[i]; }
};
// the region's entries straight from the reduced batch: the composite key's
// low bits are the fingerprint inside the region, `base` its high part
struct NewGlb {
  const uint64_t *fp, *cnt;
  uint64_t base, mask;
  __device__ uint64_t f(uint64_t i) const { return base | (fp[i] & mask); }
  __device__ uint64_t c(uint64_t i) const { return cnt[i]; }
};

// ---- writers of the new table -------------------------------------------
// emit(j, v) writes slot j (positions strictly increasing per lane), set_end()
// marks the last written slot as a run end, flush() ends the lane's output.
// Run-end bits are gathered per 64-bit word; words shared with a neighbour's
// extent are merged with and/or under the lane's mask.
template <typename T>
struct OutGlb {
  Block<T> *blk;
  int64_t hi;
  int64_t cw;
  uint64_t acc, accm;
  __device__ void init(Block<T> *blk_, int64_t hi_) {
    blk = blk_; hi = hi_; cw = -1; acc = 0; accm = 0;
  }
  __device__ void flush() {
    if (accm == ~0ull) {
      blk[cw].rend = acc;
    } else if (accm) {
      atomic_and_u64(&blk[cw].rend, ~accm);
      atomic_or_u64(&blk[cw].rend, acc);
    }
    acc = accm = 0;
  }
  __device__ void emit(int64_t j, uint64_t v) {
    if (j > hi) return;
    blk[j >> 6].s[j & 63] = static_cast<T>(v);
    const int64_t w = j >> 6;
    if (w != cw) {
      if (cw >= 0) flush();
      cw = w;
    }
    accm |= 1ull << (j & 63);
  }
  __device__ void set_end(int64_t j) {
    if (j > hi) return;
    acc |= 1ull << (j & 63);
  }
};

struct NoOut {
  __device__ void flush() {}
  __device__ void emit(int64_t, uint64_t) {}
  __device__ void set_end(int64_t) {}
};

struct Acc {
  Fn F;
  uint64_t used;       // slots of all runs
  uint64_t dent;       // change of the number of distinct fingerprints (mod 2^64)
  uint64_t dtot;       // change of the total count (mod 2^64)
  uint64_t shortfall;  // delete: instances not present
  uint32_t ovf;
};

// next quotient >= from (and < to) whose old occupied bit is set; region bits
// in occ_l are relative to RS
__device__ __forceinline__ int64_t next_occ(const uint64_t *occ_l, int64_t RS, int64_t from,
                                            int64_t to) {
  while (from < to) {
    const int64_t t = from - RS;
    const uint64_t m = occ_l[t >> 6] & (~0ull << (t & 63));
    if (m) {
      const int64_t x = RS + ((t >> 6) << 6) + ctz64(m);
      return x < to ? x : INF;
    }
    from = RS + (((t >> 6) + 1) << 6);
  }
  return INF;
}

// End of the last (old) run whose quotient is < i, or i - 1 when it ends
// before i / there is none.  i is a multiple of 64 and i <= N.
template <typename T>
__device__ int64_t carry_old(const Block<T> *b, int64_t i, int64_t N) {
  const int64_t bi = i >> 6;
  const int64_t O = b[bi].off;
  const bool occ_i = i < N && (b[bi].occ & 1ull);
  if (!occ_i) {
    if (O > 0) return i + O;
    return (b[bi].rend & 1ull) ? i : i - 1;
  }
  const int64_t e = i + O;  // end of quotient i's own run
  if (e == i) return i - 1;
  int64_t w = (e - 1) >> 6;
  uint64_t m = b[w].rend & (~0ull >> (63 - ((e - 1) & 63)));
  for (;;) {
    if (m) return (w << 6) + msb64(m);
    if (w == bi) return i - 1;
    --w;
    m = b[w].rend;
  }
}

// Before the merge, one thread per region g of the launch (all regions of
// the pipeline, or those listed in areg): the old carry at the region's
// first slot (cb[g] = carry_old(R S) for local regions R up to the first
// extra-slot region) and the filter's batch flags (by its region 0).
// The launch epoch lives in device memory (so that a captured graph replays
// with a fresh one); when it wraps, the grid (which covers all G regions of
// the pipeline) clears every look-back word, also those of regions outside
// the launch, which could otherwise carry an old word with a current epoch
// into a later launch.
template <typename T>
__global__ __launch_bounds__(NT) void k_carries(const FDesc *__restrict__ desc, const uint32_t *__restrict__ rmap,
                                                const uint32_t *__restrict__ areg, uint32_t nreg, int64_t *cb,
                                                uint64_t *tags, uint32_t G, const uint64_t *pst) {
  const uint32_t i = blockIdx.x * NT + threadIdx.x;
  if (i < G && next_epoch(pst[ST_EPOCH]) == 1u) {
    tags[i] = 0;
    tags[static_cast<uint64_t>(G) + i] = 0;
    tags[2ull * G + i] = 0;
  }
  if (i >= nreg) return;
  const uint32_t g = areg ? areg[i] : i;
  const FDesc &d = desc[rmap[g]];
  const uint32_t R = g - d.rbase;
  if (R == 0) d.state[ST_BATCH] = 0;
  if (R <= d.nqregions) {
    const bool cur = d.state[ST_CUR] & 1ull;
    cb[g] = carry_old(static_cast<const Block<T> *>(cur ? d.blk[1] : d.blk[0]), static_cast<int64_t>(R) << d.rlog,
                      d.N);
  }
}

// Merge of one quotient's old run [op, oe] with its new entries [ni, nj):
// pass 1 returns the new run length, pass 2 writes the run from `pos`.
template <bool EMIT, class Old, class New, class Out, typename P>
__device__ __forceinline__ P merge_run(const Old &old, P op, P oe, const New &nw, uint32_t ni,
                                       uint32_t nj, uint32_t r, int del, Out &out, P pos, Acc &acc) {
  const uint64_t rmask = (1ull << r) - 1ull;
  P L = 0;
  uint64_t orem = 0, ocnt = 0;
  bool ohave = false;
  if (op <= oe) {
    op = dec_entry(old, op, oe, r, orem, ocnt);
    ohave = true;
  }
  uint32_t k = ni;
  while (ohave || k < nj) {
    const uint64_t nrem = k < nj ? (nw.f(k) & rmask) : ~0ull;
    uint64_t rem, c;
    if (ohave && (k >= nj || orem < nrem)) {
      rem = orem;
      c = ocnt;
      if (op <= oe) op = dec_entry(old, op, oe, r, orem, ocnt); else ohave = false;
    } else if (!ohave || nrem < orem) {
      rem = nrem;
      const uint64_t cn = nw.c(k++);
      if (del) {
        if (!EMIT) acc.shortfall += cn;
        c = 0;
      } else {
        c = cn;
        if (!EMIT) {
          acc.dent += 1;
          acc.dtot += cn;
        }
      }
    } else {
      rem = orem;
      const uint64_t cn = nw.c(k++);
      if (del) {
        const uint64_t t = min(ocnt, cn);
        c = ocnt - t;
        if (!EMIT) {
          acc.shortfall += cn - t;
          acc.dtot -= t;
          if (c == 0) acc.dent -= 1;
        }
      } else {
        c = ocnt + cn;
        if (c < ocnt) {
          if (!EMIT) acc.ovf = 1;
          c = ~0ull;
        }
        if (!EMIT) acc.dtot += cn;
      }
      if (op <= oe) op = dec_entry(old, op, oe, r, orem, ocnt); else ohave = false;
    }
    if (c == 0) continue;
    if (EMIT)
      pos = enc_put(out, pos, rem, c, r);
    else
      L += static_cast<P>(enc_len(rem, c, r));
  }
  return EMIT ? pos : L;
}

// Walk one lane's chunk: quotients [x0, x1) (the same numbers as its slots
// [s0, s1) in a quotient region; empty in the extra slots).  Pass 1 (EMIT =
// false) composes the lane's run maps; pass 2 writes the lane's extent
// [max(carry + 1, s0), max(last end, s1 - 1)] -- runs and zero gaps -- plus
// the occupied bits and the offsets of the blocks that start in it.
template <typename T, bool EMIT, class Old, class New, class Out>
__device__ __forceinline__ void walk(uint32_t r, int del, int64_t RS, const uint64_t *occ_l,
                                     int64_t x0, int64_t x1, int64_t s0, int64_t s1, int64_t ope,
                                     uint64_t ni, uint64_t nb, const Old &old, const New &nw,
                                     Out &out, int64_t carry, Acc &acc, uint64_t *nocc_l,
                                     OffRef<T> noff) {
  int64_t wpos = max(carry + 1, s0);
  int64_t next_bs = (s0 + 63) & ~static_cast<int64_t>(63);
  int64_t xo = x0 < x1 ? next_occ(occ_l, RS, x0, x1) : INF;
  uint64_t nfp = ni < nb ? nw.f(ni) : 0;
  for (;;) {
    const int64_t xn = ni < nb ? static_cast<int64_t>(nfp >> r) : INF;
    const int64_t x = min(xo, xn);
    if (x >= INF) break;
    if (EMIT) {
      for (; next_bs < x; next_bs += 64)
        noff[next_bs >> 6] = static_cast<uint32_t>(max(carry - next_bs, static_cast<int64_t>(0)));
    }
    int64_t op = 0, oe = -1;
    if (xo == x) {
      op = max(x, ope + 1);
      oe = old.next_end(op);
      ope = oe;
      xo = next_occ(occ_l, RS, x + 1, x1);
    }
    uint64_t nj = ni;
    while (nj < nb && static_cast<int64_t>(nfp >> r) == x) {
      ++nj;
      if (nj < nb) nfp = nw.f(nj);
    }
    if (EMIT) {
      const int64_t start = max(x, carry + 1);
      for (; wpos < start; ++wpos) out.emit(wpos, 0);
      int64_t pos = start;
      if (ni == nj) {
        for (int64_t j = op; j <= oe; ++j) out.emit(pos++, old.slot(j));
      } else {
        pos = merge_run<true>(old, op, oe, nw, ni, nj, r, del, out, pos, acc);
      }
      if (pos > start) {
        out.set_end(pos - 1);
        carry = pos - 1;
        wpos = pos;
        const int64_t t = x - RS;
        atomicOr(reinterpret_cast<ull *>(&nocc_l[t >> 6]), static_cast<ull>(1ull << (t & 63)));
      }
      if (x == next_bs) {
        noff[x >> 6] = static_cast<uint32_t>(max(carry - x, static_cast<int64_t>(0)));
        next_bs += 64;
      }
    } else {
      const int64_t L = ni == nj ? oe - op + 1
                                 : merge_run<false>(old, op, oe, nw, ni, nj, r, del, out, int64_t{0}, acc);
      if (L > 0) {
        acc.F = fn_then(acc.F, Fn{x + L - 1, L});
        acc.used += static_cast<uint64_t>(L);
      }
    }
    ni = nj;
  }
  if (EMIT) {
    for (; next_bs < s1; next_bs += 64)
      noff[next_bs >> 6] = static_cast<uint32_t>(max(carry - next_bs, static_cast<int64_t>(0)));
    const int64_t ext_end = max(carry, s1 - 1);
    for (; wpos <= ext_end; ++wpos) out.emit(wpos, 0);
    out.flush();
  }
}

// ---- the staged path: one region in LDS, each lane a chunk of quotients ----
// Positions are int32: quotients relative to the region start, old slots as
// indexes into the staged blocks, new slots as indexes into the assembled
// output.  Maps are kept relative to the region start too (-1 = "none").

template <typename T>
struct OldStaged {
  const T *s;
  __device__ uint64_t slot(int32_t j) const { return s[j]; }
};
template <typename T>
struct SlotsRel {
  T *s;
  __device__ void emit(int32_t j, uint64_t v) { s[j] = static_cast<T>(v); }
};

// Next run end at or after staged index j, reading the staged run-end words
// through a one-word cursor (a lane's runs are visited in order).
struct EndCursor {
  const uint64_t *b;
  int32_t nw, w;
  uint64_t v;
  __device__ void init(const uint64_t *b_, int32_t nw_) {
    b = b_;
    nw = nw_;
    w = -1;
    v = 0;
  }
  __device__ int32_t next(int32_t j) {
    const int32_t wj = j >> 6;
    if (wj >= nw) return nw * 64 - 1;
    if (wj != w) {
      w = wj;
      v = b[wj];
    }
    uint64_t m = v & (~0ull << (j & 63));
    while (!m) {
      if (++w >= nw) return nw * 64 - 1;
      v = b[w];
      m = v;
    }
    return (w << 6) + ctz64(m);
  }
};

// The lane's old run ends, in order, from a 128-bit window of the staged
// run-end bits that starts after the end of the last old run before the chunk
// (a lane's runs almost always fit; the others use EndCursor).
struct WinEnds {
  uint64_t cur, nxt;
  int32_t base;
  __device__ void init(const uint64_t *b, int32_t nw, int32_t from) {
    const int32_t w = from >> 6, sh = from & 63;
    const uint64_t b0 = w < nw ? b[w] : 0ull, b1 = w + 1 < nw ? b[w + 1] : 0ull,
                   b2 = w + 2 < nw ? b[w + 2] : 0ull;
    cur = sh ? (b0 >> sh) | (b1 << (64 - sh)) : b0;
    nxt = sh ? (b1 >> sh) | (b2 << (64 - sh)) : b1;
    base = from;
    refill();
  }
  __device__ int count() const { return popc64(cur) + popc64(nxt); }
  __device__ void refill() {
    const bool empty = cur == 0;
    cur = empty ? nxt : cur;
    nxt = empty ? 0ull : nxt;
    base = empty ? base + 64 : base;
  }
  __device__ int32_t pop(int32_t) {
    const int32_t e = base + ctz64(cur);
    cur &= cur - 1;
    refill();
    return e;
  }
};
struct CurEnds {
  EndCursor ec;
  __device__ int32_t pop(int32_t o) { return ec.next(o); }
};

// One walk over the lane's quotients [t0, t0 + QT); occ / chg are the chunk's
// old-occupied bits and its bits of quotients that receive new entries.
// Pass 1 (EMIT = false): unchanged runs keep their length and are composed
// into maps, cut at every changed run, whose old extent is recorded for the
// merge: first = the maps before the lane's first changed run, gaf[c] = those
// after changed run c up to the next one (or the chunk's end).
// Pass 2 (EMIT = true), from the lane's carry (relative end of all earlier
// runs): copies unchanged runs to their new place, reserves the changed runs'
// slots (cst), sets run-end bits (output buffers start zeroed, so gaps cost
// nothing) and collects the chunk's new occupied bits.  Returns the carry
// after quotient t0 (for the offset of a block starting there).
template <bool EMIT, typename T, class Ends>
__device__ __forceinline__ int32_t lane_walk(int32_t t0, uint32_t occ, uint32_t chg, int32_t ob, int32_t ope,
                                             Ends ends, uint32_t c, uint16_t *cop, uint16_t *coe, Fn32 *gaf,
                                             Fn32 &first, uint32_t &used, const uint32_t *cL, uint16_t *cst,
                                             const T *old_s, T *new_s, uint64_t *new_b, int32_t xb,
                                             int32_t carry, uint32_t &nocc) {
  uint32_t u = occ | chg;
  Fn32 G = f32_id();
  bool seen = false;
  int32_t c_t0 = carry;
  int32_t cw = -1;
  uint64_t bits = 0;
  while (u) {
    const int b = __builtin_ctz(u);
    u &= u - 1;
    const int32_t x = t0 + b;
    const bool ch = (chg >> b) & 1u;
    int32_t o = 0, e = -1;
    if ((occ >> b) & 1u) {
      o = max(x - ob, ope + 1);
      e = ends.pop(o);
      ope = e;
    }
    if (!EMIT) {
      if (ch) {
        // staged indexes are < CAP < 0xFFFF, so 0xFFFF marks "no old run";
        // `first` is a value select, not a store through a pointer picked
        // between LDS and the lane's own variable
        cop[c] = static_cast<uint16_t>(o);
        coe[c] = e >= o ? static_cast<uint16_t>(e) : static_cast<uint16_t>(0xFFFF);
        first = seen ? first : G;
        if (seen) gaf[c - 1] = G;
        seen = true;
        G = f32_id();
        ++c;
      } else {
        const int32_t L = e - o + 1;
        G = f32_then(G, Fn32{x + L - 1, L});
        used += static_cast<uint32_t>(L);
      }
    } else {
      const int32_t L = ch ? static_cast<int32_t>(cL[c]) : e - o + 1;
      if (L > 0) {
        const int32_t p = max(x, carry + 1) - xb;
        if (ch) {
          cst[c] = static_cast<uint16_t>(p);
        } else {
          new_s[p] = old_s[o];
          for (int32_t k = 1; k < L; ++k) new_s[p + k] = old_s[o + k];
        }
        const int32_t pe = p + L - 1;
        carry = pe + xb;
        if ((pe >> 6) != cw) {
          if (bits) atomicOr(reinterpret_cast<ull *>(&new_b[cw]), static_cast<ull>(bits));
          cw = pe >> 6;
          bits = 0;
        }
        bits |= 1ull << (pe & 63);
        nocc |= 1u << b;
      }
      if (ch) ++c;
      c_t0 = b == 0 ? carry : c_t0;
    }
  }
  if (!EMIT) {
    first = seen ? first : G;
    if (seen) gaf[c - 1] = G;
  } else if (bits) {
    atomicOr(reinterpret_cast<ull *>(&new_b[cw]), static_cast<ull>(bits));
  }
  return c_t0;
}

// index of the k-th (0-based) set bit of v (v has more than k set bits), by
// halving with popcounts
__device__ __forceinline__ int select64_fast(uint64_t v, int k) {
  int pos = 0;
  uint32_t w = static_cast<uint32_t>(v);
  int c = __popc(w);
  if (k >= c) {
    k -= c;
    w = static_cast<uint32_t>(v >> 32);
    pos = 32;
  }
#pragma unroll
  for (int h = 16; h >= 1; h >>= 1) {
    c = __popc(w & ((1u << h) - 1u));
    if (k >= c) {
      k -= c;
      w >>= h;
      pos += h;
    }
  }
  return pos;
}

// the rare whole-region path: one lane, global memory in and out (inlined: an
// out-of-line call would cost the whole kernel a call frame and registers)
template <typename T, bool EMIT>
__device__ __forceinline__ void walk_global(const Block<T> *ob, Block<T> *nbk, int64_t nblocks,
                                         const uint64_t *ufp, const uint64_t *ucnt, uint64_t fbase,
                                         uint64_t fmask, uint32_t r,
                                         int del, int64_t RS, const uint64_t *occ_l, int64_t x0,
                                         int64_t x1, int64_t s0, int64_t s1, int64_t ope,
                                         uint64_t ni, uint64_t nb, int64_t hi, int64_t carry,
                                         Acc *acc, uint64_t *nocc_l, OffRef<T> noff) {
  OldGlb<T> old{ob, nblocks};
  NewGlb nw{ufp, ucnt, fbase, fmask};
  Acc a = *acc;
  if (EMIT) {
    OutGlb<T> out;
    out.init(nbk, hi);
    walk<T, true>(r, del, RS, occ_l, x0, x1, s0, s1, ope, ni, nb, old, nw, out, carry, a, nocc_l, noff);
  } else {
    NoOut out;
    walk<T, false>(r, del, RS, occ_l, x0, x1, s0, s1, ope, ni, nb, old, nw, out, carry, a, nocc_l, noff);
  }
  *acc = a;
}

// ---- block-wide helpers (256 lanes = 4 waves) ---------------------------
__device__ __forceinline__ Fn block_exscan_fn(Fn v, Fn *sh, Fn *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  Fn inc = v;
  for (int d = 1; d < 64; d <<= 1) {
    Fn o;
    o.A = __shfl_up(inc.A, d);
    o.B = __shfl_up(inc.B, d);
    if (lane >= d) inc = fn_then(o, inc);
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  Fn wpre = fn_id(), tot = fn_id();
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wv) wpre = fn_then(wpre, sh[w]);
    tot = fn_then(tot, sh[w]);
  }
  Fn ex;
  ex.A = __shfl_up(inc.A, 1);
  ex.B = __shfl_up(inc.B, 1);
  if (lane == 0) ex = fn_id();
  *total = tot;
  __syncthreads();
  return fn_then(wpre, ex);
}

__device__ __forceinline__ uint32_t block_exscan_u32(uint32_t v, uint32_t *sh, uint32_t *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  uint32_t wpre = 0, tot = 0;
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wv) wpre += sh[w];
    tot += sh[w];
  }
  *total = tot;
  __syncthreads();
  return wpre + inc - v;
}

// two exclusive sums at once (one set of barriers); sh holds 2 * NT / 64 words
__device__ __forceinline__ uint2 block_exscan2_u32(uint2 v, uint32_t *sh, uint2 *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint2 inc = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t ox = __shfl_up(inc.x, d), oy = __shfl_up(inc.y, d);
    if (lane >= d) {
      inc.x += ox;
      inc.y += oy;
    }
  }
  if (lane == 63) {
    sh[2 * wv] = inc.x;
    sh[2 * wv + 1] = inc.y;
  }
  __syncthreads();
  uint2 wpre = make_uint2(0, 0), tot = make_uint2(0, 0);
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wv) {
      wpre.x += sh[2 * w];
      wpre.y += sh[2 * w + 1];
    }
    tot.x += sh[2 * w];
    tot.y += sh[2 * w + 1];
  }
  *total = tot;
  __syncthreads();
  return make_uint2(wpre.x + inc.x - v.x, wpre.y + inc.y - v.y);
}

// four sums at once (one set of barriers); sh holds 4 * NT / 64 words
__device__ __forceinline__ void block_sum4_u64(uint64_t v[4], uint64_t *sh) {
  for (int k = 0; k < 4; ++k) {
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
    if ((threadIdx.x & 63) == 0) sh[4 * (threadIdx.x >> 6) + k] = v[k];
  }
  __syncthreads();
  for (int k = 0; k < 4; ++k) {
    uint64_t t = 0;
    for (int w = 0; w < NT / 64; ++w) t += sh[4 * w + k];
    v[k] = t;
  }
  __syncthreads();
}


// Carry-in of region R (called by the 64 lanes of one wave) of a filter whose
// first region is R0: lane l looks at regions hi - LBK l - k, k < LBK; the
// nearest region with a known inclusive carry ends the walk (before R0 the
// carry is -1), the aggregates of the regions in between are composed in
// order (per lane, then across the wave by an ordered tree).  One memory
// round trip covers 64 LBK predecessors.
// Work-groups are dispatched in index order on each XCD, so a region's
// predecessors have all started; the spin is still bounded: after LB_IDLE
// consecutive rounds without progress the wave gives up, flags the batch
// (which then is not applied) and returns a carry of -1.
constexpr int LBK = 1;
constexpr uint32_t LB_IDLE = 1u << 20;
__device__ int64_t look_back_wave(const uint64_t *tags, uint32_t nreg, uint32_t epoch, int64_t R,
                                  int64_t R0, bool *stalled) {
  const int lane = threadIdx.x & 63;
  Fn acc = fn_id();  // regions (hi, R-1], applied in order
  int64_t hi = R - 1;
  uint32_t idle = 0;
  for (;;) {
    Fn g[LBK];
    int64_t v[LBK];
    int first_inc = LBK, first_miss = LBK;  // within the lane, nearest first
#pragma unroll
    for (int k = LBK - 1; k >= 0; --k) {
      const int64_t j = hi - LBK * lane - k;
      g[k] = fn_id();
      v[k] = -1;
      if (j < R0) {
        first_inc = k;  // before the filter's first region the carry is -1
      } else {
        int64_t tv = 0, tA = 0, tB = 0;
        const bool hv = tag_load(&tags[2ull * nreg + j], epoch, &tv);
        const bool hA = tag_load(&tags[j], epoch, &tA);
        const bool hB = tag_load(&tags[static_cast<uint64_t>(nreg) + j], epoch, &tB);
        if (hv) {
          first_inc = k;
          v[k] = tv;
        } else if (hA && hB) {
          g[k] = Fn{tA, tB};
        } else {
          first_miss = k;
        }
      }
    }
    const uint64_t im = __ballot(first_inc < LBK), mm = __ballot(first_miss < LBK);
    const int il = im ? ctz64(im) : 0, ml = mm ? ctz64(mm) : 0;
    const int fi = __shfl(first_inc, il), fm = __shfl(first_miss, ml);
    const int stop = im ? LBK * il + fi : 64 * LBK;
    const int miss = mm ? LBK * ml + fm : 64 * LBK;
    const int take = min(stop, miss);  // positions [0, take) hold usable aggregates
    // the lane's aggregates below `take`, farthest first
    Fn M = fn_id();
#pragma unroll
    for (int k = LBK - 1; k >= 0; --k)
      if (LBK * lane + k < take) M = fn_then(M, g[k]);
    // ordered tree over the lanes: higher lanes hold earlier regions
    for (int d = 1; d < 64; d <<= 1) {
      Fn o;
      o.A = __shfl_down(M.A, d);
      o.B = __shfl_down(M.B, d);
      if ((lane & (2 * d - 1)) == 0 && lane + d < 64) M = fn_then(o, M);
    }
    Fn T;
    T.A = __shfl(M.A, 0);
    T.B = __shfl(M.B, 0);
    acc = fn_then(T, acc);
    if (stop < 64 * LBK && stop <= miss) {
      const int k = stop % LBK;
      int64_t vk = v[0];
#pragma unroll
      for (int q = 1; q < LBK; ++q)
        if (k == q) vk = v[q];
      const int64_t c = __shfl(vk, stop / LBK);
      return fn_apply(acc, c);
    }
    hi -= take;
    if (take == 0) {
      if (++idle > LB_IDLE) {
        *stalled = true;
        return -1;
      }
      __builtin_amdgcn_s_sleep(2);
    } else {
      idle = 0;
    }
  }
}

// The kernel's LDS arrays, handed to the region body.
template <typename T>
struct Smem {
  T *old_s;
  T *new_s;
  uint64_t *old_b;
  uint64_t *new_b;
  uint32_t *old_wp;
  uint64_t *occ_l;
  uint64_t *chg_l;
  uint32_t *nfp_l;
  uint32_t *ncnt_l;
  uint16_t *cxr_l;
  uint32_t *chead_l;
  uint16_t *cop_l;
  uint16_t *coe_l;
  uint32_t *cL_l;
  uint16_t *cst_l;
  Fn32 *gaf_l;
  int64_t *sh_i;
  Fn *sh_fn;
  uint32_t *sh_u;
  uint64_t *sh_r;
};

// One region (see k_merge).  SMALL: the region's entries fit the LDS arrays.
template <typename T, bool SINGLE, bool SMALL>
__device__ __forceinline__ void merge_body(const MergeArgs &a, const Smem<T> &m) {
  using C = Cfg<T>;
  T *const old_s = m.old_s;
  T *const new_s = m.new_s;
  uint64_t *const old_b = m.old_b;
  uint64_t *const new_b = m.new_b;
  uint32_t *const old_wp = m.old_wp;
  uint64_t *const occ_l = m.occ_l;
  uint64_t *const chg_l = m.chg_l;
  uint32_t *const nfp_l = m.nfp_l;
  uint32_t *const ncnt_l = m.ncnt_l;
  uint16_t *const cxr_l = m.cxr_l;
  uint32_t *const chead_l = m.chead_l;
  uint16_t *const cop_l = m.cop_l;
  uint16_t *const coe_l = m.coe_l;
  uint32_t *const cL_l = m.cL_l;
  uint16_t *const cst_l = m.cst_l;
  Fn32 *const gaf_l = m.gaf_l;
  int64_t *const sh_i = m.sh_i;
  Fn *const sh_fn = m.sh_fn;
  uint32_t *const sh_u = m.sh_u;
  uint64_t *const sh_r = m.sh_r;
  const int tid = threadIdx.x;
  // global region = work-group index (no shared ticket counter: one atomic
  // per work-group on one address serialises the whole launch); the filter
  // and its local region R follow from the pipeline's region map
  const uint32_t gR = a.areg ? a.areg[blockIdx.x] : blockIdx.x;
  // (a one-filter pipeline takes its descriptor from the kernel arguments,
  // saving two dependent loads before the region's first load)
  const FDesc &fd = SINGLE ? a.one : a.desc[a.rmap[gR]];
  const int64_t R = gR - fd.rbase;
  const uint32_t rlog = fd.rlog;
  const int64_t FN = fd.N, FP = fd.P, FNB = fd.nblocks;
  uint64_t *const fstate = fd.state;
  const int32_t S = 1 << rlog;
  const int64_t RS = R << rlog;
  // (selects, not a dynamic index into a struct, which would put it in
  // scratch memory)
  const int cur = static_cast<int>(fstate[ST_CUR] & 1ull);
  const Block<T> *ob = static_cast<const Block<T> *>(cur ? fd.blk[1] : fd.blk[0]);
  Block<T> *nbk = static_cast<Block<T> *>(cur ? fd.blk[0] : fd.blk[1]);
  const OffRef<T> noff{nbk};
  // the same pointers typed as global memory for the hot loads and stores
  // (they come from a descriptor in memory, so the compiler cannot tell)
  const GPtr<const Block<T>> gob = to_global(ob);
  const GPtr<Block<T>> gnbk = to_global(nbk);
  const GPtr<const uint64_t> gufp = to_global(a.ufp);
  const GPtr<const uint64_t> gucnt = to_global(a.ucnt);
  const bool qreg = RS < FN;
  const int64_t send = min(RS + S, FP);
  const int nw_reg = static_cast<int>((send - RS + 63) >> 6);
  const uint64_t rb0 = a.rb[gR], rb1 = a.rb[gR + 1];
  const uint64_t ne = rb1 - rb0;
  const uint32_t r = fd.r;
  const uint64_t lmask = (1ull << (rlog + r)) - 1ull;  // fingerprint bits inside the region
  const uint32_t epoch = next_epoch(a.pst[ST_EPOCH]);
  // the region's old runs: slots [lo_old, hi_old] (the carries at its two
  // boundaries).  All of the region's loads below depend only on these and
  // the words above, so they are requested before the first barrier.
  const int64_t lo_old = qreg ? a.cb[gR] + 1 : RS;
  const int64_t hi_old = qreg ? a.cb[gR + 1] : RS - 1;
  const bool has_old = hi_old >= lo_old;
  const int64_t bb = has_old ? (lo_old >> 6) : (RS >> 6);
  const int64_t nblk64 = has_old ? (hi_old >> 6) - bb + 1 : 0;
  // the staged path: the old runs fit in LDS (and positions in int32)
  const bool par = ne < (1ull << 31) && nblk64 <= C::CAPW && (bb << 6) - RS < (1ll << 30);
  const int nblk = par ? static_cast<int>(nblk64) : 0;
  const int32_t obr = static_cast<int32_t>(par ? (bb << 6) - RS : 0);  // staged base - RS

  // Every lane first requests all of its staging loads (the region's
  // occupied words, its first new entries, the old blocks' slots and run-end
  // words), then writes them to LDS: one memory round trip instead of one per
  // array.  (Counts per lane are bounded: at most OW <= NT occupied words,
  // CAPW <= NT run-end words and CAPW * CH <= BCH * NT slot chunks.)
  static_assert(C::OW <= NT && C::CAPW <= NT, "one occupied and one run-end word per lane");
  constexpr int BCH = (C::CAPW * C::CH + NT - 1) / NT;
  constexpr int ECH = 2;  // new entries per lane requested up front
  const uint64_t ov = (qreg && tid < nw_reg) ? gob[(RS >> 6) + tid].occ : 0ull;
  uint64_t ef[ECH], ec[ECH];
#pragma unroll
  for (int k = 0; k < ECH; ++k) {
    const uint64_t i = static_cast<uint64_t>(tid) + static_cast<uint64_t>(k) * NT;
    const bool ok = ne < (1ull << 31) && i < ne;
    ef[k] = ok ? gufp[rb0 + i] : 0ull;
    ec[k] = ok ? gucnt[rb0 + i] : 0ull;
  }
  u32x4 bv[BCH];
#pragma unroll
  for (int k = 0; k < BCH; ++k) {
    const int idx = tid + k * NT;
    bv[k] = u32x4{0u, 0u, 0u, 0u};
    if (par && idx < nblk * C::CH)
      bv[k] = reinterpret_cast<GPtr<const u32x4>>(gob[bb + idx / C::CH].s)[idx % C::CH];
  }
  const uint64_t rv = (par && tid < nblk) ? gob[bb + tid].rend : 0ull;

  if (tid < nw_reg) {
    occ_l[tid] = ov;
    chg_l[tid] = 0ull;
  }
  for (int w = tid; w < C::CAPW; w += NT) new_b[w] = 0ull;
  for (int i = tid; i < C::CAP * static_cast<int>(sizeof(T)) / 16; i += NT)
    reinterpret_cast<uint4 *>(new_s)[i] = make_uint4(0u, 0u, 0u, 0u);
  // (SMALL is a template argument, so the LDS case compiles to LDS
  // instructions rather than generic ones)
  uint32_t *const nfp = SMALL ? nfp_l : a.g_fp + rb0;
  uint32_t *const ncnt = SMALL ? ncnt_l : a.g_cnt + rb0;
  uint16_t *const cxr = SMALL ? cxr_l : a.g_xr + rb0;
  uint32_t *const chead = SMALL ? chead_l : a.g_head + rb0;
  uint16_t *const cop = SMALL ? cop_l : a.g_op + rb0;
  uint16_t *const coe = SMALL ? coe_l : a.g_oe + rb0;
  uint32_t *const cL = SMALL ? cL_l : a.g_L + rb0;
  uint16_t *const cst = SMALL ? cst_l : a.g_st + rb0;
  Fn32 *const gaf = SMALL ? gaf_l : a.g_gaf + rb0;
  if (ne < (1ull << 31)) {
#pragma unroll
    for (int k = 0; k < ECH; ++k) {
      const uint32_t i = static_cast<uint32_t>(tid + k * NT);
      if (i < ne) {
        nfp[i] = static_cast<uint32_t>(ef[k] & lmask);
        ncnt[i] = static_cast<uint32_t>(ec[k]);
      }
    }
    // (more than ECH entries per lane: the global-memory path's regions)
    for (uint32_t i = tid + ECH * NT; i < ne; i += NT) {
      nfp[i] = static_cast<uint32_t>(gufp[rb0 + i] & lmask);
      ncnt[i] = static_cast<uint32_t>(gucnt[rb0 + i]);
    }
  }
  // 16-byte chunks of the staged blocks' slots, then their run-end words
#pragma unroll
  for (int k = 0; k < BCH; ++k) {
    const int idx = tid + k * NT;
    if (par && idx < nblk * C::CH) reinterpret_cast<u32x4 *>(old_s)[idx] = bv[k];
  }
  if (par && tid < nblk) {
    uint64_t v = rv;
    if (tid == 0) v &= ~0ull << (lo_old & 63);
    if (tid == nblk - 1) v &= ~0ull >> (63 - (hi_old & 63));
    old_b[tid] = v;
  }
  __syncthreads();
  // changed runs = groups of equal quotient among the new entries, found in
  // rounds of 2 NT entries ([2 tid, 2 tid + 2) per lane; one round unless the
  // region has more than NCAP entries)
  uint32_t nchg = 0;
  const uint32_t ne32 = par ? static_cast<uint32_t>(ne) : 0u;
  for (uint32_t base = 0; base < ne32; base += 2 * NT) {
    uint32_t h0 = 0, h1 = 0;
    const uint32_t e0 = base + 2u * tid, e1 = e0 + 1;
    const uint32_t x0 = e0 < ne32 ? nfp[e0] >> r : 0u;
    const uint32_t x1 = e1 < ne32 ? nfp[e1] >> r : 0u;
    if (e0 < ne32) h0 = e0 == 0 || x0 != (nfp[e0 - 1] >> r);
    if (e1 < ne32) h1 = x1 != x0;
    uint32_t tot;
    const uint32_t ex = nchg + block_exscan_u32(h0 + h1, sh_u, &tot);
    nchg += tot;
    if (h0) {
      cxr[ex] = static_cast<uint16_t>(x0);
      chead[ex] = e0;
      atomicOr(reinterpret_cast<ull *>(&chg_l[x0 >> 6]), static_cast<ull>(1ull << (x0 & 63)));
    }
    if (h1) {
      cxr[ex + h0] = static_cast<uint16_t>(x1);
      chead[ex + h0] = e1;
      atomicOr(reinterpret_cast<ull *>(&chg_l[x1 >> 6]), static_cast<ull>(1ull << (x1 & 63)));
    }
  }
  __syncthreads();
  // the lane's chunk of quotients [t0, t0 + QT), its bits, and prefix counts:
  // run ends per staged word (for select), occupied and changed quotients
  // before the chunk (its first old run, its first changed run)
  const int QT = max(S >> 8, 1);
  const int32_t t0 = tid * QT;
  const bool chunk = par && qreg && t0 < S;
  uint32_t occ_c = 0, chg_c = 0;
  if (chunk) {
    const uint32_t m = QT >= 32 ? ~0u : ((1u << QT) - 1u);
    occ_c = static_cast<uint32_t>(occ_l[t0 >> 6] >> (t0 & 63)) & m;
    chg_c = static_cast<uint32_t>(chg_l[t0 >> 6] >> (t0 & 63)) & m;
  }
  uint2 tot2;
  const uint32_t pw = (par && tid < nblk) ? static_cast<uint32_t>(popc64(old_b[tid])) : 0u;
  const uint2 ex2 = block_exscan2_u32(
      make_uint2(pw, static_cast<uint32_t>(__popc(occ_c)) | (static_cast<uint32_t>(__popc(chg_c)) << 16)),
      sh_u, &tot2);
  if (par && tid < nblk) old_wp[tid] = ex2.x;
  if (par && tid == 0) old_wp[nblk] = tot2.x;
  const uint32_t kocc = ex2.y & 0xFFFFu, c0 = ex2.y >> 16;
  const uint32_t c1 = c0 + static_cast<uint32_t>(__popc(chg_c));
  __syncthreads();
  // staged index of the end of the last old run before the chunk
  int32_t ope0 = static_cast<int32_t>(lo_old - RS) - obr - 1;
  if (chunk && occ_c && kocc > 0) {
    const uint32_t k = kocc - 1;
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (old_wp[mid] <= k) lo = mid; else hi = mid - 1;
    }
    ope0 = (lo << 6) + select64_fast(old_b[lo], static_cast<int>(k - old_wp[lo]));
  }

  Acc acc{fn_id(), 0, 0, 0, 0, 0};
  Fn Flane = fn_id();
  if (par) {
    // ---- pass 1: the lane's unchanged runs, cut at its changed runs -------
    Fn32 first = f32_id();
    uint32_t used = 0;
    if (chunk) {
      uint32_t dn = 0;
      T *dt = nullptr;
      WinEnds we;
      we.init(old_b, nblk, ope0 + 1);
      if (we.count() >= __popc(occ_c)) {
        lane_walk<false, T>(t0, occ_c, chg_c, obr, ope0, we, c0, cop, coe, gaf, first, used, cL, cst, old_s,
                            dt, new_b, 0, 0, dn);
      } else {
        CurEnds ce;
        ce.ec.init(old_b, nblk);
        lane_walk<false, T>(t0, occ_c, chg_c, obr, ope0, ce, c0, cop, coe, gaf, first, used, cL, cst, old_s,
                            dt, new_b, 0, 0, dn);
      }
    }
    __syncthreads();
    // ---- pass 1a: new lengths of the changed runs, one run per lane --------
    NewRel nw{nfp, ncnt};
    OldStaged<T> old{old_s};
    NoOut none;
    for (uint32_t c = tid; c < nchg; c += NT) {
      const uint32_t ni = chead[c], nj = c + 1 < nchg ? chead[c + 1] : static_cast<uint32_t>(ne);
      const bool ho = coe[c] != 0xFFFF;
      const int32_t L = merge_run<false>(old, ho ? static_cast<int32_t>(cop[c]) : 0,
                                         ho ? static_cast<int32_t>(coe[c]) : -1, nw, ni, nj, r, a.del, none,
                                         int32_t{0}, acc);
      cL[c] = static_cast<uint32_t>(L);
      used += static_cast<uint32_t>(L);
    }
    __syncthreads();
    // ---- the lane's map: its segments and changed runs in quotient order ---
    Fn32 F = first;
    for (uint32_t c = c0; c < c1; ++c) {
      const int32_t L = static_cast<int32_t>(cL[c]);
      if (L > 0) F = f32_then(F, Fn32{static_cast<int32_t>(cxr[c]) + L - 1, L});
      F = f32_then(F, gaf[c]);
    }
    Flane.A = F.A >= 0 ? RS + F.A : RS - 1;
    Flane.B = F.B;
    acc.used = used;
  } else if (tid == 0) {
    Acc ag{fn_id(), 0, 0, 0, 0, 0};
    walk_global<T, false>(ob, nbk, FNB, a.ufp, a.ucnt, static_cast<uint64_t>(RS) << r, lmask, r, a.del, RS, occ_l, qreg ? RS : 0,
                          qreg ? send : 0, RS, send, lo_old - 1, rb0, rb1, 0, 0, &ag, chg_l, noff);
    acc = ag;
    Flane = ag.F;
  }
  Fn Ftot;
  const Fn Fex = block_exscan_fn(Flane, sh_fn, &Ftot);
  uint64_t sums[4] = {acc.used, acc.dent, acc.dtot, acc.shortfall};
  block_sum4_u64(sums, sh_r);
  const uint64_t used = sums[0], dent = sums[1], dtot = sums[2], shortfall = sums[3];
  const bool ovf = __syncthreads_or(acc.ovf != 0) != 0;

  if (tid == 0) {
    tag_store(&a.tags[gR], epoch, Ftot.A);
    tag_store(&a.tags[static_cast<uint64_t>(a.G) + gR], epoch, Ftot.B);
  }
  if (tid < 64) {
    bool stalled = false;
    const int64_t c_in = look_back_wave(a.tags, a.G, epoch, gR, fd.rbase, &stalled);
    if (tid == 0) {
      if (stalled) atomic_or_u64(&fstate[ST_BATCH], BATCH_STALL);
      const int64_t c_out = fn_apply(Ftot, c_in);
      tag_store(&a.tags[2ull * a.G + gR], epoch, c_out);
      sh_i[3] = c_in;
      sh_i[4] = c_out;
      // errors are rare and set one shared word; the statistics go to the
      // region's own words and are summed after the launch
      if (c_out >= FP) atomic_or_u64(&fstate[ST_BATCH], BATCH_FULL);
      if (ovf) atomic_or_u64(&fstate[ST_BATCH], BATCH_OVF);
      uint64_t *st = a.rstat + 4ull * gR;
      st[0] = used;
      st[1] = dent;
      st[2] = dtot;
      st[3] = shortfall;
    }
  }
  __syncthreads();

  // ---- pass 2: write the region's extent into the other copy --------------
  // A region whose runs pass the last slot fails the whole batch (the other
  // copy never becomes current), so it writes nothing; every other region's
  // runs end below P, which bounds all writes below.
  const int64_t c_in = sh_i[3], c_out = sh_i[4];
  const bool emit = c_out < FP;
  const int64_t ext_lo = max(c_in + 1, RS);
  const int64_t ext_hi = max(c_out, send - 1);
  const int64_t xbase = (ext_lo >> 6) << 6;
  const int nxb = ext_hi >= ext_lo ? static_cast<int>((ext_hi >> 6) - (ext_lo >> 6) + 1) : 0;
  const bool lds_out = emit && par && nxb <= C::CAPW && xbase - RS < (1ll << 30);
  if (lds_out) {
    const int32_t xb = static_cast<int32_t>(xbase - RS);
    uint32_t nocc = 0;
    if (chunk) {
      const int64_t c_t = fn_apply(Fex, c_in);
      const int32_t carry = static_cast<int32_t>(max(c_t - RS, static_cast<int64_t>(-1)));
      Fn32 df = f32_id();
      uint32_t du = 0;
      int32_t ct0;
      WinEnds we;
      we.init(old_b, nblk, ope0 + 1);
      if (we.count() >= __popc(occ_c)) {
        ct0 = lane_walk<true, T>(t0, occ_c, chg_c, obr, ope0, we, c0, cop, coe, gaf, df, du, cL, cst, old_s,
                                 new_s, new_b, xb, carry, nocc);
      } else {
        CurEnds ce;
        ce.ec.init(old_b, nblk);
        ct0 = lane_walk<true, T>(t0, occ_c, chg_c, obr, ope0, ce, c0, cop, coe, gaf, df, du, cL, cst, old_s,
                                 new_s, new_b, xb, carry, nocc);
      }
      if ((t0 & 63) == 0) gnbk[(RS + t0) >> 6].off = static_cast<uint32_t>(max(ct0 - t0, 0));
    }
    if (qreg) {
      // the new occupied words: OR the chunks of each 64-quotient word into
      // its first lane (all lanes take part in the shuffles)
      uint64_t wv = chunk ? static_cast<uint64_t>(nocc) << (t0 & 63) : 0ull;
      for (int d = 1; d < 64 / QT; d <<= 1) wv |= __shfl_down(wv, d);
      if (chunk && (t0 & 63) == 0) gnbk[(RS + t0) >> 6].occ = wv;
    } else {
      for (int w = tid; w < nw_reg; w += NT) {
        gnbk[(RS >> 6) + w].occ = 0ull;
        gnbk[(RS >> 6) + w].off = static_cast<uint32_t>(max(c_in - (RS + 64ll * w), static_cast<int64_t>(0)));
      }
    }
    __syncthreads();
    // 2b: the changed runs' slots, one run per lane
    NewRel nw{nfp, ncnt};
    OldStaged<T> old{old_s};
    SlotsRel<T> so{new_s};
    Acc dummy{fn_id(), 0, 0, 0, 0, 0};
    for (uint32_t c = tid; c < nchg; c += NT) {
      if (cL[c] == 0) continue;
      const uint32_t ni = chead[c], nj = c + 1 < nchg ? chead[c + 1] : static_cast<uint32_t>(ne);
      const bool ho = coe[c] != 0xFFFF;
      merge_run<true>(old, ho ? static_cast<int32_t>(cop[c]) : 0, ho ? static_cast<int32_t>(coe[c]) : -1, nw,
                      ni, nj, r, a.del, so, static_cast<int32_t>(cst[c]), dummy);
    }
    __syncthreads();
    // slots: whole 16-byte chunks inside the extent, single slots at its ends
    for (int idx = tid; idx < nxb * C::CH; idx += NT) {
      const int b = idx / C::CH, c = idx % C::CH;
      const int64_t p0 = xbase + b * 64 + c * C::PER;
      const int64_t p1 = p0 + C::PER - 1;
      GPtr<T> dst = gnbk[(xbase >> 6) + b].s + c * C::PER;
      const T *src = new_s + b * 64 + c * C::PER;
      if (p0 >= ext_lo && p1 <= ext_hi) {
        *reinterpret_cast<GPtr<u32x4>>(dst) = *reinterpret_cast<const u32x4 *>(src);
      } else {
        for (int k = 0; k < C::PER; ++k)
          if (p0 + k >= ext_lo && p0 + k <= ext_hi) dst[k] = src[k];
      }
    }
    for (int b = tid; b < nxb; b += NT) {
      const int64_t w = (xbase >> 6) + b;
      const int64_t plo = max(w << 6, ext_lo), phi = min((w << 6) + 63, ext_hi);
      const uint64_t mask = (~0ull >> (63 - (phi & 63))) & (~0ull << (plo & 63));
      const uint64_t v = new_b[b] & mask;
      if (mask == ~0ull) {
        gnbk[w].rend = v;
      } else {
        atomic_and_u64(&nbk[w].rend, ~mask);
        atomic_or_u64(&nbk[w].rend, v);
      }
    }
  } else if (emit) {
    // one lane redoes the whole region from global memory; chg_l collects
    // the new occupied bits
    for (int w = tid; w < nw_reg; w += NT) chg_l[w] = 0ull;
    __syncthreads();
    if (tid == 0) {
      Acc dummy{fn_id(), 0, 0, 0, 0, 0};
      walk_global<T, true>(ob, nbk, FNB, a.ufp, a.ucnt, static_cast<uint64_t>(RS) << r, lmask, r, a.del, RS, occ_l, qreg ? RS : 0,
                           qreg ? send : 0, RS, send, lo_old - 1, rb0, rb1, ext_hi, c_in, &dummy, chg_l, noff);
    }
    __syncthreads();
    for (int w = tid; w < nw_reg; w += NT) nbk[(RS >> 6) + w].occ = chg_l[w];
  }
}

template <typename T, bool SINGLE>
__global__ __launch_bounds__(NT) void k_merge(MergeArgs a) {
  using C = Cfg<T>;
  __shared__ __align__(16) T old_s[C::CAP];
  __shared__ __align__(16) T new_s[C::CAP];
  __shared__ uint64_t old_b[C::CAPW];
  __shared__ uint64_t new_b[C::CAPW];
  __shared__ uint32_t old_wp[C::CAPW + 1];
  __shared__ uint64_t occ_l[C::OW];
  // quotients that receive new entries; reused for the new occupied bits of
  // the one-lane path
  __shared__ uint64_t chg_l[C::OW];
  // the region's new entries, and its changed runs (one per distinct
  // quotient), in LDS when there are at most NCAP entries, else in the
  // launch's per-entry scratch
  __shared__ uint32_t nfp_l[C::NCAP];
  __shared__ uint32_t ncnt_l[C::NCAP];
  __shared__ uint16_t cxr_l[C::NCAP];   // quotient - RS
  __shared__ uint32_t chead_l[C::NCAP]; // first entry
  __shared__ uint16_t cop_l[C::NCAP];   // old run, staged indexes (coe 0xFFFF: none)
  __shared__ uint16_t coe_l[C::NCAP];
  __shared__ uint32_t cL_l[C::NCAP];    // new length
  __shared__ uint16_t cst_l[C::NCAP];   // new first slot, output index
  __shared__ Fn32 gaf_l[C::NCAP];       // maps of the unchanged runs after it
  __shared__ int64_t sh_i[8];
  __shared__ Fn sh_fn[NT / 64];
  __shared__ uint32_t sh_u[2 * NT / 64];
  __shared__ uint64_t sh_r[4 * NT / 64];

  const Smem<T> m{old_s, new_s, old_b, new_b, old_wp, occ_l, chg_l, nfp_l, ncnt_l, cxr_l, chead_l, cop_l, coe_l, cL_l, cst_l, gaf_l, sh_i, sh_fn, sh_u, sh_r};
  const uint32_t g = a.areg ? a.areg[blockIdx.x] : blockIdx.x;
  if (a.rb[g + 1] - a.rb[g] <= static_cast<uint64_t>(C::NCAP))
    merge_body<T, SINGLE, true>(a, m);
  else
    merge_body<T, SINGLE, false>(a, m);
}

// After the merge, per filter: work-group (f, y) sums the statistics of
// regions [y FIN_REG, (y + 1) FIN_REG) of filter f into the filter's
// accumulator words; the last of its work-groups (a ticket counter) takes the
// sums, clears the words for the next launch, flips the filter's current copy
// if none of its regions failed, else records the error (all-or-nothing per
// filter), and adds its delete shortfall to not_found[f].  Work-group (0, 0)
// records the launch's epoch as the pipeline's last.
__global__ __launch_bounds__(FIN_NT) void k_finish(const FDesc *__restrict__ desc, const uint32_t *__restrict__ afil,
                                                   const uint64_t *rstat, int del, uint64_t *not_found,
                                                   uint64_t *pst) {
  __shared__ uint64_t sh[4][FIN_NT / 64];
  const uint32_t f = afil ? afil[blockIdx.x] : blockIdx.x;
  const FDesc &d = desc[f];
  const uint32_t nsl = (d.nregions + FIN_REG - 1) / FIN_REG;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) pst[ST_EPOCH] = next_epoch(pst[ST_EPOCH]);
  if (blockIdx.y >= nsl) return;  // (the whole work-group)
  uint64_t v[4] = {0, 0, 0, 0};
  // (16-byte loads, several regions in flight per lane)
  const u32x4 *rs4 = reinterpret_cast<const u32x4 *>(rstat + 4ull * d.rbase);
  const uint32_t r1 = min(d.nregions, (blockIdx.y + 1) * FIN_REG);
#pragma unroll 8
  for (uint32_t R = blockIdx.y * FIN_REG + threadIdx.x; R < r1; R += FIN_NT) {
    const u32x4 a = rs4[2ull * R], b = rs4[2ull * R + 1];
    v[0] += (static_cast<uint64_t>(a[1]) << 32) | a[0];
    v[1] += (static_cast<uint64_t>(a[3]) << 32) | a[2];
    v[2] += (static_cast<uint64_t>(b[1]) << 32) | b[0];
    v[3] += (static_cast<uint64_t>(b[3]) << 32) | b[2];
  }
  for (int k = 0; k < 4; ++k) {
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = v[k];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  uint64_t t[4] = {0, 0, 0, 0};
  for (int k = 0; k < 4; ++k)
    for (int w = 0; w < FIN_NT / 64; ++w) t[k] += sh[k][w];
  uint64_t *state = d.state;
  if (nsl > 1) {
    for (int k = 0; k < 4; ++k)
      if (t[k]) atomicAdd(reinterpret_cast<ull *>(&state[ST_ACC + k]), static_cast<ull>(t[k]));
    __threadfence();
    const uint64_t tk = atomicAdd(reinterpret_cast<ull *>(&state[ST_TICKET]), 1ull);
    if (tk != nsl - 1) return;
    // the last work-group: every other one's sums are in the words
    __threadfence();
    for (int k = 0; k < 4; ++k) t[k] = atomicExch(reinterpret_cast<ull *>(&state[ST_ACC + k]), 0ull);
    (void)atomicExch(reinterpret_cast<ull *>(&state[ST_TICKET]), 0ull);
  }
  const uint64_t st = state[ST_BATCH];
  if (st == 0) {
    state[ST_USED] = t[0];
    state[ST_DIST] += t[1];
    state[ST_TOTAL] += t[2];
    state[ST_CUR] ^= 1ull;
  } else if (state[ST_ERR] == 0) {
    state[ST_ERR] = static_cast<uint64_t>((st & BATCH_STALL) ? QF_ERR_STALLED
                                          : (st & BATCH_FULL) ? QF_ERR_FULL
                                                              : QF_ERR_COUNT_OVERFLOW);
  }
  if (del && not_found) not_found[f] += t[3];
  state[ST_BATCHES] += 1;
}

template <typename T>
hipError_t launch_merge_t(Pipe &p, const uint64_t *ufp, const uint64_t *ucnt, int del, uint64_t *not_found,
                          hipStream_t s) {
  MergeArgs a;
  a.desc = p.d_desc;
  a.rmap = p.d_rmap;
  a.ufp = ufp;
  a.ucnt = ucnt;
  a.rb = p.rb;
  a.tags = p.tags;
  a.rstat = p.rstat;
  a.cb = p.cb;
  a.G = p.G;
  a.pst = p.pst;
  a.del = del;
  // per-entry scratch: bufE holds cap entries of 32 bytes
  uint8_t *e = reinterpret_cast<uint8_t *>(p.bufE);
  const uint64_t cap = p.cap;
  a.g_fp = reinterpret_cast<uint32_t *>(e);
  a.g_cnt = reinterpret_cast<uint32_t *>(e + 4 * cap);
  a.g_head = reinterpret_cast<uint32_t *>(e + 8 * cap);
  a.g_L = reinterpret_cast<uint32_t *>(e + 12 * cap);
  a.g_gaf = reinterpret_cast<Fn32 *>(e + 16 * cap);
  a.g_xr = reinterpret_cast<uint16_t *>(e + 24 * cap);
  a.g_op = reinterpret_cast<uint16_t *>(e + 26 * cap);
  a.g_oe = reinterpret_cast<uint16_t *>(e + 28 * cap);
  a.g_st = reinterpret_cast<uint16_t *>(e + 30 * cap);
  if (p.timer) p.timer->begin(QF_PROF_MERGE, s);
  // the launch's regions: all, or those of the listed filters
  const uint32_t *areg = p.nareg ? p.d_areg : nullptr;
  const uint32_t nreg = p.nareg ? p.nareg : p.G;
  a.areg = areg;
  const uint32_t ncar = nreg > p.G ? nreg : p.G;
  k_carries<T><<<(ncar + NT - 1) / NT, NT, 0, s>>>(p.d_desc, p.d_rmap, areg, nreg, p.cb, p.tags, p.G, p.pst);
  if (p.nf == 1) {
    a.one = p.one;
    k_merge<T, true><<<nreg, NT, 0, s>>>(a);
  } else {
    k_merge<T, false><<<nreg, NT, 0, s>>>(a);
  }
  k_finish<<<dim3(p.nareg ? p.nafil : p.nf, p.fin_slices), FIN_NT, 0, s>>>(
      p.d_desc, p.nareg ? p.d_afil : nullptr, p.rstat, del, not_found, p.pst);
  if (p.timer) p.timer->end(QF_PROF_MERGE, s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_merge(Pipe &p, const uint64_t *ufp, const uint64_t *ucnt, int del, uint64_t *not_found,
                        hipStream_t s) {
  if (p.r == 8) return launch_merge_t<uint8_t>(p, ufp, ucnt, del, not_found, s);
  return launch_merge_t<uint16_t>(p, ufp, ucnt, del, not_found, s);
}

int max_region_log2(uint32_t r) { return r == 8 ? Cfg<uint8_t>::SMAXLOG : Cfg<uint16_t>::SMAXLOG; }

}  // namespace qf
