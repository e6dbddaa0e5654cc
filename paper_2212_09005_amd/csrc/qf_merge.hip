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
//     of quotients.  Pass 1 composes the lanes' run maps; a run that receives
//     no new entry keeps its length, read off the run-end bits without
//     decoding.  A block scan of the maps gives each lane its carry; pass 2
//     copies unchanged runs, decodes/merges/re-encodes the others, assembles
//     the region's new slots in LDS and writes them with 16-byte stores.
//     Regions whose runs or entries do not fit in LDS are done by one lane
//     straight from and to global memory.
#include "qf.h"
#include "qf_dev.h"
#include "qf_lib.h"

namespace qf {
namespace {

constexpr int NT = 256;
constexpr int64_t INF = INT64_MAX / 4;

template <typename T>
struct Cfg {
  // largest region: 8192 slots (r = 8), 4096 (r = 16); LDS buffers hold 1.5
  // regions of slots (a region's runs plus what spills past its end)
  static constexpr int SMAXLOG = sizeof(T) == 1 ? 13 : 12;
  static constexpr int SMAX = 1 << SMAXLOG;
  static constexpr int CAP = SMAX + SMAX / 2;
  static constexpr int CAPW = CAP / 64;
  static constexpr int OW = SMAX / 64;
  static constexpr int NCAP = 512;  // new entries staged in LDS (2 per lane)
  static constexpr int CH = 64 * static_cast<int>(sizeof(T)) / 16;  // 16-byte chunks per block
  static constexpr int PER = 16 / static_cast<int>(sizeof(T));      // slots per chunk
};

template <typename T>
struct MergeArgs {
  Block<T> *blk[2];
  uint32_t *off[2];
  int64_t N, P, nblocks;
  uint32_t r, rlog, nregions;
  const uint64_t *ufp, *ucnt, *rb;
  uint64_t *tags;
  uint32_t epoch;
  uint64_t *state;
  int del;
  uint64_t *not_found;
};

// ---- readers of the current (old) table -------------------------------------
template <typename T>
struct OldLds {  // whole blocks staged from slot `base` (a multiple of 64); hi = last slot
  const T *s;
  const uint64_t *b;  // run-end words, bits outside the region's span cleared
  int64_t base, hi;
  __device__ uint64_t slot(int64_t j) const { return s[j - base]; }
  __device__ int64_t next_end(int64_t from) const {
    const int64_t t = from - base;
    int64_t w = t >> 6;
    const int64_t wl = (hi - base) >> 6;
    uint64_t m = b[w] & (~0ull << (t & 63));
    while (!m) {
      if (++w > wl) return hi;
      m = b[w];
    }
    return base + (w << 6) + ctz64(m);
  }
};

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
struct NewLds {
  const uint64_t *fp;
  const uint32_t *cnt;
  __device__ uint64_t f(uint64_t i) const { return fp[i]; }
  __device__ uint64_t c(uint64_t i) const { return cnt[i]; }
};
struct NewGlb {
  const uint64_t *fp, *cnt;
  __device__ uint64_t f(uint64_t i) const { return fp[i]; }
  __device__ uint64_t c(uint64_t i) const { return cnt[i]; }
};

// ---- writers of the new table -------------------------------------------
// emit(j, v) writes slot j (positions strictly increasing per lane), set_end()
// marks the last written slot as a run end, flush() ends the lane's output.
// Run-end bits are gathered per 64-bit word; words shared with a neighbour's
// extent are merged with and/or under the lane's mask.
template <typename T>
struct OutLds {
  T *s;
  uint64_t *b;
  int64_t base, hi;  // base is a multiple of 64; positions [.., hi]
  int64_t cw;
  uint64_t acc, accm;
  __device__ void init(T *s_, uint64_t *b_, int64_t base_, int64_t hi_) {
    s = s_; b = b_; base = base_; hi = hi_; cw = -1; acc = 0; accm = 0;
  }
  __device__ void flush() {
    if (accm == ~0ull) {
      b[cw] = acc;
    } else if (accm) {
      atomicAnd(reinterpret_cast<ull *>(&b[cw]), static_cast<ull>(~accm));
      atomicOr(reinterpret_cast<ull *>(&b[cw]), static_cast<ull>(acc));
    }
    acc = accm = 0;
  }
  __device__ void emit(int64_t j, uint64_t v) {
    if (j > hi) return;
    const int64_t t = j - base;
    s[t] = static_cast<T>(v);
    const int64_t w = t >> 6;
    if (w != cw) {
      if (cw >= 0) flush();
      cw = w;
    }
    accm |= 1ull << (t & 63);
  }
  __device__ void set_end(int64_t j) {
    if (j > hi) return;
    acc |= 1ull << ((j - base) & 63);
  }
  // account for slot j without storing it (its value is written later)
  __device__ void mark(int64_t j) {
    if (j > hi) return;
    const int64_t t = j - base;
    const int64_t w = t >> 6;
    if (w != cw) {
      if (cw >= 0) flush();
      cw = w;
    }
    accm |= 1ull << (t & 63);
  }
};

// slot values only (run-end bits of these slots are set by the owning lane)
template <typename T>
struct SlotsLds {
  T *s;
  int64_t base, hi;
  __device__ void emit(int64_t j, uint64_t v) {
    if (j <= hi) s[j - base] = static_cast<T>(v);
  }
  __device__ void set_end(int64_t) {}
  __device__ void flush() {}
};

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
__device__ int64_t carry_old(const Block<T> *b, const uint32_t *off, int64_t i, int64_t N) {
  const int64_t bi = i >> 6;
  const int64_t O = off[bi];
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
                                     uint32_t *noff) {
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

// The per-lane walk of the staged path.  Runs that receive no new entry keep
// their old length (read off the run-end bits); the lengths of the lane's
// changed runs [c0, c1) were computed beforehand, one run per lane.  Pass 1
// (EMIT = false) composes the lane's run maps; pass 2 copies unchanged runs to
// their new place, reserves the changed runs' slots (cstart), zero-fills gaps
// and writes run-end and occupied bits and the offsets of the blocks that
// start in the lane's chunk.
template <typename T, bool EMIT>
__device__ __forceinline__ void walk_fast(int64_t RS, const uint64_t *occ_l, int64_t x0, int64_t x1,
                                          int64_t s0, int64_t s1, int64_t ope, const OldLds<T> &old,
                                          uint32_t c0, uint32_t c1, const uint16_t *cxr,
                                          const uint32_t *cL, uint16_t *cstart, OutLds<T> &out,
                                          int64_t carry, Fn &F, uint64_t &used, uint64_t *nocc_l,
                                          uint32_t *noff) {
  int64_t wpos = max(carry + 1, s0);
  int64_t next_bs = (s0 + 63) & ~static_cast<int64_t>(63);
  // the chunk's occupied bits (a chunk never crosses a 64-bit word) and the
  // run-end word being consumed stay in registers
  uint64_t occ = 0;
  if (x0 < x1) {
    const int64_t t0 = x0 - RS;
    occ = occ_l[t0 >> 6] >> (t0 & 63);
    if (x1 - x0 < 64) occ &= (1ull << (x1 - x0)) - 1ull;
  }
  uint64_t nocc = 0;  // new occupied bits of the chunk
  int64_t rw = -1;    // index of the run-end word held in rv
  uint64_t rv = 0;
  const int64_t rwl = (old.hi - old.base) >> 6;
  auto next_end = [&](int64_t from) -> int64_t {
    int64_t w = (from - old.base) >> 6;
    if (w != rw) {
      rw = w;
      rv = old.b[w];
    }
    uint64_t m = rv & (~0ull << ((from - old.base) & 63));
    while (!m) {
      if (++rw > rwl) return old.hi;
      rv = old.b[rw];
      m = rv;
    }
    return old.base + (rw << 6) + ctz64(m);
  };
  int64_t xo = occ ? x0 + ctz64(occ) : INF;
  uint32_t c = c0;
  int64_t xc = c < c1 ? RS + cxr[c] : INF;
  for (;;) {
    const int64_t x = min(xo, xc);
    if (x >= INF) break;
    if (EMIT) {
      for (; next_bs < x; next_bs += 64)
        noff[next_bs >> 6] = static_cast<uint32_t>(max(carry - next_bs, static_cast<int64_t>(0)));
    }
    int64_t op = 0, oe = -1;
    if (xo == x) {
      op = max(x, ope + 1);
      oe = next_end(op);
      ope = oe;
      occ &= occ - 1;
      xo = occ ? x0 + ctz64(occ) : INF;
    }
    const bool changed = xc == x;
    const int64_t L = changed ? static_cast<int64_t>(cL[c]) : oe - op + 1;
    if (EMIT) {
      const int64_t start = max(x, carry + 1);
      for (; wpos < start; ++wpos) out.emit(wpos, 0);
      if (L > 0) {
        if (changed) {
          cstart[c] = static_cast<uint16_t>(start - out.base);
          for (int64_t j = start; j < start + L; ++j) out.mark(j);
        } else {
          int64_t pos = start;
          for (int64_t j = op; j <= oe; ++j) out.emit(pos++, old.slot(j));
        }
        out.set_end(start + L - 1);
        carry = start + L - 1;
        wpos = start + L;
        nocc |= 1ull << (x - x0);
      }
      if (x == next_bs) {
        noff[x >> 6] = static_cast<uint32_t>(max(carry - x, static_cast<int64_t>(0)));
        next_bs += 64;
      }
    } else if (L > 0) {
      F = fn_then(F, Fn{x + L - 1, L});
      used += static_cast<uint64_t>(L);
    }
    if (changed) {
      ++c;
      xc = c < c1 ? RS + cxr[c] : INF;
    }
  }
  if (EMIT) {
    for (; next_bs < s1; next_bs += 64)
      noff[next_bs >> 6] = static_cast<uint32_t>(max(carry - next_bs, static_cast<int64_t>(0)));
    const int64_t ext_end = max(carry, s1 - 1);
    for (; wpos <= ext_end; ++wpos) out.emit(wpos, 0);
    out.flush();
    if (nocc) {
      const int64_t t0 = x0 - RS;
      atomicOr(reinterpret_cast<ull *>(&nocc_l[t0 >> 6]), static_cast<ull>(nocc << (t0 & 63)));
    }
  }
}

// the rare whole-region path: one lane, global memory in and out (inlined: an
// out-of-line call would cost the whole kernel a call frame and registers)
template <typename T, bool EMIT>
__device__ __forceinline__ void walk_global(const Block<T> *ob, Block<T> *nbk, int64_t nblocks,
                                         const uint64_t *ufp, const uint64_t *ucnt, uint32_t r,
                                         int del, int64_t RS, const uint64_t *occ_l, int64_t x0,
                                         int64_t x1, int64_t s0, int64_t s1, int64_t ope,
                                         uint64_t ni, uint64_t nb, int64_t hi, int64_t carry,
                                         Acc *acc, uint64_t *nocc_l, uint32_t *noff) {
  OldGlb<T> old{ob, nblocks};
  NewGlb nw{ufp, ucnt};
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
__device__ Fn block_exscan_fn(Fn v, Fn *sh, Fn *total) {
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

__device__ uint32_t block_exscan_u32(uint32_t v, uint32_t *sh, uint32_t *total) {
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

__device__ uint64_t block_sum_u64(uint64_t v, uint64_t *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t t = 0;
  for (int w = 0; w < NT / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// Carry-in of region R (called by the 64 lanes of one wave): lane l looks at
// region hi - l; the nearest region with a known inclusive carry ends the walk,
// the aggregates of the regions in between are composed in order.  One memory
// round trip covers 64 predecessors.
__device__ int64_t look_back_wave(const uint64_t *tags, uint32_t nreg, uint32_t epoch, int64_t R) {
  const int lane = threadIdx.x & 63;
  Fn acc = fn_id();  // regions (hi, R-1], applied in order
  int64_t hi = R - 1;
  for (;;) {
    const int64_t j = hi - lane;
    int kind = 0;  // 0 not ready, 1 aggregate, 2 inclusive, 3 before region 0
    int64_t v = -1, A = -1, B = 0;
    if (j < 0) {
      kind = 3;
    } else {
      int64_t tv = 0, tA = 0, tB = 0;
      const bool hv = tag_load(&tags[2ull * nreg + j], epoch, &tv);
      const bool hA = tag_load(&tags[j], epoch, &tA);
      const bool hB = tag_load(&tags[static_cast<uint64_t>(nreg) + j], epoch, &tB);
      if (hv) {
        kind = 2;
        v = tv;
      } else if (hA && hB) {
        kind = 1;
        A = tA;
        B = tB;
      }
    }
    const uint64_t stop_m = __ballot(kind >= 2);
    const uint64_t miss_m = __ballot(kind == 0);
    const int stop = stop_m ? ctz64(stop_m) : 64;
    const int miss = miss_m ? ctz64(miss_m) : 64;
    const int take = min(stop, miss);  // lanes [0, take) hold usable aggregates
    for (int l = 0; l < take; ++l) {
      Fn g;
      g.A = __shfl(A, l);
      g.B = __shfl(B, l);
      acc = fn_then(g, acc);  // region hi - l is applied before the ones already in acc
    }
    if (stop < 64 && stop <= miss) {
      const int64_t c = __shfl(v, stop);
      return fn_apply(acc, c);
    }
    hi -= take;
    if (take == 0) __builtin_amdgcn_s_sleep(2);
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_merge(MergeArgs<T> a) {
  using C = Cfg<T>;
  __shared__ __align__(16) T old_s[C::CAP];
  __shared__ __align__(16) T new_s[C::CAP];
  __shared__ uint64_t old_b[C::CAPW];
  __shared__ uint32_t old_wp[C::CAPW + 1];
  __shared__ uint64_t new_b[C::CAPW];
  __shared__ uint64_t occ_l[C::OW];
  __shared__ uint32_t occ_wp[C::OW + 1];
  __shared__ uint64_t nocc_l[C::OW];
  // the region's new entries, and its changed runs (one per distinct quotient)
  __shared__ uint64_t nfp_l[C::NCAP];
  __shared__ uint32_t ncnt_l[C::NCAP];
  __shared__ uint16_t chg_of[C::NCAP];  // changed run of each entry
  __shared__ uint16_t cxr[C::NCAP];     // its quotient - RS
  __shared__ uint16_t chead[C::NCAP];   // its first entry
  __shared__ uint16_t cop[C::NCAP];     // its old run, relative to the staged base
  __shared__ uint16_t coe[C::NCAP];
  __shared__ uint32_t cL[C::NCAP];      // its new length
  __shared__ uint16_t cstart[C::NCAP];  // its new first slot, relative to the output base
  __shared__ uint32_t lane_start[NT + 1];
  __shared__ int64_t sh_i[8];
  __shared__ Fn sh_fn[NT / 64];
  __shared__ uint32_t sh_u[NT / 64];
  __shared__ uint64_t sh_r[NT / 64];

  const int tid = threadIdx.x;
  if (tid == 0) sh_i[0] = static_cast<int64_t>(atomic_add_u64(&a.state[ST_TILE], 1));
  __syncthreads();
  const int64_t R = sh_i[0];
  const int64_t S = 1ll << a.rlog;
  const int64_t RS = R << a.rlog;
  // (selects, not a dynamic index into the argument struct, which would put
  // the struct in scratch memory)
  const int cur = static_cast<int>(a.state[ST_CUR] & 1ull);
  const Block<T> *ob = cur ? a.blk[1] : a.blk[0];
  Block<T> *nbk = cur ? a.blk[0] : a.blk[1];
  const uint32_t *ooff = cur ? a.off[1] : a.off[0];
  uint32_t *noff = cur ? a.off[0] : a.off[1];
  const bool qreg = RS < a.N;
  const int64_t send = min(RS + S, a.P);
  const int nw_reg = static_cast<int>((send - RS + 63) >> 6);
  const uint64_t rb0 = a.rb[R], rb1 = a.rb[R + 1];
  const uint64_t ne = rb1 - rb0;

  for (int w = tid; w < nw_reg; w += NT) {
    occ_l[w] = qreg ? ob[(RS >> 6) + w].occ : 0ull;
    nocc_l[w] = 0ull;
  }
  if (qreg) {
    if (tid == 0) sh_i[1] = carry_old(ob, ooff, RS, a.N);
    if (tid == 64) sh_i[2] = carry_old(ob, ooff, RS + S, a.N);
  }
  const bool new_lds = ne <= static_cast<uint64_t>(C::NCAP);
  if (new_lds) {
    for (uint64_t i = tid; i < ne; i += NT) {
      nfp_l[i] = a.ufp[rb0 + i];
      ncnt_l[i] = static_cast<uint32_t>(a.ucnt[rb0 + i]);
    }
  }
  __syncthreads();
  const int64_t lo_old = qreg ? sh_i[1] + 1 : RS;
  const int64_t hi_old = qreg ? sh_i[2] : RS - 1;
  const bool has_old = hi_old >= lo_old;
  const int64_t bb = has_old ? (lo_old >> 6) : (RS >> 6);
  const int nblk = has_old ? static_cast<int>((hi_old >> 6) - bb + 1) : 0;
  const bool par = new_lds && nblk <= C::CAPW;
  const int64_t obase = bb << 6;

  if (par && nblk > 0) {
    // 16-byte chunks of the staged blocks' slots, then their run-end words
    for (int idx = tid; idx < nblk * C::CH; idx += NT) {
      const int b = idx / C::CH, c = idx % C::CH;
      const uint4 v = reinterpret_cast<const uint4 *>(ob[bb + b].s)[c];
      reinterpret_cast<uint4 *>(old_s + b * 64)[c] = v;
    }
    for (int w = tid; w < nblk; w += NT) {
      uint64_t v = ob[bb + w].rend;
      if (w == 0) v &= ~0ull << (lo_old & 63);
      if (w == nblk - 1) v &= ~0ull >> (63 - (hi_old & 63));
      old_b[w] = v;
    }
  }
  // lane ranges of the new entries; changed runs = groups of equal quotient
  const int64_t QT = max(S >> 8, static_cast<int64_t>(1));
  const int qshift = __builtin_ctzll(static_cast<uint64_t>(QT));
  if (par) {
    lane_start[tid] = static_cast<uint32_t>(ne);
    if (tid == 0) lane_start[NT] = static_cast<uint32_t>(ne);
  }
  __syncthreads();
  uint32_t nchg = 0;
  if (par) {
    for (uint64_t e = tid; e < ne; e += NT) {
      const int le = static_cast<int>((static_cast<int64_t>(nfp_l[e] >> a.r) - RS) >> qshift);
      const int lp = e == 0 ? -1 : static_cast<int>((static_cast<int64_t>(nfp_l[e - 1] >> a.r) - RS) >> qshift);
      for (int l = lp + 1; l <= le; ++l) lane_start[l] = static_cast<uint32_t>(e);
    }
  }
  {
    // heads of quotient groups: entries [2 tid, 2 tid + 2) per lane (ne <= 512
    // here; more entries take the global path)
    uint32_t h0 = 0, h1 = 0;
    const uint64_t e0 = 2ull * tid, e1 = e0 + 1;
    if (par && e0 < ne) h0 = e0 == 0 || (nfp_l[e0] >> a.r) != (nfp_l[e0 - 1] >> a.r);
    if (par && e1 < ne) h1 = (nfp_l[e1] >> a.r) != (nfp_l[e0] >> a.r);
    uint32_t tot;
    const uint32_t ex = block_exscan_u32(h0 + h1, sh_u, &tot);
    nchg = tot;
    if (par && e0 < ne) {
      chg_of[e0] = static_cast<uint16_t>(ex + h0 - 1);
      if (h0) {
        cxr[ex] = static_cast<uint16_t>((nfp_l[e0] >> a.r) - RS);
        chead[ex] = static_cast<uint16_t>(e0);
      }
    }
    if (par && e1 < ne) {
      chg_of[e1] = static_cast<uint16_t>(ex + h0 + h1 - 1);
      if (h1) {
        cxr[ex + h0] = static_cast<uint16_t>((nfp_l[e1] >> a.r) - RS);
        chead[ex + h0] = static_cast<uint16_t>(e1);
      }
    }
  }
  // prefix counts of run ends per staged word and of occupied quotients per
  // region word (for rank / select)
  {
    uint32_t tot;
    const uint32_t pc = (par && tid < nblk) ? static_cast<uint32_t>(popc64(old_b[tid])) : 0u;
    const uint32_t ex = block_exscan_u32(pc, sh_u, &tot);
    if (par && tid < nblk) old_wp[tid] = ex;
    if (par && tid == 0) old_wp[nblk] = tot;
    const uint32_t po = (par && tid < nw_reg) ? static_cast<uint32_t>(popc64(occ_l[tid])) : 0u;
    const uint32_t exo = block_exscan_u32(po, sh_u, &tot);
    if (par && tid < nw_reg) occ_wp[tid] = exo;
    if (par && tid == 0) occ_wp[nw_reg] = tot;
  }

  // lane chunk: quotients / slots [s0, s1)
  int64_t s0, s1;
  if (par) {
    s0 = min(RS + tid * QT, send);
    s1 = min(s0 + QT, send);
  } else {
    s0 = tid == 0 ? RS : send;
    s1 = send;
  }
  const int64_t x0 = qreg ? s0 : 0, x1 = qreg ? s1 : 0;
  // end of the last old run before the lane's chunk
  int64_t ope = lo_old - 1;
  uint32_t c0 = 0, c1 = 0;
  auto select_end = [&](uint32_t k) -> int64_t {  // position of the k-th (0-based) staged run end
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (old_wp[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return obase + (static_cast<int64_t>(lo) << 6) + select64(old_b[lo], static_cast<int>(k - old_wp[lo]));
  };
  if (par && qreg && x0 < x1) {
    const int64_t t0 = x0 - RS;
    const uint32_t k = occ_wp[t0 >> 6] + static_cast<uint32_t>(popc64(occ_l[t0 >> 6] & ((1ull << (t0 & 63)) - 1ull)));
    if (k > 0) ope = select_end(k - 1);
    const uint32_t ea = lane_start[tid], eb = lane_start[tid + 1];
    c0 = ea < ne ? chg_of[ea] : nchg;
    c1 = eb < ne ? chg_of[eb] : nchg;
  }
  __syncthreads();

  Acc acc{fn_id(), 0, 0, 0, 0, 0};
  if (par) {
    // ---- pass 1a: new lengths of the changed runs, one run per lane --------
    OldLds<T> old{old_s, old_b, obase, hi_old};
    NewLds nw{nfp_l, ncnt_l};
    NoOut none;
    for (uint32_t c = tid; c < nchg; c += NT) {
      const int64_t x = RS + cxr[c];
      const uint64_t ni = chead[c], nj = c + 1 < nchg ? chead[c + 1] : ne;
      const int64_t t = x - RS;
      int64_t op = 0, oe = -1;
      if ((occ_l[t >> 6] >> (t & 63)) & 1ull) {
        const uint32_t k = occ_wp[t >> 6] + static_cast<uint32_t>(popc64(occ_l[t >> 6] & ((1ull << (t & 63)) - 1ull)));
        oe = select_end(k);
        op = max(x, (k > 0 ? select_end(k - 1) : lo_old - 1) + 1);
      }
      // staged positions are < CAP, so 0xFFFF marks "no old run"
      cop[c] = oe >= op ? static_cast<uint16_t>(op - obase) : 0;
      coe[c] = oe >= op ? static_cast<uint16_t>(oe - obase) : 0xFFFF;
      cL[c] = static_cast<uint32_t>(merge_run<false>(old, op, oe, nw, ni, nj, a.r, a.del, none, int64_t{0}, acc));
    }
    __syncthreads();
    // ---- pass 1b: the lane's run maps -------------------------------------
    OutLds<T> dummy_out;
    dummy_out.init(new_s, new_b, 0, -1);
    walk_fast<T, false>(RS, occ_l, x0, x1, s0, s1, ope, old, c0, c1, cxr, cL, cstart, dummy_out, 0,
                        acc.F, acc.used, nocc_l, noff);
  } else if (tid == 0) {
    Acc ag{fn_id(), 0, 0, 0, 0, 0};
    walk_global<T, false>(ob, nbk, a.nblocks, a.ufp, a.ucnt, a.r, a.del, RS, occ_l, x0, x1, s0, s1, ope,
                          rb0, rb1, 0, 0, &ag, nocc_l, noff);
    acc = ag;
  }
  Fn Ftot;
  const Fn Fex = block_exscan_fn(acc.F, sh_fn, &Ftot);
  const uint64_t used = block_sum_u64(acc.used, sh_r);
  const uint64_t dent = block_sum_u64(acc.dent, sh_r);
  const uint64_t dtot = block_sum_u64(acc.dtot, sh_r);
  const uint64_t shortfall = block_sum_u64(acc.shortfall, sh_r);
  const uint64_t ovf = block_sum_u64(acc.ovf, sh_r);

  if (tid == 0) {
    tag_store(&a.tags[R], a.epoch, Ftot.A);
    tag_store(&a.tags[static_cast<uint64_t>(a.nregions) + R], a.epoch, Ftot.B);
  }
  if (tid < 64) {
    const int64_t c_in = look_back_wave(a.tags, a.nregions, a.epoch, R);
    if (tid == 0) {
      const int64_t c_out = fn_apply(Ftot, c_in);
      tag_store(&a.tags[2ull * a.nregions + R], a.epoch, c_out);
      sh_i[3] = c_in;
      sh_i[4] = c_out;
      if (c_out >= a.P) atomic_or_u64(&a.state[ST_BATCH], BATCH_FULL);
      if (ovf) atomic_or_u64(&a.state[ST_BATCH], BATCH_OVF);
      if (used) atomic_add_u64(&a.state[ST_NUSED], used);
      if (dent) atomic_add_u64(&a.state[ST_NDIST], dent);
      if (dtot) atomic_add_u64(&a.state[ST_NTOTAL], dtot);
      if (a.del && shortfall) atomic_add_u64(a.not_found, shortfall);
    }
  }
  __syncthreads();

  // ---- pass 2: write the region's extent into the other copy --------------
  const int64_t c_in = sh_i[3], c_out = sh_i[4];
  const int64_t ext_lo = max(c_in + 1, RS);
  const int64_t ext_hi = min(max(c_out, send - 1), a.P - 1);
  const int64_t xbase = (ext_lo >> 6) << 6;
  const int nxb = ext_hi >= ext_lo ? static_cast<int>((ext_hi >> 6) - (ext_lo >> 6) + 1) : 0;
  const bool lds_out = par && nxb <= C::CAPW;
  const int64_t c_t = fn_apply(Fex, c_in);
  if (lds_out) {
    // 2a: unchanged runs, gaps, bits, offsets; reserve the changed runs
    OldLds<T> old{old_s, old_b, obase, hi_old};
    OutLds<T> out;
    out.init(new_s, new_b, xbase, ext_hi);
    Fn Fd = fn_id();
    uint64_t ud = 0;
    walk_fast<T, true>(RS, occ_l, x0, x1, s0, s1, ope, old, c0, c1, cxr, cL, cstart, out, c_t, Fd, ud,
                       nocc_l, noff);
    __syncthreads();
    // 2b: the changed runs' slots, one run per lane
    NewLds nw{nfp_l, ncnt_l};
    SlotsLds<T> so{new_s, xbase, ext_hi};
    Acc dummy{fn_id(), 0, 0, 0, 0, 0};
    for (uint32_t c = tid; c < nchg; c += NT) {
      if (cL[c] == 0) continue;
      const uint64_t ni = chead[c], nj = c + 1 < nchg ? chead[c + 1] : ne;
      const int64_t op = coe[c] == 0xFFFF ? 0 : obase + cop[c];
      const int64_t oe = coe[c] == 0xFFFF ? -1 : obase + coe[c];
      merge_run<true>(old, op, oe, nw, ni, nj, a.r, a.del, so, static_cast<int64_t>(xbase + cstart[c]), dummy);
    }
  } else if (tid == 0) {
    // one lane redoes the whole region from global memory
    Acc dummy{fn_id(), 0, 0, 0, 0, 0};
    walk_global<T, true>(ob, nbk, a.nblocks, a.ufp, a.ucnt, a.r, a.del, RS, occ_l, qreg ? RS : 0,
                         qreg ? send : 0, RS, send, lo_old - 1, rb0, rb1, ext_hi, c_in, &dummy, nocc_l,
                         noff);
  }
  __syncthreads();

  if (lds_out && nxb > 0) {
    // slots: whole 16-byte chunks inside the extent, single slots at its ends
    for (int idx = tid; idx < nxb * C::CH; idx += NT) {
      const int b = idx / C::CH, c = idx % C::CH;
      const int64_t p0 = xbase + b * 64 + c * C::PER;
      const int64_t p1 = p0 + C::PER - 1;
      T *dst = nbk[(xbase >> 6) + b].s + c * C::PER;
      const T *src = new_s + b * 64 + c * C::PER;
      if (p0 >= ext_lo && p1 <= ext_hi) {
        *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
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
        nbk[w].rend = v;
      } else {
        atomic_and_u64(&nbk[w].rend, ~mask);
        atomic_or_u64(&nbk[w].rend, v);
      }
    }
  }
  for (int w = tid; w < nw_reg; w += NT) nbk[(RS >> 6) + w].occ = nocc_l[w];

  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const uint64_t d = atomic_add_u64(&a.state[ST_DONE], 1);
    if (d + 1 == a.nregions) {
      __threadfence();
      const uint64_t st = __hip_atomic_load(&a.state[ST_BATCH], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (st == 0) {
        a.state[ST_USED] = __hip_atomic_load(&a.state[ST_NUSED], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.state[ST_DIST] += __hip_atomic_load(&a.state[ST_NDIST], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.state[ST_TOTAL] += __hip_atomic_load(&a.state[ST_NTOTAL], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.state[ST_CUR] = static_cast<uint64_t>(cur ^ 1);
      } else {
        const int64_t code = (st & BATCH_FULL) ? -2 : -5;
        atomicCAS(reinterpret_cast<ull *>(&a.state[ST_ERR]), 0ull, static_cast<ull>(code));
      }
      a.state[ST_BATCHES] += 1;
    }
  }
}

template <typename T>
hipError_t launch_merge_t(qf_filter *f, const uint64_t *ufp, const uint64_t *ucnt, int del,
                          uint64_t *not_found, hipStream_t s) {
  MergeArgs<T> a;
  a.blk[0] = static_cast<Block<T> *>(f->blk[0]);
  a.blk[1] = static_cast<Block<T> *>(f->blk[1]);
  a.off[0] = f->off[0];
  a.off[1] = f->off[1];
  a.N = static_cast<int64_t>(f->N);
  a.P = static_cast<int64_t>(f->P);
  a.nblocks = static_cast<int64_t>(f->nblocks);
  a.r = f->r;
  a.rlog = f->rlog;
  a.nregions = f->nregions;
  a.ufp = ufp;
  a.ucnt = ucnt;
  a.rb = f->rb;
  a.tags = f->tags;
  a.epoch = f->epoch;
  a.state = f->state;
  a.del = del;
  a.not_found = not_found ? not_found : f->state + ST_SCRATCH;
  if (f->timer) f->timer->begin(QF_PROF_MERGE, s);
  k_merge<T><<<f->nregions, NT, 0, s>>>(a);
  if (f->timer) f->timer->end(QF_PROF_MERGE, s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_merge(qf_filter *f, const uint64_t *ufp, const uint64_t *ucnt, int del,
                        uint64_t *not_found, hipStream_t s) {
  if (f->r == 8) return launch_merge_t<uint8_t>(f, ufp, ucnt, del, not_found, s);
  return launch_merge_t<uint16_t>(f, ufp, ucnt, del, not_found, s);
}

int max_region_log2(uint32_t r) { return r == 8 ? Cfg<uint8_t>::SMAXLOG : Cfg<uint16_t>::SMAXLOG; }

}  // namespace qf
