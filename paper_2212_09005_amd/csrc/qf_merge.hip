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
//     composition of its runs, a decoupled look-back gives every region the
//     exact end of all earlier runs (its carry-in), and no spill limit exists.
//   * The table has two device copies; a batch reads the current one and
//     writes the other, so no region reads what another region writes.  The
//     last region to finish flips the current copy -- unless a run ran past
//     the last slot or a count overflowed, which leaves the old copy current
//     (all-or-nothing without a host round trip).
//   * Inside a region, the old runs are staged in LDS; each of the 256 lanes
//     merges a contiguous chunk of quotients; lane carries are a block scan of
//     the same max-plus maps; the new runs are assembled in LDS and written out
//     with coalesced stores.  Regions whose runs do not fit in LDS fall back
//     to one lane reading and writing global memory directly.
#include "qf_dev.h"
#include "qf.h"
#include "qf_lib.h"

namespace qf {
namespace {

constexpr int NT = 256;
constexpr int64_t INF = INT64_MAX / 4;

template <typename T>
struct Cfg {
  static constexpr int CAP = 16384 / static_cast<int>(sizeof(T));  // LDS slots per buffer
  static constexpr int CAPW = CAP / 64;
  static constexpr int SMAX = CAP / 2;  // largest region
  static constexpr int OW = SMAX / 64;
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
struct OldLds {  // slots [base, base + len) staged in LDS; bits relative to base
  const T *s;
  const uint64_t *b;
  int64_t base, len;
  __device__ uint64_t slot(int64_t j) const { return s[j - base]; }
  __device__ int64_t next_end(int64_t from) const {
    int64_t t = from - base;
    if (t >= len) return base + len - 1;
    int w = static_cast<int>(t >> 6);
    const int nw = static_cast<int>((len + 63) >> 6);
    uint64_t m = b[w] & (~0ull << (t & 63));
    while (!m) {
      if (++w >= nw) return base + len - 1;
      m = b[w];
    }
    return base + (static_cast<int64_t>(w) << 6) + ctz64(m);
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

// ---- writers of the new table -------------------------------------------
// emit(j, v) writes slot j (positions strictly increasing per lane), set_end()
// marks the last written slot as a run end, flush() ends the lane's output.
// Run-end bits are gathered per 64-bit word; words shared with a neighbour's
// extent are merged with and/or under the lane's mask.
template <typename T>
struct OutLds {
  T *s;
  uint64_t *b;
  int64_t base, hi;  // positions [base, hi]
  int64_t cw;
  uint64_t acc, accm;
  __device__ void init(T *s_, uint64_t *b_, int64_t base_, int64_t hi_) {
    s = s_; b = b_; base = base_; hi = hi_; cw = -1; acc = 0; accm = 0;
  }
  __device__ void flush() {
    if (accm) {
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
      flush();
      cw = w;
    }
    accm |= 1ull << (t & 63);
  }
  __device__ void set_end(int64_t j) {
    if (j > hi) return;
    acc |= 1ull << ((j - base) & 63);
  }
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
      flush();
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
  uint64_t entries, total, shortfall, used;
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

// Walk one lane's chunk: quotients [x0, x1) (the same numbers as its slots
// [s0, s1) in a quotient region; empty in the extra slots).  Pass 1 (EMIT =
// false) composes the lane's run maps and counts; pass 2 writes the lane's
// extent [max(carry + 1, s0), max(last end, s1 - 1)] -- runs and zero gaps --
// plus the occupied bits and the offsets of the blocks that start in it.
template <typename T, bool EMIT, class Old, class Out>
__device__ void walk(const MergeArgs<T> &a, int64_t RS, const uint64_t *occ_l, int64_t x0,
                     int64_t x1, int64_t s0, int64_t s1, int64_t ope, uint64_t ni, uint64_t nb,
                     const Old &old, Out &out, int64_t carry, Acc &acc, uint64_t *nocc_l,
                     uint32_t *noff) {
  const uint32_t r = a.r;
  const uint64_t rmask = (1ull << r) - 1ull;
  int64_t wpos = max(carry + 1, s0);
  int64_t next_bs = (s0 + 63) & ~static_cast<int64_t>(63);
  int64_t xo = x0 < x1 ? next_occ(occ_l, RS, x0, x1) : INF;
  for (;;) {
    const int64_t xn = ni < nb ? static_cast<int64_t>(a.ufp[ni] >> r) : INF;
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
    while (nj < nb && static_cast<int64_t>(a.ufp[nj] >> r) == x) ++nj;

    int64_t start = 0, pos = 0;
    if (EMIT) {
      start = max(x, carry + 1);
      for (; wpos < start; ++wpos) out.emit(wpos, 0);
      pos = start;
    }
    int64_t L = 0;
    uint64_t orem = 0, ocnt = 0;
    bool ohave = false;
    if (op <= oe) {
      op = dec_entry(old, op, oe, r, orem, ocnt);
      ohave = true;
    }
    uint64_t k = ni;
    while (ohave || k < nj) {
      const uint64_t nrem = k < nj ? (a.ufp[k] & rmask) : ~0ull;
      uint64_t rem, c;
      if (ohave && (k >= nj || orem < nrem)) {
        rem = orem;
        c = ocnt;
        if (op <= oe) op = dec_entry(old, op, oe, r, orem, ocnt); else ohave = false;
      } else if (!ohave || nrem < orem) {
        rem = nrem;
        const uint64_t cn = a.ucnt[k++];
        if (a.del) {
          if (!EMIT) acc.shortfall += cn;
          c = 0;
        } else {
          c = cn;
        }
      } else {
        rem = orem;
        const uint64_t cn = a.ucnt[k++];
        if (a.del) {
          const uint64_t t = min(ocnt, cn);
          if (!EMIT) acc.shortfall += cn - t;
          c = ocnt - t;
        } else {
          c = ocnt + cn;
          if (c < ocnt) {
            if (!EMIT) acc.ovf = 1;
            c = ~0ull;
          }
        }
        if (op <= oe) op = dec_entry(old, op, oe, r, orem, ocnt); else ohave = false;
      }
      if (c == 0) continue;
      if (EMIT) {
        pos = enc_put(out, pos, rem, c, r);
      } else {
        L += enc_len(rem, c, r);
        acc.entries += 1;
        acc.total += c;
      }
    }
    if (EMIT) {
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
    } else if (L > 0) {
      acc.F = fn_then(acc.F, Fn{x + L - 1, L});
      acc.used += static_cast<uint64_t>(L);
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

__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t *a, uint64_t lo, uint64_t hi,
                                                    uint64_t key) {
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Carry-in of region R: compose the published maps of R-1, R-2, ... until a
// region whose inclusive carry is already known.
__device__ int64_t look_back(const uint64_t *tags, uint32_t nreg, uint32_t epoch, int64_t R) {
  Fn acc = fn_id();
  int64_t j = R - 1;
  while (j >= 0) {
    int64_t v, A, B;
    if (tag_load(&tags[2ull * nreg + j], epoch, &v)) return fn_apply(acc, v);
    if (tag_load(&tags[j], epoch, &A) && tag_load(&tags[static_cast<uint64_t>(nreg) + j], epoch, &B)) {
      acc = fn_then(Fn{A, B}, acc);
      --j;
      continue;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return fn_apply(acc, -1);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_merge(MergeArgs<T> a) {
  using C = Cfg<T>;
  __shared__ T old_s[C::CAP];
  __shared__ uint64_t old_b[C::CAPW];
  __shared__ uint32_t old_wp[C::CAPW + 1];
  __shared__ T new_s[C::CAP];
  __shared__ uint64_t new_b[C::CAPW];
  __shared__ uint64_t occ_l[C::OW];
  __shared__ uint64_t nocc_l[C::OW];
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
  const int cur = static_cast<int>(a.state[ST_CUR] & 1ull);
  const Block<T> *ob = a.blk[cur];
  Block<T> *nbk = a.blk[cur ^ 1];
  const uint32_t *ooff = a.off[cur];
  uint32_t *noff = a.off[cur ^ 1];
  const bool qreg = RS < a.N;
  const int64_t send = min(RS + S, a.P);
  const int nw_reg = static_cast<int>((send - RS + 63) >> 6);

  for (int w = tid; w < nw_reg; w += NT) {
    occ_l[w] = qreg ? ob[(RS >> 6) + w].occ : 0ull;
    nocc_l[w] = 0ull;
  }
  if (qreg) {
    if (tid == 0) sh_i[1] = carry_old(ob, ooff, RS, a.N);
    if (tid == 64) sh_i[2] = carry_old(ob, ooff, RS + S, a.N);
  }
  __syncthreads();
  const int64_t lo_old = qreg ? sh_i[1] + 1 : RS;
  const int64_t hi_old = qreg ? sh_i[2] : RS - 1;
  const int64_t len_old = max(hi_old - lo_old + 1, static_cast<int64_t>(0));
  const bool par = len_old <= C::CAP;
  const int nwo = static_cast<int>((len_old + 63) >> 6);

  if (par) {
    for (int64_t t = tid; t < len_old; t += NT) {
      const int64_t j = lo_old + t;
      old_s[t] = ob[j >> 6].s[j & 63];
    }
    for (int w = tid; w < nwo; w += NT) {
      const int64_t p = lo_old + 64ll * w;
      const int64_t gw = p >> 6;
      const int shf = static_cast<int>(p & 63);
      uint64_t v = ob[gw].rend >> shf;
      if (shf && gw + 1 < a.nblocks) v |= ob[gw + 1].rend << (64 - shf);
      const int64_t left = len_old - 64ll * w;
      if (left < 64) v &= (1ull << left) - 1ull;
      old_b[w] = v;
    }
  }
  __syncthreads();
  // prefix of run-end counts per staged word (for the lanes' select)
  {
    uint32_t tot;
    const uint32_t pc = (par && tid < nwo) ? static_cast<uint32_t>(popc64(old_b[tid])) : 0u;
    const uint32_t ex = block_exscan_u32(pc, sh_u, &tot);
    // only the staged (parallel) path has nwo <= CAPW words to index
    if (par && tid < nwo) old_wp[tid] = ex;
    if (par && tid == 0) old_wp[nwo] = tot;
  }

  // lane chunk: quotients / slots [cs0, cs1)
  const int64_t QT = max(S >> 8, static_cast<int64_t>(1));
  int64_t s0, s1;
  if (par) {
    s0 = min(RS + tid * QT, send);
    s1 = min(s0 + QT, send);
  } else {
    s0 = tid == 0 ? RS : send;
    s1 = send;
  }
  const int64_t x0 = qreg ? s0 : 0, x1 = qreg ? s1 : 0;
  // old runs before the chunk, and the end of the last of them
  uint32_t pc_occ = 0;
  if (qreg && x0 < x1) {
    const int64_t t0 = x0 - RS;
    const int nbits = static_cast<int>(x1 - x0);
    uint64_t m = occ_l[t0 >> 6] >> (t0 & 63);
    if (nbits < 64) m &= (1ull << nbits) - 1ull;
    pc_occ = static_cast<uint32_t>(popc64(m));
  }
  uint32_t occ_tot;
  const uint32_t k_t = block_exscan_u32(par ? pc_occ : 0u, sh_u, &occ_tot);
  int64_t ope = lo_old - 1;
  if (par && k_t > 0 && x0 < x1) {
    int lo = 0, hi = nwo - 1;  // word w with old_wp[w] <= k_t - 1 < old_wp[w + 1]
    const uint32_t k = k_t - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (old_wp[mid] <= k) lo = mid; else hi = mid - 1;
    }
    ope = lo_old + (static_cast<int64_t>(lo) << 6) + select64(old_b[lo], static_cast<int>(k - old_wp[lo]));
  }
  const uint64_t rb0 = a.rb[R], rb1 = a.rb[R + 1];
  uint64_t na = rb0, nb = rb0;
  if (qreg && x0 < x1) {
    na = lower_bound_u64(a.ufp, rb0, rb1, static_cast<uint64_t>(x0) << a.r);
    nb = lower_bound_u64(a.ufp, na, rb1, static_cast<uint64_t>(x1) << a.r);
  }

  // ---- pass 1: lengths -------------------------------------------------
  Acc acc{fn_id(), 0, 0, 0, 0, 0};
  NoOut none;
  if (par) {
    OldLds<T> old{old_s, old_b, lo_old, len_old};
    walk<T, false>(a, RS, occ_l, x0, x1, s0, s1, ope, na, nb, old, none, 0, acc, nocc_l, noff);
  } else if (tid == 0) {
    OldGlb<T> old{ob, a.nblocks};
    walk<T, false>(a, RS, occ_l, x0, x1, s0, s1, ope, na, nb, old, none, 0, acc, nocc_l, noff);
  }
  Fn Ftot;
  const Fn Fex = block_exscan_fn(acc.F, sh_fn, &Ftot);
  const uint64_t entries = block_sum_u64(acc.entries, sh_r);
  const uint64_t total = block_sum_u64(acc.total, sh_r);
  const uint64_t shortfall = block_sum_u64(acc.shortfall, sh_r);
  const uint64_t used = block_sum_u64(acc.used, sh_r);
  const uint64_t ovf = block_sum_u64(acc.ovf, sh_r);

  if (tid == 0) {
    tag_store(&a.tags[R], a.epoch, Ftot.A);
    tag_store(&a.tags[static_cast<uint64_t>(a.nregions) + R], a.epoch, Ftot.B);
    const int64_t c_in = look_back(a.tags, a.nregions, a.epoch, R);
    const int64_t c_out = fn_apply(Ftot, c_in);
    tag_store(&a.tags[2ull * a.nregions + R], a.epoch, c_out);
    sh_i[3] = c_in;
    sh_i[4] = c_out;
    if (c_out >= a.P) atomic_or_u64(&a.state[ST_BATCH], BATCH_FULL);
    if (ovf) atomic_or_u64(&a.state[ST_BATCH], BATCH_OVF);
    if (used) atomic_add_u64(&a.state[ST_NUSED], used);
    if (entries) atomic_add_u64(&a.state[ST_NDIST], entries);
    if (total) atomic_add_u64(&a.state[ST_NTOTAL], total);
    if (a.del && shortfall) atomic_add_u64(a.not_found, shortfall);
  }
  __syncthreads();

  // ---- pass 2: write the region's extent into the other copy ------------
  const int64_t c_in = sh_i[3], c_out = sh_i[4];
  const int64_t ext_lo = max(c_in + 1, RS);
  const int64_t ext_hi = min(max(c_out, send - 1), a.P - 1);
  const int64_t ext_len = max(ext_hi - ext_lo + 1, static_cast<int64_t>(0));
  const bool lds_out = ext_len <= C::CAP;
  const int64_t c_t = fn_apply(Fex, c_in);
  Acc dummy{fn_id(), 0, 0, 0, 0, 0};
  if (par || tid == 0) {
    if (lds_out) {
      OutLds<T> out;
      out.init(new_s, new_b, ext_lo, ext_hi);
      if (par) {
        OldLds<T> old{old_s, old_b, lo_old, len_old};
        walk<T, true>(a, RS, occ_l, x0, x1, s0, s1, ope, na, nb, old, out, c_t, dummy, nocc_l, noff);
      } else {
        OldGlb<T> old{ob, a.nblocks};
        walk<T, true>(a, RS, occ_l, x0, x1, s0, s1, ope, na, nb, old, out, c_t, dummy, nocc_l, noff);
      }
    } else {
      OutGlb<T> out;
      out.init(nbk, ext_hi);
      if (par) {
        OldLds<T> old{old_s, old_b, lo_old, len_old};
        walk<T, true>(a, RS, occ_l, x0, x1, s0, s1, ope, na, nb, old, out, c_t, dummy, nocc_l, noff);
      } else {
        OldGlb<T> old{ob, a.nblocks};
        walk<T, true>(a, RS, occ_l, x0, x1, s0, s1, ope, na, nb, old, out, c_t, dummy, nocc_l, noff);
      }
    }
  }
  __syncthreads();

  // copy-out of the LDS extent: slots, then run-end words (masked at the ends)
  if (lds_out && ext_len > 0) {
    for (int64_t t = tid; t < ext_len; t += NT) {
      const int64_t j = ext_lo + t;
      nbk[j >> 6].s[j & 63] = new_s[t];
    }
    const int64_t w0 = ext_lo >> 6, w1 = ext_hi >> 6;
    for (int64_t w = w0 + tid; w <= w1; w += NT) {
      const int64_t plo = max(w << 6, ext_lo), phi = min((w << 6) + 63, ext_hi);
      const int n = static_cast<int>(phi - plo + 1);
      const int64_t t = plo - ext_lo;
      const int shf = static_cast<int>(t & 63);
      uint64_t v = new_b[t >> 6] >> shf;
      if (shf && n > 64 - shf) v |= new_b[(t >> 6) + 1] << (64 - shf);
      const uint64_t lowm = n == 64 ? ~0ull : ((1ull << n) - 1ull);
      v &= lowm;
      const int pos = static_cast<int>(plo & 63);
      const uint64_t mask = lowm << pos;
      v <<= pos;
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
        a.state[ST_DIST] = __hip_atomic_load(&a.state[ST_NDIST], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.state[ST_TOTAL] = __hip_atomic_load(&a.state[ST_NTOTAL], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

int max_region_log2(uint32_t r) { return r == 8 ? 13 : 12; }

}  // namespace qf
