// qf_lookup.hip -- bulk query and count (Sec. 6.2; API table of Sec. 6), and
// the conversions between the physical table and the logical layout.
//
// One lane per key: hash, split the fingerprint, read the home block's
// occupieds word; if the quotient has a run, locate its end with the block
// offset plus rank (popcount of occupieds) and select (walk of the run-end
// words), its start as one past the previous run end (or the quotient itself),
// then decode the run's entries in remainder order until the remainder is
// reached or passed.
#include "qf_dev.h"
#include "qf.h"
#include "qf_lib.h"

namespace qf {
namespace {

constexpr int NT = 256;

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The entries of quotient x's run in remainder order, each offered to
// visit(remainder, count) until it returns true; returns whether x has a run.
// ls: null, or the lane's LDS area of 64 bytes (r = 8 only) that receives the
// home block's slots, requested with its header: the run's slots then come
// from LDS unless the run lies (partly) in a later block.
template <typename T, class V>
__device__ __forceinline__ bool visit_run(const Block<T> *__restrict__ b, int64_t nblocks, int64_t x, uint32_t r,
                                          u32x4 *ls, V &visit) {
  const int64_t bi = x >> 6;
  const int bit = static_cast<int>(x & 63);
  // the home block's occupied word, run-end word and offset, requested
  // together (one line): most runs end and start inside the home block, so
  // the run-end words below usually come from these registers
  const u64x2 h = *reinterpret_cast<const u64x2 *>(&b[bi]);
  const uint32_t off = b[bi].off;
  if (sizeof(T) == 1 && ls) {
    const u32x4 *src = reinterpret_cast<const u32x4 *>(b[bi].s);
    const u32x4 v0 = src[0], v1 = src[1], v2 = src[2], v3 = src[3];
    ls[0] = v0;
    ls[1] = v1;
    ls[2] = v2;
    ls[3] = v3;
  }
  // (an empty asm that takes the offset keeps its load in front of the
  // branch below, in flight with the first one, instead of after it)
  __asm__ volatile("" : : "v"(off));
  const uint64_t occ = h.x, rend0 = h.y;
  if (!((occ >> bit) & 1ull)) return false;
  int d = popc64(occ & ((2ull << bit) - 2ull));  // occupied quotients in (64*bi, x]
  const int64_t p = (bi << 6) + off;
  const auto rend_of = [&](int64_t w) -> uint64_t { return w == bi ? rend0 : b[w].rend; };
  int64_t e;
  if (d == 0) {
    e = p;
  } else {
    // d-th run end strictly after p
    int64_t w = (p + 1) >> 6;
    if (w >= nblocks) return false;
    uint64_t m = rend_of(w) & (~0ull << ((p + 1) & 63));
    for (;;) {
      const int pc = popc64(m);
      if (pc >= d) {
        e = (w << 6) + select64(m, d - 1);
        break;
      }
      d -= pc;
      if (++w >= nblocks) return false;
      m = rend_of(w);
    }
  }
  // run start: one past the last run end in [x, e-1], else x
  int64_t s = x;
  if (e > x) {
    int64_t w = (e - 1) >> 6;
    const int64_t wx = x >> 6;
    uint64_t m = rend_of(w) & (~0ull >> (63 - ((e - 1) & 63)));
    for (;;) {
      if (w == wx) m &= ~0ull << (x & 63);
      if (m) {
        s = (w << 6) + msb64(m) + 1;
        break;
      }
      if (w == wx) break;
      --w;
      m = rend_of(w);
    }
  }
  struct G {
    const Block<T> *b;
    const uint8_t *ls;
    int64_t bi;
    __device__ uint64_t slot(int64_t j) const {
      return (sizeof(T) == 1 && ls && (j >> 6) == bi) ? ls[j & 63] : b[j >> 6].s[j & 63];
    }
  } g{b, reinterpret_cast<const uint8_t *>(ls), bi};
  int64_t pos = s;
  while (pos <= e) {
    uint64_t xr, c;
    pos = dec_entry(g, pos, e, r, xr, c);
    if (visit(xr, c)) break;
  }
  return true;
}

// the count of remainder rem in quotient x's run (0 if none)
template <typename T>
__device__ __forceinline__ uint64_t lookup_one(const Block<T> *__restrict__ b, int64_t nblocks,
                                               int64_t x, uint64_t rem, uint32_t r, u32x4 *ls) {
  uint64_t res = 0;
  auto v = [&](uint64_t xr, uint64_t c) {
    if (xr == rem) res = c;
    return xr >= rem;
  };
  visit_run(b, nblocks, x, r, ls, v);
  return res;
}

// Value association: the remainders of a key's entries are
// (key remainder << vbits) | value, so the values of a key are the entries of
// its run with remainders in [lo, lo + 2^vbits); the smallest and how many
// distinct ones there are.
template <typename T>
__global__ __launch_bounds__(NT) void k_kv_lookup(const Block<T> *b0, const Block<T> *b1, const uint64_t *state,
                                                  const uint64_t *__restrict__ keys, uint64_t n, uint32_t q,
                                                  uint32_t r, uint32_t vbits, int64_t nblocks,
                                                  uint64_t *__restrict__ value, uint32_t *__restrict__ nvalues) {
  const Block<T> *b = (state[ST_CUR] & 1ull) ? b1 : b0;
  const uint32_t rk = r - vbits;  // key remainder bits
  const uint64_t kmask = (1ull << (q + rk)) - 1ull, vmask = (1ull << vbits) - 1ull;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride) {
    const uint64_t fk = mix64(keys[i]) & kmask;
    const uint64_t lo = (fk & ((1ull << rk) - 1ull)) << vbits, hi = lo | vmask;
    uint64_t first = ~0ull;
    uint32_t cnt = 0;
    auto v = [&](uint64_t xr, uint64_t) {
      if (xr > hi) return true;
      if (xr >= lo) {
        if (cnt == 0) first = xr & vmask;
        ++cnt;
      }
      return false;
    };
    visit_run(b, nblocks, static_cast<int64_t>(fk >> rk), r, static_cast<u32x4 *>(nullptr), v);
    value[i] = first;
    if (nvalues) nvalues[i] = cnt;
  }
}

// KPL keys per lane, NT apart (coalesced key loads and result stores; the
// lookups of one lane are independent, so their loads can overlap)
template <typename T, bool COUNT, int KPL>
__global__ __launch_bounds__(NT) void k_lookup(const Block<T> *b0, const Block<T> *b1,
                                               const uint64_t *state,
                                               const uint64_t *__restrict__ keys, uint64_t n,
                                               uint32_t q, uint32_t r, int64_t nblocks,
                                               uint8_t *__restrict__ out8,
                                               uint64_t *__restrict__ out64) {
  // (one key at a time per lane: each lane stages its home block's slots)
  __shared__ u32x4 stage[KPL == 1 && sizeof(T) == 1 ? NT * 4 : 1];
  u32x4 *ls = KPL == 1 && sizeof(T) == 1 ? &stage[threadIdx.x * 4] : nullptr;
  const int cur = static_cast<int>(state[ST_CUR] & 1ull);
  const Block<T> *b = cur ? b1 : b0;
  const uint32_t p = q + r;
  const uint64_t pmask = p >= 64 ? ~0ull : ((1ull << p) - 1ull);
  const uint64_t rmask = (1ull << r) - 1ull;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT * KPL;
  for (uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * NT * KPL + threadIdx.x; i0 < n; i0 += stride) {
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
      const uint64_t i = i0 + static_cast<uint64_t>(k) * NT;
      if (i < n) {
        const uint64_t fp = mix64(keys[i]) & pmask;
        const uint64_t c = lookup_one(b, nblocks, static_cast<int64_t>(fp >> r), fp & rmask, r, ls);
        if (COUNT)
          out64[i] = c;
        else
          out8[i] = c != 0;
      }
    }
  }
}

// Lookups over a filter set: key i is looked up in filter fid[i] (0 for a
// filter index out of range, which also flags the call in pst[ST_ERR]).
template <typename T, bool COUNT, int KPL>
__global__ __launch_bounds__(NT) void k_lookup_multi(const FDesc *__restrict__ desc, uint32_t nf,
                                                     const uint64_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ fid, uint64_t n,
                                                     uint8_t *__restrict__ out8, uint64_t *__restrict__ out64,
                                                     uint64_t *pst) {
  // (no LDS slots here: on a mix of many small filters they made the launch
  // slower, 1.57 against 1.12 ms for 2^24 keys over 4096 filters)
  u32x4 *ls = nullptr;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT * KPL;
  for (uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * NT * KPL + threadIdx.x; i0 < n; i0 += stride) {
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
      const uint64_t i = i0 + static_cast<uint64_t>(k) * NT;
      if (i >= n) break;
      const uint32_t f = fid[i];
      uint64_t c = 0;
      if (f < nf) {
        const FDesc &d = desc[f];
        const bool cur = d.state[ST_CUR] & 1ull;
        const uint32_t p = d.q + d.r;
        const uint64_t fp = mix64(keys[i]) & ((1ull << p) - 1ull);
        c = lookup_one(static_cast<const Block<T> *>(cur ? d.blk[1] : d.blk[0]), d.nblocks,
                       static_cast<int64_t>(fp >> d.r), fp & ((1ull << d.r) - 1ull), d.r, ls);
      } else {
        pst[ST_ERR] = static_cast<uint64_t>(static_cast<int64_t>(QF_ERR_ARG));
      }
      if (COUNT)
        out64[i] = c;
      else
        out8[i] = c != 0;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_export(const Block<T> *b0, const Block<T> *b1,
                                               const uint64_t *state, int64_t nblocks,
                                               int64_t nqblocks, uint64_t *occ, uint64_t *rend,
                                               uint16_t *slots, uint32_t *offs) {
  const int cur = static_cast<int>(state[ST_CUR] & 1ull);
  const Block<T> *b = cur ? b1 : b0;
  const uint64_t total = static_cast<uint64_t>(nblocks) * 64;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; j < total; j += stride) {
    const int64_t bi = static_cast<int64_t>(j >> 6);
    slots[j] = static_cast<uint16_t>(b[bi].s[j & 63]);
    if ((j & 63) == 0) {
      rend[bi] = b[bi].rend;
      offs[bi] = b[bi].off;
      if (bi < nqblocks) occ[bi] = b[bi].occ;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_import(Block<T> *b, int64_t nblocks,
                                               int64_t nqblocks, const uint64_t *occ,
                                               const uint64_t *rend, const uint16_t *slots,
                                               const uint32_t *offs) {
  const uint64_t total = static_cast<uint64_t>(nblocks) * 64;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; j < total; j += stride) {
    const int64_t bi = static_cast<int64_t>(j >> 6);
    b[bi].s[j & 63] = static_cast<T>(slots[j]);
    if ((j & 63) == 0) {
      b[bi].rend = rend[bi];
      b[bi].off = offs[bi];
      b[bi].occ = bi < nqblocks ? occ[bi] : 0ull;
    }
  }
}

inline uint32_t grid_for(uint64_t n, uint32_t kpl = 1) {
  uint64_t g = (n + NT * kpl - 1) / (NT * kpl);
  if (g < 1) g = 1;
  if (g > 262140) g = 262140;
  return static_cast<uint32_t>(g);
}

template <typename T, int KPL>
void lookup_kpl(qf_filter *f, const uint64_t *keys, uint64_t n, uint8_t *out8, uint64_t *out64, hipStream_t s) {
  const Block<T> *b0 = static_cast<const Block<T> *>(f->blk[0]);
  const Block<T> *b1 = static_cast<const Block<T> *>(f->blk[1]);
  const int64_t nb = static_cast<int64_t>(f->nblocks);
  if (out64)
    k_lookup<T, true, KPL><<<grid_for(n, KPL), NT, 0, s>>>(b0, b1, f->state, keys, n, f->q, f->r, nb, nullptr,
                                                           out64);
  else
    k_lookup<T, false, KPL><<<grid_for(n, KPL), NT, 0, s>>>(b0, b1, f->state, keys, n, f->q, f->r, nb, out8,
                                                            nullptr);
}

template <typename T>
hipError_t lookup_t(qf_filter *f, const uint64_t *keys, uint64_t n, uint8_t *out8,
                    uint64_t *out64, hipStream_t s) {
  Timer *t = f->pipe.timer;
  if (t) t->begin(QF_PROF_LOOKUP, s);
  const uint32_t kpl = f->pipe.tune.lookup_kpl;
  if (kpl >= 4)
    lookup_kpl<T, 4>(f, keys, n, out8, out64, s);
  else if (kpl == 2)
    lookup_kpl<T, 2>(f, keys, n, out8, out64, s);
  else
    lookup_kpl<T, 1>(f, keys, n, out8, out64, s);
  if (t) t->end(QF_PROF_LOOKUP, s);
  return hipGetLastError();
}

template <typename T, int KPL>
void lookup_multi_kpl(const Pipe &p, const uint64_t *keys, const uint32_t *fid, uint64_t n, uint8_t *out8,
                      uint64_t *out64, hipStream_t s) {
  if (out64)
    k_lookup_multi<T, true, KPL><<<grid_for(n, KPL), NT, 0, s>>>(p.d_desc, p.nf, keys, fid, n, nullptr, out64,
                                                                 p.pst);
  else
    k_lookup_multi<T, false, KPL><<<grid_for(n, KPL), NT, 0, s>>>(p.d_desc, p.nf, keys, fid, n, out8, nullptr,
                                                                  p.pst);
}

template <typename T>
hipError_t lookup_multi_t(const Pipe &p, const uint64_t *keys, const uint32_t *fid, uint64_t n, uint8_t *out8,
                          uint64_t *out64, hipStream_t s) {
  if (p.timer) p.timer->begin(QF_PROF_LOOKUP, s);
  if (p.tune.lookup_kpl >= 4)
    lookup_multi_kpl<T, 4>(p, keys, fid, n, out8, out64, s);
  else if (p.tune.lookup_kpl == 2)
    lookup_multi_kpl<T, 2>(p, keys, fid, n, out8, out64, s);
  else
    lookup_multi_kpl<T, 1>(p, keys, fid, n, out8, out64, s);
  if (p.timer) p.timer->end(QF_PROF_LOOKUP, s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lookup_multi(const Pipe &p, const uint64_t *keys, const uint32_t *fid, uint64_t n,
                               uint8_t *out8, uint64_t *out64, hipStream_t s) {
  if (p.r == 8) return lookup_multi_t<uint8_t>(p, keys, fid, n, out8, out64, s);
  return lookup_multi_t<uint16_t>(p, keys, fid, n, out8, out64, s);
}

uint64_t table_bytes(uint64_t nblocks, uint32_t r) {
  const uint64_t bb = r == 8 ? sizeof(Block<uint8_t>) : sizeof(Block<uint16_t>);
  return nblocks * bb;
}

hipError_t launch_lookup(qf_filter *f, const uint64_t *keys, uint64_t n, uint8_t *out8,
                         uint64_t *out64, hipStream_t s) {
  if (f->r == 8) return lookup_t<uint8_t>(f, keys, n, out8, out64, s);
  return lookup_t<uint16_t>(f, keys, n, out8, out64, s);
}

hipError_t launch_kv_lookup(qf_filter *f, const uint64_t *keys, uint64_t n, uint64_t *value, uint32_t *nvalues,
                            hipStream_t s) {
  const int64_t nb = static_cast<int64_t>(f->nblocks);
  if (f->r == 8)
    k_kv_lookup<uint8_t><<<grid_for(n), NT, 0, s>>>(static_cast<const Block<uint8_t> *>(f->blk[0]),
                                                    static_cast<const Block<uint8_t> *>(f->blk[1]), f->state, keys,
                                                    n, f->q, f->r, f->vbits, nb, value, nvalues);
  else
    k_kv_lookup<uint16_t><<<grid_for(n), NT, 0, s>>>(static_cast<const Block<uint16_t> *>(f->blk[0]),
                                                     static_cast<const Block<uint16_t> *>(f->blk[1]), f->state,
                                                     keys, n, f->q, f->r, f->vbits, nb, value, nvalues);
  return hipGetLastError();
}

hipError_t launch_export(qf_filter *f, uint64_t *occ, uint64_t *rend, uint16_t *slots,
                         uint32_t *offs, hipStream_t s) {
  const uint64_t total = f->nblocks * 64;
  const int64_t nb = static_cast<int64_t>(f->nblocks), nq = static_cast<int64_t>(f->N / 64);
  if (f->r == 8)
    k_export<uint8_t><<<grid_for(total), NT, 0, s>>>(
        static_cast<const Block<uint8_t> *>(f->blk[0]), static_cast<const Block<uint8_t> *>(f->blk[1]),
        f->state, nb, nq, occ, rend, slots, offs);
  else
    k_export<uint16_t><<<grid_for(total), NT, 0, s>>>(
        static_cast<const Block<uint16_t> *>(f->blk[0]), static_cast<const Block<uint16_t> *>(f->blk[1]),
        f->state, nb, nq, occ, rend, slots, offs);
  return hipGetLastError();
}

hipError_t launch_import(qf_filter *f, const uint64_t *occ, const uint64_t *rend,
                         const uint16_t *slots, const uint32_t *offs, hipStream_t s) {
  const uint64_t total = f->nblocks * 64;
  const int64_t nb = static_cast<int64_t>(f->nblocks), nq = static_cast<int64_t>(f->N / 64);
  if (f->r == 8)
    k_import<uint8_t><<<grid_for(total), NT, 0, s>>>(static_cast<Block<uint8_t> *>(f->blk[0]),
                                                     nb, nq, occ, rend, slots, offs);
  else
    k_import<uint16_t><<<grid_for(total), NT, 0, s>>>(static_cast<Block<uint16_t> *>(f->blk[0]),
                                                      nb, nq, occ, rend, slots, offs);
  return hipGetLastError();
}

}  // namespace qf
