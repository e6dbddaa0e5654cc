// qf_enum.hip -- enumeration of a filter's multiset, the basis of union,
// difference and re-layout of filters.
//
// The paper lists enumeration, merging and resizing among the counting
// quotient filter's features (Sec. 1 and 2) without describing how; this is
// the library's design.  A filter's table is a pure function of the multiset
// of p-bit fingerprints it stores, and the table keeps every fingerprint
// whole (quotient = high q bits, remainder = low r bits), so:
//   * enumeration decodes the runs in quotient order into sorted
//     <fingerprint, count> pairs;
//   * the union (or saturating difference) of two filters with the same
//     fingerprint length p is the bulk merge of one filter's enumeration into
//     the other, as an already sorted and reduced batch (Sec. 5.3-5.4 without
//     the sort);
//   * re-laying a filter under another split q' + r' = q + r (for example
//     2^20 quotients with 16-bit remainders into 2^28 quotients with 8-bit
//     remainders) is the union of it into an empty filter of that shape.
// One lane per 64-quotient block: it finds the run of the block's first
// occupied quotient with the block offset and the run-end words (offset +
// select), then walks the following runs (each ends at the next run-end bit)
// and decodes their entries.  A count pass, an exclusive scan of the per-block
// counts and a write pass give the pairs in order.
#include "qf_dev.h"
#include "qf.h"
#include "qf_lib.h"

namespace qf {
namespace {

constexpr int NT = 256;

// position of the first set run-end bit strictly after position q (or -1)
template <typename T>
__device__ __forceinline__ int64_t next_end_after(const Block<T> *b, int64_t nblocks, int64_t q) {
  int64_t w = (q + 1) >> 6;
  if (w >= nblocks) return -1;
  uint64_t m = b[w].rend & (~0ull << ((q + 1) & 63));
  while (!m) {
    if (++w >= nblocks) return -1;
    m = b[w].rend;
  }
  return (w << 6) + ctz64(m);
}

template <typename T>
struct GlbSlots {
  const Block<T> *b;
  __device__ uint64_t slot(int64_t j) const { return b[j >> 6].s[j & 63]; }
};

// Count (WRITE = false: entries per quotient block into counts[]) or write
// (fingerprint, count) pairs at offs[block] of the runs of quotient block bi.
// A count of 2^32 or more sets *big (the staged merge keeps counts in 32 bits).
template <typename T, bool WRITE>
__global__ __launch_bounds__(NT) void k_enum(const Block<T> *b0, const Block<T> *b1, const uint64_t *state,
                                             int64_t nqb, int64_t nblocks, uint32_t r, uint32_t *counts,
                                             const uint32_t *offs, const uint64_t *base_hi,
                                             uint64_t *__restrict__ fp_out, uint64_t *__restrict__ cnt_out,
                                             uint64_t *big) {
  const int64_t bi = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (bi >= nqb) return;
  const Block<T> *b = (state[ST_CUR] & 1ull) ? b1 : b0;
  uint64_t occ = b[bi].occ;
  uint32_t k = 0;
  // (the exclusive offsets are 32-bit per block within a segment of the
  // scan; base_hi adds the segment's 64-bit base)
  const uint64_t o = WRITE ? base_hi[bi / (NT * 16)] + offs[bi] : 0ull;
  if (occ) {
    GlbSlots<T> g{b};
    int64_t x = (bi << 6) + ctz64(occ);
    // the run of the block's first occupied quotient x: it ends at the
    // block offset's position when x is the block's first quotient, else at
    // the first run end after it; it starts one past the last run end in
    // [x, e - 1], or at x
    const int64_t p = (bi << 6) + static_cast<int64_t>(b[bi].off);
    int64_t e = x == (bi << 6) ? p : next_end_after(b, nblocks, p);
    int64_t s = x;
    for (int64_t j = e - 1; j >= x; --j) {
      if ((b[j >> 6].rend >> (j & 63)) & 1ull) {
        s = j + 1;
        break;
      }
    }
    for (;;) {
      int64_t pos = s;
      while (pos <= e) {
        uint64_t rem, c;
        pos = dec_entry(g, pos, e, r, rem, c);
        if (WRITE) {
          fp_out[o + k] = (static_cast<uint64_t>(x) << r) | rem;
          cnt_out[o + k] = c;
          if (c >> 32) *big = 1;
        }
        ++k;
      }
      occ &= occ - 1;
      if (!occ) break;
      x = (bi << 6) + ctz64(occ);
      s = max(x, e + 1);
      e = next_end_after(b, nblocks, e);
      if (e < 0) break;  // (a consistent table always has the run end)
    }
  }
  if (!WRITE) counts[bi] = k;
}

// Exclusive scan of counts[0, n) in segments of NT * 16 values: each
// work-group scans its segment in place (32-bit: every entry takes at least
// one slot and a table has fewer than 2^32 slots) and writes the segment
// total; a single work-group then turns the totals into 64-bit bases.
__global__ __launch_bounds__(NT) void k_seg_scan(uint32_t *counts, int64_t n, uint64_t *seg_tot) {
  __shared__ uint32_t sh[NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t s0 = static_cast<int64_t>(blockIdx.x) * NT * 16;
  uint32_t v[16];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t i = s0 + static_cast<int64_t>(tid) * 16 + k;
    v[k] = i < n ? counts[i] : 0u;
    sum += v[k];
  }
  uint32_t inc = sum;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(inc, d);
    if (lane >= d) inc += t;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  uint32_t run = inc - sum;
  for (int w = 0; w < wv; ++w) run += sh[w];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t i = s0 + static_cast<int64_t>(tid) * 16 + k;
    if (i < n) counts[i] = run;
    run += v[k];
  }
  if (tid == NT - 1) seg_tot[blockIdx.x] = run;
}

// seg_tot[0, m) -> exclusive 64-bit bases; the grand total goes to *total
__global__ __launch_bounds__(1024) void k_seg_bases(uint64_t *seg_tot, uint32_t m, uint64_t *total) {
  __shared__ uint64_t part[1024];
  const int tid = threadIdx.x;
  const uint32_t per = (m + 1023) / 1024;
  const uint32_t lo = min(m, tid * per), hi = min(m, lo + per);
  uint64_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += seg_tot[i];
  part[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint64_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint64_t run = part[tid] - s;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint64_t v = seg_tot[i];
    seg_tot[i] = run;
    run += v;
  }
  if (tid == 1023) {
    total[0] = part[1023];
    total[1] = 0;  // the write pass's flag for counts of 2^32 or more
  }
}

template <typename T>
hipError_t enum_t(qf_filter *f, uint32_t *counts, uint64_t *seg, uint64_t *words, uint64_t *fp, uint64_t *cnt,
                  bool write, hipStream_t s) {
  const int64_t nqb = static_cast<int64_t>(f->N / 64);
  const uint32_t grid = static_cast<uint32_t>((nqb + NT - 1) / NT);
  const Block<T> *b0 = static_cast<const Block<T> *>(f->blk[0]);
  const Block<T> *b1 = static_cast<const Block<T> *>(f->blk[1]);
  const int64_t nb = static_cast<int64_t>(f->nblocks);
  if (!write) {
    k_enum<T, false><<<grid, NT, 0, s>>>(b0, b1, f->state, nqb, nb, f->r, counts, nullptr, nullptr, nullptr,
                                         nullptr, nullptr);
    const uint32_t nseg = static_cast<uint32_t>((nqb + NT * 16 - 1) / (NT * 16));
    k_seg_scan<<<nseg, NT, 0, s>>>(counts, nqb, seg);
    k_seg_bases<<<1, 1024, 0, s>>>(seg, nseg, words);
  } else {
    k_enum<T, true><<<grid, NT, 0, s>>>(b0, b1, f->state, nqb, nb, f->r, nullptr, counts, seg, fp, cnt,
                                        words + 1);
  }
  return hipGetLastError();
}

}  // namespace

uint64_t enum_scratch_bytes(const qf_filter *f) {
  const uint64_t nqb = f->N / 64;
  const uint64_t nseg = (nqb + NT * 16 - 1) / (NT * 16);
  return nqb * 4 + nseg * 8 + 2 * 8;
}

hipError_t launch_enum(qf_filter *f, void *scratch, uint64_t *fp, uint64_t *cnt, bool write, hipStream_t s) {
  const uint64_t nqb = f->N / 64;
  const uint64_t nseg = (nqb + NT * 16 - 1) / (NT * 16);
  uint8_t *p = static_cast<uint8_t *>(scratch);
  uint32_t *counts = reinterpret_cast<uint32_t *>(p);
  uint64_t *seg = reinterpret_cast<uint64_t *>(p + ((nqb * 4 + 7) / 8) * 8);
  uint64_t *words = seg + nseg;  // [0] total, [1] a count of 2^32 or more
  if (f->r == 8) return enum_t<uint8_t>(f, counts, seg, words, fp, cnt, write, s);
  return enum_t<uint16_t>(f, counts, seg, words, fp, cnt, write, s);
}

}  // namespace qf
