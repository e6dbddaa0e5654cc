// qf_sort.hip -- batch preparation: hash, radix sort, reduction to <fingerprint,
// count> and region bounds.
//
// Sec. 5.3 (Sorting hashes): the batch is hashed and sorted so that a region
// can take its items in remainder order and the buffers of the regions are
// contiguous pieces of the sorted input, found by successor search.
// Sec. 5.4: duplicates are reduced to <item, count> pairs before the insert.
// The sort is an LSD radix sort written for wave64: 8-bit digits, one LDS
// histogram per wave, stable ranks from wave ballots.
#include <algorithm>

#include "qf_dev.h"
#include "qf.h"
#include "qf_lib.h"

namespace qf {
namespace {

constexpr int NT = 256;
constexpr int NWAVE = NT / 64;
constexpr uint32_t RADIX_BITS = 8;                 // widest digit
constexpr int RADIX_MAX = 1 << RADIX_BITS;        // digits per pass, at most

__device__ __forceinline__ uint64_t chunk_lo(uint64_t n, uint32_t G, uint32_t g) {
  return (n * g) / G;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << __lane_id()) - 1ull;
}

__global__ __launch_bounds__(NT) void k_hash(const uint64_t *__restrict__ keys, uint64_t n,
                                             uint64_t pmask, uint64_t *__restrict__ fp) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride)
    fp[i] = mix64(keys[i]) & pmask;
}

// Value association: the fingerprint of (key i, value i) is the key's
// fingerprint of q + r - vbits bits followed by the value's low vbits bits.
__global__ __launch_bounds__(NT) void k_kv_compose(const uint64_t *__restrict__ keys,
                                                   const uint64_t *__restrict__ values, uint64_t n,
                                                   uint64_t kmask, uint32_t vbits, uint64_t *__restrict__ fp) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  const uint64_t vmask = (1ull << vbits) - 1ull;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride)
    fp[i] = ((mix64(keys[i]) & kmask) << vbits) | (values[i] & vmask);
}

// Composite keys of a filter set: key i goes to filter fid[i]; its
// fingerprint's region becomes a global region index in the high bits, the
// fingerprint bits inside the region stay in the low RL + r bits.  A filter
// index out of range gives the key ~0 (past every region, so it is dropped)
// and flags the call (pst[ST_ERR]).
__global__ __launch_bounds__(NT) void k_hash_multi(const uint64_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ fid, uint64_t n,
                                                   const FDesc *__restrict__ desc, uint32_t nf,
                                                   uint32_t RL, uint64_t *__restrict__ out,
                                                   uint64_t *pst) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride) {
    const uint32_t f = fid[i];
    if (f >= nf) {
      out[i] = ~0ull;
      pst[ST_ERR] = static_cast<uint64_t>(static_cast<int64_t>(QF_ERR_ARG));
      continue;
    }
    const FDesc &d = desc[f];
    const uint32_t p = d.q + d.r, lb = d.rlog + d.r;
    const uint64_t fp = mix64(keys[i]) & ((1ull << p) - 1ull);
    const uint64_t g = d.rbase + (fp >> lb);
    out[i] = (g << (RL + d.r)) | (fp & ((1ull << lb) - 1ull));
  }
}

__global__ __launch_bounds__(NT) void k_take_errors(const FDesc *__restrict__ desc, uint32_t nf,
                                                    int64_t *__restrict__ err) {
  const uint32_t f = blockIdx.x * NT + threadIdx.x;
  if (f >= nf) return;
  uint64_t *st = desc[f].state;
  err[f] = static_cast<int64_t>(st[ST_ERR]);
  st[ST_ERR] = 0;
}

// Used slots past the last quotient: a slot at or after N is used only if
// the slot before it is, so they form one stretch [N, N + t) that ends at the
// table's last run end, and block N/64's offset is that end's distance from N
// (0 both when it is N itself, which sets the block's first run-end bit, and
// when it lies before N).
template <typename T>
__device__ int64_t tail_used(const FDesc &d) {
  const Block<T> *b = static_cast<const Block<T> *>(d.blk[d.state[ST_CUR] & 1ull]);
  const Block<T> &h = b[d.N >> 6];
  return (h.off || (h.rend & 1ull)) ? static_cast<int64_t>(h.off) + 1 : 0;
}

__global__ __launch_bounds__(NT) void k_take_tails(const FDesc *__restrict__ desc, uint32_t nf,
                                                   int64_t *__restrict__ tail) {
  const uint32_t f = blockIdx.x * NT + threadIdx.x;
  if (f >= nf) return;
  tail[f] = desc[f].r == 8 ? tail_used<uint8_t>(desc[f]) : tail_used<uint16_t>(desc[f]);
}

__global__ __launch_bounds__(NT) void k_fill(uint64_t *p, uint64_t n, uint64_t v) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += stride)
    p[i] = v;
}

// per-group digit histogram, stored digit-major: hist[d * G + g], for digits
// of nbits <= log2(ND) bits at `shift`.  With HASH the input is the raw keys
// and the sorted value is mix64(key) & pmask (the hash is fused into the
// first pass).
template <bool HASH, int ND>
__global__ __launch_bounds__(NT) void k_rs_hist(const uint64_t *__restrict__ in, uint64_t n,
                                                uint32_t G, uint32_t shift, uint32_t nbits, uint64_t pmask,
                                                uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[NWAVE][ND];
  const int tid = threadIdx.x, wv = tid >> 6;
  for (int d = tid; d < ND; d += NT)
    for (int w = 0; w < NWAVE; ++w) h[w][d] = 0;
  __syncthreads();
  const uint32_t g = blockIdx.x;
  const uint32_t dmask = (1u << nbits) - 1u;
  const uint64_t lo = chunk_lo(n, G, g), hi = chunk_lo(n, G, g + 1);
  // (eight loads in flight per lane, then their counts)
  for (uint64_t i0 = lo + tid; i0 < hi; i0 += 8ull * NT) {
    uint64_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t i = i0 + static_cast<uint64_t>(k) * NT;
      v[k] = i < hi ? in[i] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool valid = i0 + static_cast<uint64_t>(k) * NT < hi;
      const uint64_t x = HASH ? (mix64(v[k]) & pmask) : v[k];
      const uint32_t d = static_cast<uint32_t>(x >> shift) & dmask;
      // Skewed keys put many lanes of a wave on one digit, and LDS atomics
      // on one address serialise: the lanes that share the first valid
      // lane's digit are counted by one atomic of that lane.
      const uint64_t act = __ballot(valid);
      if (act) {
        const uint32_t d0 = static_cast<uint32_t>(__shfl(static_cast<int>(d), __builtin_ctzll(act)));
        const uint64_t same = __ballot(valid && d == d0);
        if (valid && d == d0) {
          if ((same & ((1ull << (threadIdx.x & 63)) - 1ull)) == 0)
            atomicAdd(&h[wv][d0], static_cast<uint32_t>(popc64(same)));
        } else if (valid) {
          atomicAdd(&h[wv][d], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (int d = tid; d < ND; d += NT) {
    uint32_t t = 0;
    for (int w = 0; w < NWAVE; ++w) t += h[w][d];
    hist[static_cast<uint64_t>(d) * G + g] = t;
  }
}

// Work-group d turns the G group counts of digit d into exclusive prefixes
// and writes the digit's total to dtot[d].
__global__ __launch_bounds__(NT) void k_rs_offsets(uint32_t *__restrict__ hist, uint32_t G,
                                                   uint32_t *__restrict__ dtot) {
  __shared__ uint32_t sh[NWAVE];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t d = blockIdx.x;
  uint32_t *row = hist + static_cast<uint64_t>(d) * G;
  const uint32_t per = (G + NT - 1) / NT;
  const uint32_t lo = min(G, tid * per), hi = min(G, lo + per);
  uint32_t loc = 0;
  for (uint32_t i = lo; i < hi; ++i) loc += row[i];
  uint32_t inc = loc;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  uint32_t run = inc - loc;
  for (int w = 0; w < wv; ++w) run += sh[w];
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t c = row[i];
    row[i] = run;
    run += c;
  }
  if (tid == NT - 1) {
    uint32_t t = 0;
    for (int w = 0; w < NWAVE; ++w) t += sh[w];
    dtot[d] = t;
  }
}

// exclusive scan of a[0..n) in place by one work-group of 1024 threads (used
// for the G tile counts of the duplicate reduction); the total goes to
// *total if it is not null
__global__ __launch_bounds__(1024) void k_scan_u32(uint32_t *a, uint32_t n, uint64_t *total) {
  __shared__ uint32_t part[1024];
  const int tid = threadIdx.x;
  const uint32_t per = (n + 1023) / 1024;
  const uint32_t lo = min(n, tid * per), hi = min(n, lo + per);
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += a[i];
  part[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint32_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = part[tid] - s;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  if (tid == 1023 && total) *total = part[1023];
}

// Exclusive scan over the ND digits of a work-group, DPT = ND / NT digits per
// lane (lane t holds digits t DPT .. t DPT + DPT - 1, in order).
template <int DPT>
__device__ __forceinline__ void digits_exscan(const uint32_t (&v)[DPT], uint32_t (&ex)[DPT], uint32_t *sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < DPT; ++j) sum += v[j];
  uint32_t inc = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  uint32_t run = inc - sum;
  for (int w = 0; w < wv; ++w) run += sh[w];
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    ex[j] = run;
    run += v[j];
  }
  __syncthreads();
}

// Stable scatter of one digit.  Each group takes its chunk in tiles of TILE
// keys; wave w of the work-group owns the tile's w-th quarter, read in
// rounds of 64 consecutive keys.  A wave ranks its keys on its own (wave
// ballots over the digit bits give the rank inside a round, a per-wave LDS
// counter per digit the keys of earlier rounds), so the only work-group
// barriers are between the tile's phases: rank, per-digit offsets (tile digit
// starts, then the waves in order), placement into LDS in digit order, and the
// copy-out, where each digit's keys of the tile land as one contiguous run
// (coalesced stores).  The order inside a digit is the input order: stable.
template <bool HASH, int TILE, int ND>
// (at most 128 VGPRs, so four 4096-key work-groups fit a CU's registers as
// well as its LDS: a 2^22-key pass of 1024 groups runs in one round)
__global__ __launch_bounds__(NT, 4) void k_rs_scatter(const uint64_t *__restrict__ in,
                                                   uint64_t *__restrict__ out, uint64_t n,
                                                   uint32_t G, uint32_t shift, uint32_t nbits,
                                                   uint64_t pmask,
                                                   const uint32_t *__restrict__ hist,
                                                   const uint32_t *__restrict__ dtot) {
  constexpr int KPL = TILE / NT;    // rounds per wave
  constexpr int WQ = TILE / NWAVE;  // keys per wave and tile
  constexpr int DPT = ND / NT;
  __shared__ uint64_t tile[TILE];
  __shared__ uint32_t gpos[ND];  // global position of the group's next key of digit d
  __shared__ uint32_t loff[ND];  // start of digit d in the tile
  __shared__ uint32_t placed[ND];
  __shared__ uint32_t wc[NWAVE][ND];  // per wave: keys of digit d (then: its first tile position)
  __shared__ uint32_t sh[NWAVE];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const uint32_t g = blockIdx.x;
  {
    // keys with a smaller digit: exclusive scan of the digit totals
    uint32_t v[DPT], ex[DPT];
#pragma unroll
    for (int j = 0; j < DPT; ++j) v[j] = dtot[tid * DPT + j];
    digits_exscan<DPT>(v, ex, sh);
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = tid * DPT + j;
      gpos[d] = ex[j] + hist[static_cast<uint64_t>(d) * G + g];
      for (int w = 0; w < NWAVE; ++w) wc[w][d] = 0;
    }
  }
  __syncthreads();
  const uint64_t lo = chunk_lo(n, G, g), hi = chunk_lo(n, G, g + 1);
  const uint32_t dmask = (1u << nbits) - 1u;
  const uint64_t below = (1ull << lane) - 1ull;
  for (uint64_t t0 = lo; t0 < hi; t0 += TILE) {
    const uint32_t cnt = static_cast<uint32_t>(min(static_cast<uint64_t>(TILE), hi - t0));
    // 1. rank: each wave over its quarter, round by round
    uint64_t key[KPL];
    uint32_t rk[KPL];
    // (all of the wave's loads first, so that they are in flight together)
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
      const uint32_t jj = wv * WQ + k * 64 + lane;
      key[k] = jj < cnt ? in[t0 + jj] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
      const uint32_t jj = wv * WQ + k * 64 + lane;
      const bool valid = jj < cnt;
      if (HASH) key[k] = mix64(key[k]) & pmask;
      const uint32_t d = static_cast<uint32_t>(key[k] >> shift) & dmask;
      uint64_t peers = __ballot(valid);
      for (uint32_t b = 0; b < nbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
      }
      const uint32_t before = valid ? wc[wv][d] : 0u;
      const uint32_t r = static_cast<uint32_t>(popc64(peers & below));
      rk[k] = before + r;
      // (the wave's lanes read the counter before its first lane of the
      // digit writes it: a wave's LDS accesses complete in program order)
      if (valid && r == 0) wc[wv][d] = before + static_cast<uint32_t>(popc64(peers));
    }
    __syncthreads();
    // 2. per digit: the tile's digit starts, then each wave's first position
    {
      uint32_t v[DPT], ex[DPT];
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const int d = tid * DPT + j;
        uint32_t t = 0;
        for (int w = 0; w < NWAVE; ++w) t += wc[w][d];
        v[j] = t;
      }
      digits_exscan<DPT>(v, ex, sh);
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const int d = tid * DPT + j;
        loff[d] = ex[j];
        placed[d] = v[j];
        uint32_t run = ex[j];
        for (int w = 0; w < NWAVE; ++w) {
          const uint32_t c = wc[w][d];
          wc[w][d] = run;
          run += c;
        }
      }
    }
    __syncthreads();
    // 3. the tile in digit order in LDS
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
      const uint32_t jj = wv * WQ + k * 64 + lane;
      if (jj < cnt) {
        const uint32_t d = static_cast<uint32_t>(key[k] >> shift) & dmask;
        tile[wc[wv][d] + rk[k]] = key[k];
      }
    }
    __syncthreads();
    // 4. each digit's run to its global place
    for (uint32_t jj = tid; jj < cnt; jj += NT) {
      const uint64_t v = tile[jj];
      const uint32_t d = static_cast<uint32_t>(v >> shift) & dmask;
      out[gpos[d] + (jj - loff[d])] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = tid * DPT + j;
      gpos[d] += placed[d];
      for (int w = 0; w < NWAVE; ++w) wc[w][d] = 0;
    }
    __syncthreads();
  }
}

// ---- run-length reduction -------------------------------------------------
__device__ __forceinline__ bool is_head(const uint64_t *s, uint64_t i) {
  return i == 0 || s[i] != s[i - 1];
}

__global__ __launch_bounds__(NT) void k_rle_count(const uint64_t *__restrict__ s, uint64_t n,
                                                  uint32_t G, uint32_t *__restrict__ cnt) {
  __shared__ uint32_t red[NWAVE];
  const int tid = threadIdx.x;
  const uint32_t g = blockIdx.x;
  const uint64_t lo = chunk_lo(n, G, g), hi = chunk_lo(n, G, g + 1);
  uint32_t c = 0;
#pragma unroll 8
  for (uint64_t i = lo + tid; i < hi; i += NT) c += is_head(s, i);
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((tid & 63) == 0) red[tid >> 6] = c;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
    for (int w = 0; w < NWAVE; ++w) t += red[w];
    cnt[g] = t;
  }
}

// The run heads of group g's chunk, in order, from output index cnt[g] (the
// exclusive scan of k_rle_count's head counts).  A round takes RLE_K rows of
// NT consecutive keys, all requested at once (coalesced).  A key's
// predecessor comes from the lane before (a shuffle), across waves and rows
// from each wave's last keys in LDS; wave ballots mark the heads, and one
// wave scans the RLE_K x NWAVE per-wave head counts (row-major = key order).
constexpr int RLE_K = 16;
static_assert(RLE_K * NWAVE == 64, "one wave scans the per-wave head counts");
__global__ __launch_bounds__(NT) void k_rle_write(const uint64_t *__restrict__ s, uint64_t n,
                                                  uint32_t G, const uint32_t *__restrict__ cnt,
                                                  uint64_t *__restrict__ ufp,
                                                  uint64_t *__restrict__ ustart) {
  __shared__ uint64_t edge[RLE_K * NWAVE];  // each wave's last key of each row
  __shared__ uint32_t wcnt[RLE_K * NWAVE];  // heads per (row, wave), then their exclusive prefix
  __shared__ uint32_t tot_s;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const uint32_t g = blockIdx.x;
  const uint64_t lo = chunk_lo(n, G, g), hi = chunk_lo(n, G, g + 1);
  const uint64_t lt = lanemask_lt();
  uint32_t base = cnt[g];
  for (uint64_t t0 = lo; t0 < hi; t0 += static_cast<uint64_t>(NT) * RLE_K) {
    uint64_t v[RLE_K];
#pragma unroll
    for (int k = 0; k < RLE_K; ++k) {
      const uint64_t i = t0 + static_cast<uint64_t>(k) * NT + tid;
      v[k] = i < hi ? s[i] : 0ull;
    }
    const uint64_t before0 = (tid == 0 && t0 > 0) ? s[t0 - 1] : 0ull;
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < RLE_K; ++k) edge[k * NWAVE + wv] = v[k];
    }
    __syncthreads();
    uint64_t bal[RLE_K];
#pragma unroll
    for (int k = 0; k < RLE_K; ++k) {
      const uint64_t i = t0 + static_cast<uint64_t>(k) * NT + tid;
      const uint64_t up = __shfl_up(v[k], 1);
      uint64_t before = up;
      if (lane == 0) before = wv ? edge[k * NWAVE + wv - 1] : (k ? edge[(k - 1) * NWAVE + NWAVE - 1] : before0);
      const bool h = i < hi && (i == 0 || v[k] != before);
      bal[k] = __ballot(h);
      if (lane == 0) wcnt[k * NWAVE + wv] = static_cast<uint32_t>(popc64(bal[k]));
    }
    __syncthreads();
    if (wv == 0) {
      const uint32_t c = wcnt[lane];
      uint32_t inc = c;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
      }
      wcnt[lane] = inc - c;
      if (lane == 63) tot_s = inc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RLE_K; ++k) {
      if ((bal[k] >> lane) & 1ull) {
        const uint32_t pos = base + wcnt[k * NWAVE + wv] + static_cast<uint32_t>(popc64(bal[k] & lt));
        ufp[pos] = v[k];
        ustart[pos] = t0 + static_cast<uint64_t>(k) * NT + tid;
      }
    }
    base += tot_s;
    __syncthreads();  // (edge, wcnt and tot_s are rewritten by the next round)
  }
}

__global__ __launch_bounds__(NT) void k_rle_counts(const uint64_t *__restrict__ ustart,
                                                   uint64_t n, const uint64_t *state,
                                                   uint64_t *__restrict__ ucnt) {
  const uint64_t u = state[ST_NUNIQ];
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * NT + threadIdx.x; j < u; j += stride)
    ucnt[j] = (j + 1 < u ? ustart[j + 1] : n) - ustart[j];
}

// Batches of at most SMALL_KEYS keys: one work-group sorts them in LDS with
// the same LSD passes and wave-ballot ranking as the scatter (the keys stay in
// registers between passes and go through LDS only to be reordered), then
// reduces runs of equal keys, writing the distinct keys, their counts and
// their number (state[ST_NUNIQ]).  One launch instead of three per radix pass
// and four for the reduction, which dominate small updates.  With HASH the
// input is raw keys and the sorted value is mix64(key) & pmask.
template <bool HASH>
__global__ __launch_bounds__(NT) void k_small_prep(const uint64_t *__restrict__ in, uint32_t n, uint32_t bits,
                                                   uint64_t pmask, uint64_t *__restrict__ ufp,
                                                   uint64_t *__restrict__ ucnt, uint64_t *state) {
  constexpr int KPL = SMALL_KEYS / NT;    // rounds of 64 keys per wave
  constexpr int WQ = SMALL_KEYS / NWAVE;  // keys per wave
  static_assert(NWAVE * KPL == 64, "one wave scans the per-(wave, round) head counts");
  static_assert(RADIX_MAX == NT, "one digit per lane");
  __shared__ uint64_t tile[SMALL_KEYS];
  __shared__ uint32_t wc[NWAVE][RADIX_MAX];
  __shared__ uint32_t sh[NWAVE];
  __shared__ uint32_t rowc[NWAVE * KPL];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  // key k of a lane has index wv WQ + 64 k + lane (wave-major, then round)
  uint64_t key[KPL];
#pragma unroll
  for (int k = 0; k < KPL; ++k) {
    const uint32_t j = wv * WQ + k * 64 + lane;
    key[k] = j < n ? (HASH ? (mix64(in[j]) & pmask) : in[j]) : 0ull;
  }
  const uint32_t npass = (bits + RADIX_BITS - 1) / RADIX_BITS;
  const uint32_t db = npass ? (bits + npass - 1) / npass : 0;
  for (uint32_t p = 0; p < npass; ++p) {
    const uint32_t shift = db * p;
    const uint32_t nb = bits - shift < db ? bits - shift : db;
    const uint32_t dmask = (1u << nb) - 1u;
    for (int w = 0; w < NWAVE; ++w) wc[w][tid] = 0;
    __syncthreads();
    // 1. rank inside each wave, round by round
    uint32_t rk[KPL];
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
      const uint32_t j = wv * WQ + k * 64 + lane;
      const bool valid = j < n;
      const uint32_t d = static_cast<uint32_t>(key[k] >> shift) & dmask;
      uint64_t peers = __ballot(valid);
      for (uint32_t b = 0; b < nb; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
      }
      const uint32_t before = valid ? wc[wv][d] : 0u;
      const uint32_t r = static_cast<uint32_t>(popc64(peers & below));
      rk[k] = before + r;
      // (the wave's lanes read the counter before its first lane of the
      // digit writes it: a wave's LDS accesses complete in program order)
      if (valid && r == 0) wc[wv][d] = before + static_cast<uint32_t>(popc64(peers));
    }
    __syncthreads();
    // 2. digit starts, then each wave's first position per digit
    {
      uint32_t v[1], ex[1];
      uint32_t t = 0;
      for (int w = 0; w < NWAVE; ++w) t += wc[w][tid];
      v[0] = t;
      digits_exscan<1>(v, ex, sh);
      uint32_t run = ex[0];
      for (int w = 0; w < NWAVE; ++w) {
        const uint32_t c = wc[w][tid];
        wc[w][tid] = run;
        run += c;
      }
    }
    __syncthreads();
    // 3. reorder through LDS
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
      const uint32_t j = wv * WQ + k * 64 + lane;
      if (j < n) {
        const uint32_t d = static_cast<uint32_t>(key[k] >> shift) & dmask;
        tile[wc[wv][d] + rk[k]] = key[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
      const uint32_t j = wv * WQ + k * 64 + lane;
      key[k] = j < n ? tile[j] : 0ull;
    }
  }
  // the sorted keys are in tile and, by index, in the lanes' registers:
  // run heads by wave ballots, their order by one wave's scan of the
  // per-(wave, round) counts
  uint64_t hb[KPL];
#pragma unroll
  for (int k = 0; k < KPL; ++k) {
    const uint32_t j = wv * WQ + k * 64 + lane;
    const bool h = j < n && (j == 0 || key[k] != tile[j - 1]);
    hb[k] = __ballot(h);
    if (lane == 0) rowc[wv * KPL + k] = static_cast<uint32_t>(popc64(hb[k]));
  }
  __syncthreads();
  if (wv == 0) {
    const uint32_t c = rowc[lane];
    uint32_t inc = c;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(inc, o);
      if (lane >= o) inc += t;
    }
    rowc[lane] = inc - c;
    if (lane == 63) sh[0] = inc;
  }
  __syncthreads();
  const uint32_t nu = sh[0];
  // each head's position, in head order, over the (no longer needed) tile
  uint32_t *const start = reinterpret_cast<uint32_t *>(tile);
  uint32_t ui[KPL];
#pragma unroll
  for (int k = 0; k < KPL; ++k) {
    ui[k] = rowc[wv * KPL + k] + static_cast<uint32_t>(popc64(hb[k] & below));
    if ((hb[k] >> lane) & 1ull) start[ui[k]] = wv * WQ + k * 64 + lane;
  }
  if (tid == 0) start[nu] = n;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KPL; ++k) {
    if ((hb[k] >> lane) & 1ull) {
      ufp[ui[k]] = key[k];
      ucnt[ui[k]] = start[ui[k] + 1] - start[ui[k]];
    }
  }
  if (tid == 0) state[ST_NUNIQ] = nu;
}

// Successor search (Sec. 5.3): rb[g] = first reduced entry whose (composite)
// key is >= the first key of region g, for the G regions of a pipeline.
__global__ __launch_bounds__(NT) void k_bounds(const uint64_t *__restrict__ ufp,
                                               const uint64_t *pst, uint32_t G, uint32_t shift,
                                               uint64_t *__restrict__ rb) {
  const uint32_t g = blockIdx.x * NT + threadIdx.x;
  if (g > G) return;
  const uint64_t u = pst[ST_NUNIQ];
  const uint64_t key = static_cast<uint64_t>(g) << shift;
  uint64_t lo = 0, hi = u;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (ufp[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  rb[g] = lo;
}

inline uint32_t blocks_for(uint64_t n, uint32_t cap = 65535u * 4u) {
  const uint64_t b = (n + NT - 1) / NT;
  return static_cast<uint32_t>(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

uint64_t sort_count_words(uint64_t cap) {
  const uint64_t g = std::min<uint64_t>(SORT_MAX_GROUPS, (cap + SORT_MIN_CHUNK - 1) / SORT_MIN_CHUNK);
  return static_cast<uint64_t>(RADIX_MAX) * (1 + std::max<uint64_t>(g, 1));
}

uint32_t sort_groups(uint64_t n, uint32_t chunk) {
  uint64_t g = (n + chunk - 1) / chunk;
  if (g < 1) g = 1;
  if (g > SORT_MAX_GROUPS) g = SORT_MAX_GROUPS;
  return static_cast<uint32_t>(g);
}

hipError_t launch_hash(const uint64_t *keys, uint64_t n, uint64_t pmask, uint64_t *fp,
                       hipStream_t s, Timer *t) {
  if (t) t->begin(QF_PROF_HASH, s);
  k_hash<<<blocks_for(n), NT, 0, s>>>(keys, n, pmask, fp);
  if (t) t->end(QF_PROF_HASH, s);
  return hipGetLastError();
}

hipError_t launch_kv_compose(const uint64_t *keys, const uint64_t *values, uint64_t n, uint64_t kmask,
                             uint32_t vbits, uint64_t *fp, hipStream_t s, Timer *t) {
  if (t) t->begin(QF_PROF_HASH, s);
  k_kv_compose<<<blocks_for(n), NT, 0, s>>>(keys, values, n, kmask, vbits, fp);
  if (t) t->end(QF_PROF_HASH, s);
  return hipGetLastError();
}

hipError_t launch_hash_multi(const uint64_t *keys, const uint32_t *fid, uint64_t n, const Pipe &p,
                             uint64_t *out, hipStream_t s, Timer *t) {
  if (t) t->begin(QF_PROF_HASH, s);
  k_hash_multi<<<blocks_for(n), NT, 0, s>>>(keys, fid, n, p.d_desc, p.nf, p.RL, out, p.pst);
  if (t) t->end(QF_PROF_HASH, s);
  return hipGetLastError();
}

hipError_t launch_take_errors(const Pipe &p, int64_t *err, hipStream_t s) {
  k_take_errors<<<(p.nf + NT - 1) / NT, NT, 0, s>>>(p.d_desc, p.nf, err);
  return hipGetLastError();
}

hipError_t launch_take_tails(const Pipe &p, int64_t *tail, hipStream_t s) {
  k_take_tails<<<(p.nf + NT - 1) / NT, NT, 0, s>>>(p.d_desc, p.nf, tail);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_fill<<<blocks_for(n), NT, 0, s>>>(p, n, v);
  return hipGetLastError();
}

// One LSD pass: histogram, digit offsets, scatter, with ND-digit kernels.
template <int ND>
void sort_pass(const uint64_t *in, uint64_t *out, const uint64_t *raw, bool hash, uint64_t n, uint32_t G,
               uint32_t shift, uint32_t nb, uint64_t pmask, uint32_t *hist, uint32_t *dtot, bool small,
               hipStream_t s, Timer *t) {
  if (t) t->begin(QF_PROF_SORT_HIST, s);
  if (hash)
    k_rs_hist<true, ND><<<G, NT, 0, s>>>(raw, n, G, shift, nb, pmask, hist);
  else
    k_rs_hist<false, ND><<<G, NT, 0, s>>>(in, n, G, shift, nb, 0, hist);
  if (t) t->end(QF_PROF_SORT_HIST, s);
  if (t) t->begin(QF_PROF_SORT_SCAN, s);
  k_rs_offsets<<<ND, NT, 0, s>>>(hist, G, dtot);
  if (t) t->end(QF_PROF_SORT_SCAN, s);
  if (t) t->begin(QF_PROF_SORT_SCATTER, s);
  if (hash && small)
    k_rs_scatter<true, 2048, ND><<<G, NT, 0, s>>>(raw, out, n, G, shift, nb, pmask, hist, dtot);
  else if (hash)
    k_rs_scatter<true, 4096, ND><<<G, NT, 0, s>>>(raw, out, n, G, shift, nb, pmask, hist, dtot);
  else if (small)
    k_rs_scatter<false, 2048, ND><<<G, NT, 0, s>>>(in, out, n, G, shift, nb, 0, hist, dtot);
  else
    k_rs_scatter<false, 4096, ND><<<G, NT, 0, s>>>(in, out, n, G, shift, nb, 0, hist, dtot);
  if (t) t->end(QF_PROF_SORT_SCATTER, s);
}

hipError_t launch_sort(uint64_t *a, uint64_t *b, uint64_t n, uint32_t bits, uint32_t *hist,
                       uint64_t **result, hipStream_t s, const Pipe &pp, const uint64_t *raw, uint64_t pmask) {
  Timer *t = pp.timer;
  const uint32_t G = sort_groups(n, pp.tune.sort_chunk);
  const bool small = pp.tune.sort_tile == 2048;
  // as few passes as digits of up to RADIX_BITS bits allow, the bits spread
  // evenly over them (36 bits: one 8-bit and four 7-bit passes; each bit of
  // a digit costs a wave ballot per key round of the scatter)
  const uint32_t npass = bits == 0 ? 0 : (bits + RADIX_BITS - 1) / RADIX_BITS;
  const uint32_t db = npass ? (bits + npass - 1) / npass : 0;
  // the count buffer: RADIX_MAX digit totals, then the G x RADIX_MAX histogram
  uint32_t *dtot = hist;
  hist += RADIX_MAX;
  uint64_t *in = a, *out = b;
  for (uint32_t p = 0; p < npass; ++p) {
    const uint32_t shift = db * p;
    const uint32_t nb = bits - shift < db ? bits - shift : db;
    // with raw keys the first pass hashes them itself (its output goes to b)
    const bool hash = raw && p == 0;
    sort_pass<RADIX_MAX>(in, out, raw, hash, n, G, shift, nb, pmask, hist, dtot, small, s, t);
    uint64_t *tmp = in;
    in = out;
    out = tmp;
  }
  *result = in;
  return hipGetLastError();
}

hipError_t launch_small_prep(const uint64_t *in, uint64_t n, uint32_t bits, uint64_t pmask, bool hash,
                             uint64_t *ufp, uint64_t *ucnt, uint64_t *state, hipStream_t s, Timer *t) {
  if (t) t->begin(QF_PROF_SORT_SCATTER, s);
  if (hash)
    k_small_prep<true><<<1, NT, 0, s>>>(in, static_cast<uint32_t>(n), bits, pmask, ufp, ucnt, state);
  else
    k_small_prep<false><<<1, NT, 0, s>>>(in, static_cast<uint32_t>(n), bits, pmask, ufp, ucnt, state);
  if (t) t->end(QF_PROF_SORT_SCATTER, s);
  return hipGetLastError();
}

hipError_t launch_rle(const uint64_t *sorted, uint64_t n, uint64_t *scratch_start,
                      uint64_t *ufp, uint64_t *ucnt, uint32_t *tile_counts, uint64_t *state,
                      hipStream_t s, const Pipe &pp) {
  Timer *t = pp.timer;
  const uint32_t G = sort_groups(n, pp.tune.sort_chunk);
  if (t) t->begin(QF_PROF_REDUCE, s);
  k_rle_count<<<G, NT, 0, s>>>(sorted, n, G, tile_counts);
  k_scan_u32<<<1, 1024, 0, s>>>(tile_counts, G, state + ST_NUNIQ);
  k_rle_write<<<G, NT, 0, s>>>(sorted, n, G, tile_counts, ufp, scratch_start);
  k_rle_counts<<<blocks_for(n), NT, 0, s>>>(scratch_start, n, state, ucnt);
  if (t) t->end(QF_PROF_REDUCE, s);
  return hipGetLastError();
}

hipError_t launch_bounds(const uint64_t *ufp, Pipe &p, hipStream_t s) {
  const uint32_t nthreads = p.G + 1;
  if (p.timer) p.timer->begin(QF_PROF_BOUNDS, s);
  k_bounds<<<(nthreads + NT - 1) / NT, NT, 0, s>>>(ufp, p.pst, p.G, p.RL + p.r, p.rb);
  if (p.timer) p.timer->end(QF_PROF_BOUNDS, s);
  return hipGetLastError();
}

}  // namespace qf
