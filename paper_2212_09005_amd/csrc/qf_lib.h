// qf_lib.h -- host-side state of a filter and the kernel launchers the C ABI uses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qf {
// Optional launch timer: begin/end record events on the launch stream.
struct Timer {
  virtual void begin(int kind, hipStream_t s) = 0;
  virtual void end(int kind, hipStream_t s) = 0;
  virtual ~Timer() {}
};
}  // namespace qf

struct qf_filter {
  uint32_t q, r, rlog;      // region = 2^rlog slots
  uint64_t N, E, P, nblocks;
  uint32_t nregions, nqregions;
  uint32_t block_bytes;     // 80 (r = 8) or 144 (r = 16)
  int device;
  void *blk[2];             // two table copies (blocks)
  uint32_t *off[2];         // and their offsets
  uint64_t *state;          // qf::ST_WORDS device words
  uint64_t *rb;             // nregions + 1 region bounds into the reduced batch
  uint64_t *tags;           // 3 * nregions look-back words, then
  uint64_t *rstat;          // 4 * nregions per-region merge statistics, then
  int64_t *cb;              // nqregions + 1 old carries at region boundaries
  uint32_t epoch;
  uint64_t batches;
  // grow-only scratch, capacity in keys
  uint64_t cap;
  uint64_t *bufA, *bufB, *bufC, *bufD;
  uint32_t *hist;           // radix histograms / tile counts
  uint64_t hist_words;
  uint64_t device_bytes;
  qf::Timer *timer;         // non-null while profiling is enabled
};

namespace qf {

// one table's device bytes
uint64_t table_bytes(uint64_t nblocks, uint32_t r);

hipError_t launch_hash(const uint64_t *keys, uint64_t n, uint64_t pmask, uint64_t *fp,
                       hipStream_t s, Timer *t);
// LSD radix sort of n keys over the low `bits` bits; returns the buffer that
// holds the result (a or b).
hipError_t launch_sort(uint64_t *a, uint64_t *b, uint64_t n, uint32_t bits, uint32_t *hist,
                       uint64_t **result, hipStream_t s, Timer *t);
// run-length reduction of the sorted fingerprints: ufp/ucnt, count in state
hipError_t launch_rle(const uint64_t *sorted, uint64_t n, uint64_t *scratch_start,
                      uint64_t *ufp, uint64_t *ucnt, uint32_t *tile_counts, uint64_t *state,
                      hipStream_t s, Timer *t);
hipError_t launch_bounds(const uint64_t *ufp, uint64_t *state, qf_filter *f, hipStream_t s);
hipError_t launch_merge(qf_filter *f, const uint64_t *ufp, const uint64_t *ucnt, int del,
                        uint64_t *not_found, hipStream_t s);
hipError_t launch_lookup(qf_filter *f, const uint64_t *keys, uint64_t n, uint8_t *out8,
                         uint64_t *out64, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_export(qf_filter *f, uint64_t *occ, uint64_t *rend, uint16_t *slots,
                         uint32_t *offs, hipStream_t s);
hipError_t launch_import(qf_filter *f, const uint64_t *occ, const uint64_t *rend,
                         const uint16_t *slots, const uint32_t *offs, hipStream_t s);

// sort tiling: G work-groups each own a contiguous chunk of the keys
uint32_t sort_groups(uint64_t n);

}  // namespace qf
