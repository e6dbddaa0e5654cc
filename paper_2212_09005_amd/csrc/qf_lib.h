// qf_lib.h -- host-side state of a filter and of a filter set, and the kernel
// launchers the C ABI uses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace qf {
// Optional launch timer: begin/end record events on the launch stream.
struct Timer {
  virtual void begin(int kind, hipStream_t s) = 0;
  virtual void end(int kind, hipStream_t s) = 0;
  virtual ~Timer() {}
};

// Launch parameters of a pipeline.  They change how the work is cut into
// work-groups, never the results (the table is canonical).
struct Tune {
  uint32_t region_log2 = 0;   // slots per merge region, log2 (0: the largest the LDS holds)
  uint32_t sort_tile = 4096;  // keys a sort work-group orders in LDS per step (2048 or 4096)
  uint32_t sort_chunk = 4096; // fewest keys per sort work-group (power of two, 2^12..2^16)
  uint32_t lookup_kpl = 1;    // keys per lane of a lookup launch (1, 2 or 4)
};

// One filter as the kernels see it (an array of these lives in device memory
// for every pipeline; a single filter's pipeline has one).
struct FDesc {
  void *blk[2];       // the two table copies (blocks, offsets inside)
  uint64_t *state;    // ST_WORDS device words of the filter
  int64_t N, P, nblocks;
  uint32_t q, r, rlog, nregions, nqregions;
  uint32_t rbase;     // first region of this filter in its pipeline's region numbering
};

// The machinery of bulk updates over nf filters with the same r: regions of
// all filters are numbered 0..G-1 (filter f owns [rbase_f, rbase_f +
// nregions_f)); keys are grouped by the composite key
//   (global region << (RL + r)) | fingerprint bits inside the region,
// RL = the largest region log2.  For one filter the composite key is the
// fingerprint itself.
struct Pipe {
  uint32_t nf = 0, G = 0, RL = 0, r = 0;
  uint32_t fin_slices = 1;    // work-groups per filter of the merge's finish (most regions / FIN_REG)
  uint32_t gbits = 0;         // bits of a global region index
  FDesc *d_desc = nullptr;    // nf
  FDesc one;                  // host copy of the descriptor when nf == 1
  uint32_t *d_rmap = nullptr; // G: global region -> filter
  uint64_t *rb = nullptr;     // G + 1 region bounds into the reduced batch
  uint64_t *tags = nullptr;   // 3 G look-back words, then
  uint64_t *rstat = nullptr;  // 4 G per-region merge statistics, then
  int64_t *cb = nullptr;      // G old carries (region boundaries)
  uint64_t *pst = nullptr;    // ST_WORDS pipeline words (unique count, launch epoch)
  int64_t *d_err = nullptr;   // nf: per-filter deferred errors gathered by qf_set_errors
  // a launch restricted to some filters: their indexes and regions
  uint32_t *d_afil = nullptr, *d_areg = nullptr;  // capacity nf, G
  uint32_t nafil = 0, nareg = 0;                  // 0: all filters
  std::vector<uint32_t> h_rbase, h_nreg, h_afil, h_areg;  // host copies
  // pinned host staging of those lists, PIN_RING buffers used in turn; a
  // buffer is rewritten only after the copy that last read it has run (its
  // event), so a call does not wait for the stream's earlier work (a copy
  // from pageable memory would); with a server's two update calls per set
  // and round, the buffer reused was read two rounds before
  static constexpr int PIN_RING = 4;
  uint32_t *h_pin[PIN_RING] = {};
  uint64_t h_pin_cap[PIN_RING] = {};  // words
  hipEvent_t pin_ev[PIN_RING] = {};
  int pin_i = 0;
  Tune tune;
  int device = 0;
  // grow-only scratch, capacity in keys
  uint64_t cap = 0;
  uint64_t *bufA = nullptr, *bufB = nullptr, *bufC = nullptr, *bufD = nullptr;
  uint64_t *bufE = nullptr;   // 32 bytes per key: the merge's per-entry scratch
  uint32_t *hist = nullptr;   // radix digit totals and histograms / tile counts (sized with the scratch)
  uint64_t hist_words = 0;
  uint64_t device_bytes = 0;
  uint64_t batches = 0;
  Timer *timer = nullptr;     // non-null while profiling is enabled
};
}  // namespace qf

struct qf_filter {
  uint32_t q, r;
  uint64_t N, E, P, nblocks;
  uint32_t block_bytes;     // 128 (r = 8) or 160 (r = 16)
  int device;
  void *blk[2];             // two table copies (blocks, offsets inside)
  uint64_t *state;          // qf::ST_WORDS device words
  uint64_t table_device_bytes;
  uint32_t *plocks;         // point updates: one lock word per 4096 slots (zero = free)
  uint32_t vbits;           // value association: value bits at the low end of each remainder (0: none)
  qf::Pipe pipe;            // the single-filter update pipeline
};

struct qf_set {
  uint32_t nf;
  qf_filter **fs;           // host copies of the handles (not owned)
  qf::Pipe pipe;
  uint32_t **d_plocks = nullptr;  // device: each filter's point-update lock words
};

namespace qf {

// one table's device bytes
uint64_t table_bytes(uint64_t nblocks, uint32_t r);

hipError_t launch_hash(const uint64_t *keys, uint64_t n, uint64_t pmask, uint64_t *fp,
                       hipStream_t s, Timer *t);
// value association: fp[i] = (hash(keys[i]) & kmask) << vbits | (values[i] & (2^vbits - 1))
hipError_t launch_kv_compose(const uint64_t *keys, const uint64_t *values, uint64_t n, uint64_t kmask,
                             uint32_t vbits, uint64_t *fp, hipStream_t s, Timer *t);
// value association lookups: smallest value (or ~0) and number of distinct values per key
hipError_t launch_kv_lookup(qf_filter *f, const uint64_t *keys, uint64_t n, uint64_t *value, uint32_t *nvalues,
                            hipStream_t s);
// composite keys of a filter set: key i belongs to filter fid[i]
hipError_t launch_hash_multi(const uint64_t *keys, const uint32_t *fid, uint64_t n, const Pipe &p,
                             uint64_t *out, hipStream_t s, Timer *t);
// LSD radix sort of n keys over the low `bits` bits; returns the buffer that
// holds the result (a or b).  With raw != nullptr the input is raw keys
// (a is not read): the first pass sorts mix64(raw[i]) & pmask.
hipError_t launch_sort(uint64_t *a, uint64_t *b, uint64_t n, uint32_t bits, uint32_t *hist,
                       uint64_t **result, hipStream_t s, const Pipe &p, const uint64_t *raw = nullptr,
                       uint64_t pmask = 0);
// batches of at most SMALL_KEYS keys: sort and run-length reduction in one
// work-group (keys hashed on load when hash is set): ufp/ucnt, count in
// state[ST_NUNIQ]
constexpr uint32_t SMALL_KEYS = 4096;
hipError_t launch_small_prep(const uint64_t *in, uint64_t n, uint32_t bits, uint64_t pmask, bool hash,
                             uint64_t *ufp, uint64_t *ucnt, uint64_t *state, hipStream_t s, Timer *t);
// run-length reduction of the sorted keys: ufp/ucnt, count in state[ST_NUNIQ]
hipError_t launch_rle(const uint64_t *sorted, uint64_t n, uint64_t *scratch_start,
                      uint64_t *ufp, uint64_t *ucnt, uint32_t *tile_counts, uint64_t *state,
                      hipStream_t s, const Pipe &p);
// region bounds of the pipeline's G regions
hipError_t launch_bounds(const uint64_t *ufp, Pipe &p, hipStream_t s);
// old carries, per-filter batch flags, tag reset on epoch wrap, region merge
// into the other table copies, finish (statistics, flip or deferred error).
// not_found: nullptr or one word per filter of the pipeline.
hipError_t launch_merge(Pipe &p, const uint64_t *ufp, const uint64_t *ucnt, int del,
                        uint64_t *not_found, hipStream_t s);
hipError_t launch_lookup(qf_filter *f, const uint64_t *keys, uint64_t n, uint8_t *out8,
                         uint64_t *out64, hipStream_t s);
hipError_t launch_lookup_multi(const Pipe &p, const uint64_t *keys, const uint32_t *fid, uint64_t n,
                               uint8_t *out8, uint64_t *out64, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
// copy each filter's deferred error word to err[f] and clear it
hipError_t launch_take_errors(const Pipe &p, int64_t *err, hipStream_t s);
// tail[i] = used slots past the last quotient of the pipeline's filter i
// (they form one stretch from N), on the filter's current copy
hipError_t launch_take_tails(const Pipe &p, int64_t *tail, hipStream_t s);
hipError_t launch_export(qf_filter *f, uint64_t *occ, uint64_t *rend, uint16_t *slots,
                         uint32_t *offs, hipStream_t s);
hipError_t launch_import(qf_filter *f, const uint64_t *occ, const uint64_t *rend,
                         const uint16_t *slots, const uint32_t *offs, hipStream_t s);

// sort tiling: G work-groups each own a contiguous chunk of at least
// `chunk` keys (at most SORT_MAX_GROUPS groups; chunks are never below
// SORT_MIN_CHUNK keys)
constexpr uint32_t SORT_MAX_GROUPS = 16384;
constexpr uint32_t SORT_MIN_CHUNK = 4096;
uint32_t sort_groups(uint64_t n, uint32_t chunk);
// words of the sort's count buffer for batches of up to cap keys: 256 digit
// totals, then 256 counts per work-group (also the reduction's per-group counts)
uint64_t sort_count_words(uint64_t cap);
int max_region_log2(uint32_t r);
// point updates (one lane per key, in place): words of the lock array of a
// table of P slots, and the launch (status, not_found may be null)
uint64_t point_lock_words(uint64_t P);
// lock regions of a point update on a table of P slots
uint64_t point_regions(uint64_t P);
hipError_t launch_point(qf_filter *f, const uint64_t *keys, uint64_t n, int del, int32_t *status,
                        uint64_t *not_found, hipStream_t s);
// point updates over a set's filters, key i to filter fid[i] (locks: the
// set's d_plocks); errors go to each filter's error word
hipError_t launch_point_multi(const Pipe &p, uint32_t *const *locks, const uint32_t *fid, const uint64_t *keys,
                              uint64_t n, int del, hipStream_t s);
// records code as the calling thread's last error (qf_last_error) and returns it
int record_error(int code);
// enumeration (qf_enum.hip): scratch bytes for a filter, and the two passes:
// write = false counts entries per quotient block and scans them (the total
// goes to the scratch's total word, read by enum_total); write = true writes
// the sorted <fingerprint, count> pairs to fp / cnt
uint64_t enum_scratch_bytes(const qf_filter *f);
hipError_t launch_enum(qf_filter *f, void *scratch, uint64_t *fp, uint64_t *cnt, bool write, hipStream_t s);
// device address of the scratch words [total, big count] inside the scratch
inline uint64_t *enum_words(const qf_filter *f, void *scratch) {
  const uint64_t nqb = f->N / 64, nseg = (nqb + 4095) / 4096;
  return reinterpret_cast<uint64_t *>(static_cast<uint8_t *>(scratch) + ((nqb * 4 + 7) / 8) * 8) + nseg;
}
// the merge's finish: work-group size and regions per work-group
constexpr uint32_t FIN_NT = 256;
constexpr uint32_t FIN_REG = 2048;

}  // namespace qf
