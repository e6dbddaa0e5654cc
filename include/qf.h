/*
 * qf.h -- C ABI of libqf.so, a counting quotient filter on one MI355X (gfx950).
 *
 * The filter is the bulk GPU counting quotient filter of McCoy, Hofmeyr,
 * Yelick and Pandey, "High-Performance Filters for GPUs" (PPoPP'23):
 *   - Sec. 1 (footnote): a counting filter stores a multiset; a count may
 *     over-estimate (fingerprint collisions) but never under-estimates.
 *   - Sec. 5.1: each key is hashed to a p = q + r bit fingerprint, split into
 *     a q-bit quotient (canonical slot) and an r-bit remainder; remainders of
 *     one quotient form a run, runs are stored in quotient order, shifted right
 *     as far as needed.
 *   - Sec. 5.3: a bulk insert hashes and sorts the batch, groups it by region
 *     and merges each region; remainders are sorted inside a run.
 *   - Sec. 5.4: duplicates in a batch are reduced to <item, count> first.
 *   - Sec. 6.2/6.4 and the API table of Sec. 6: bulk query, count and delete.
 * The hash (SplitMix64 finalizer), the fingerprint bits (low p bits), the
 * counter encoding, the 10*sqrt(2^q) extra slots after the last quotient and
 * the per-64-slot offsets are this library's readings of what the paper leaves
 * open; the result is one canonical table per multiset, which qf_export
 * returns.
 *
 * Conventions for every call below:
 *   - `d_*` pointers are device pointers (e.g. torch tensors' data_ptr());
 *     keys are any 64-bit values; the caller owns keys and outputs, which hold
 *     n elements and must not alias.  n == 0 is a no-op that returns QF_OK.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Calls are stream-ordered and asynchronous: they return after enqueueing.
 *   - Argument errors return at once with no side effects.  Errors found on
 *     the device (QF_ERR_FULL, QF_ERR_COUNT_OVERFLOW) make that batch a no-op
 *     (all or nothing: the table is left exactly as before the call) and are
 *     reported by the next qf_sync (or qf_export) on that filter.
 *   - A filter must not be used from two streams without ordering them.
 *   - The library owns the table (two device copies, written alternately) and
 *     a grow-only scratch area sized by the largest batch seen.
 */
#ifndef QF_H
#define QF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qf_filter qf_t;

/* Largest q a filter may have (2^30 quotients, about 2.7 GB per table copy
 * at r = 16): every size the library accepts is one the CPU checker can
 * build and compare bit for bit. */
#define QF_Q_MAX 30

enum {
  QF_OK = 0,
  QF_ERR_ARG = -1,            /* bad argument (nothing happened)              */
  QF_ERR_FULL = -2,           /* a run would end past the last slot           */
  QF_ERR_OOM = -3,            /* device allocation failed                     */
  QF_ERR_DEVICE = -4,         /* a HIP runtime call failed                    */
  QF_ERR_COUNT_OVERFLOW = -5, /* a count would exceed 2^64 - 1                */
  QF_ERR_STALLED = -6,        /* a merge region waited too long for the carry
                                 of the regions before it, or a point update
                                 failed to take its locks 2^20 times (safety
                                 bounds that should never trigger); not applied */
  QF_ERR_BUDGET = -7,         /* serving: a filter larger than the HBM budget */
  QF_ERR_LIMIT = -8           /* qf_insert_batch_noalloc: batch larger than
                                 QF_NOALLOC_MAX_KEYS (nothing happened)        */
};

/* Logical layout of a table, as host arrays (qf_export / qf_import).
 *   header       : q, r, N = 2^q, E (extra slots), P = N + E, used slots,
 *                  distinct fingerprints, total count (mod 2^64)
 *   occ_words    : N/64 words; bit x%64 of word x/64 = quotient x has a run
 *   runend_words : P/64 words; bit j%64 of word j/64 = slot j ends a run
 *   slots        : P values (remainders and counter digits), 0 outside runs
 *   offsets      : P/64 values; for block b starting at slot i = 64b, the
 *                  distance from i to the end of the run of the last occupied
 *                  quotient <= i, or 0 when that end lies before i / no such
 *                  quotient exists.
 * The caller allocates the four arrays with the sizes above. */
typedef struct qf_layout {
  uint64_t header[8];
  uint64_t *occ_words;
  uint64_t *runend_words;
  uint16_t *slots;
  uint32_t *offsets;
} qf_layout_t;

/* Sec. 5.1: a table of 2^q quotients with r-bit remainders.  q in [6, QF_Q_MAX],
 * r in {8, 16}.  Returns NULL on error (see qf_last_error()).  The new filter
 * is empty and lives on the current HIP device. */
qf_t *qf_create(uint32_t q, uint32_t r);

/* Frees the filter and its device memory (waits for its pending work).
 * NULL is ignored. */
void qf_destroy(qf_t *f);

/* Batch limits of the update calls (insert, delete, and their set and
 * value-association forms): at most 2^32 - 1 keys per batch (a larger n
 * returns QF_ERR_ARG at once).  An update sorts its batch in the filter's
 * scratch area, 64 bytes per key, grown on demand and kept (QF_ERR_OOM when
 * the device cannot hold it): a one-batch insert of 9.66e8 keys needs about
 * 62 GB beside the two table copies.  qf_reserve grows it ahead of time. */

/* Sec. 5.3-5.4: insert one instance of each key (duplicates are counted).
 * d_keys: device, n uint64.  All or nothing; QF_ERR_FULL / COUNT_OVERFLOW are
 * deferred to qf_sync. */
int qf_insert_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * insert as qf_insert_batch, with the same result, but the batch scratch is a
 * fixed device array of the library (about 32 MiB, one per GPU, held until
 * the process ends) instead of the filter's grow-only area, and the call
 * allocates nothing.  d_keys: device, n uint64 with n <= QF_NOALLOC_MAX_KEYS;
 * a larger n returns QF_ERR_LIMIT at once (nothing happens).  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (from two
 * streams, or two host threads, without ordering) race and corrupt each
 * other.  Errors and all-or-nothing behaviour as qf_insert_batch.  Kernel
 * timing (qf_profile_enable) does not cover these calls. */
#define QF_NOALLOC_MAX_KEYS (1ull << 19)
int qf_insert_batch_noalloc(qf_t *f, const uint64_t *d_keys, uint64_t n, void *stream);

/* Sec. 6.2: d_out[i] = 1 if the fingerprint of d_keys[i] is stored, else 0.
 * d_keys: device, n uint64; d_out: device, n uint8. */
int qf_query_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint8_t *d_out, void *stream);

/* Count (API table of Sec. 6): d_out[i] = stored multiplicity of the
 * fingerprint of d_keys[i] (>= the true count of the key, Sec. 1 footnote).
 * d_keys: device, n uint64; d_out: device, n uint64. */
int qf_count_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint64_t *d_out, void *stream);

/* Sec. 6.4: for a fingerprint present k times in the batch, remove
 * min(k, stored count) instances; the shortfall summed over the batch is
 * ADDED to *d_not_found (device, one uint64; may be NULL). */
int qf_delete_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint64_t *d_not_found,
                    void *stream);

/* Waits for the filter's work on `stream`; returns the first deferred device
 * error since the previous qf_sync (and clears it), or QF_OK. */
int qf_sync(qf_t *f, void *stream);

/* Copies the current table to the caller's host arrays (synchronous; also
 * returns and clears a pending deferred error, like qf_sync). */
int qf_export(qf_t *f, qf_layout_t *out, void *stream);

/* Replaces the table by the given logical layout (header q, r must match the
 * filter; the layout must be a valid canonical table).  Synchronous. */
int qf_import(qf_t *f, const qf_layout_t *in, void *stream);

/* Error code of the last failed call in this thread. */
int qf_last_error(void);

/* Grows the filter's scratch area (grow-only, 64 bytes per key) to hold
 * batches of n keys, so that later calls with batches up to n allocate
 * nothing.  May wait for `stream` when the area grows. */
int qf_reserve(qf_t *f, uint64_t n, void *stream);

/* Device bytes of one table copy of a (q, r) filter: 64-slot blocks of 128
 * bytes (r = 8) or 160 bytes (r = 16), each holding its occupied bits, run-end
 * bits, offset and slots. */
uint64_t qf_table_bytes(uint32_t q, uint32_t r);

/* info[0..7] = q, r, N, E, P, region slots, device bytes held, batches run. */
int qf_info(const qf_t *f, uint64_t *info);

/* Kernel timing (for benchmarks): kinds is a bit mask of (1 << QF_PROF_*)
 * values (QF_PROF_ALL: every kind; 0 disables timing and drops what was not
 * read).  While enabled, every kernel launch of this filter of a selected
 * kind is bracketed by two HIP events recorded on the launch stream (each
 * pair delays the stream by a few microseconds, so time only the kinds of
 * interest).  Calling it again while enabled changes the selection.
 * qf_profile_read waits for the recorded events, returns per kind the summed
 * milliseconds ms[k] and the number of launches n[k] since the last read
 * (arrays of QF_PROF_KINDS entries, host memory) and clears them.  The sort
 * kinds count each radix pass as one launch; QF_PROF_REDUCE covers the four
 * small kernels of the duplicate reduction; QF_PROF_MERGE covers the merge
 * and its two small companions (old carries before, statistics after). */
enum {
  QF_PROF_HASH = 0,
  QF_PROF_SORT_HIST = 1,
  QF_PROF_SORT_SCAN = 2,
  QF_PROF_SORT_SCATTER = 3,
  QF_PROF_REDUCE = 4,
  QF_PROF_BOUNDS = 5,
  QF_PROF_MERGE = 6,
  QF_PROF_LOOKUP = 7,
  QF_PROF_KINDS = 8,
  QF_PROF_ALL = (1 << QF_PROF_KINDS) - 1
};
int qf_profile_enable(qf_t *f, int kinds);
int qf_profile_read(qf_t *f, double *ms, uint64_t *n);

/* ---- enumeration, union, difference, re-layout --------------------------------
 * The paper lists enumeration, merging and resizing among the counting quotient
 * filter's features (Sec. 1, 2) without describing them.  A table stores every
 * p-bit fingerprint whole (quotient = high q bits, remainder = low r bits), so
 * these are exact operations on the stored fingerprint multiset.  All are
 * synchronous (they wait for `stream`) and allocate temporary device memory. */

/* out[0..2] = used slots, distinct fingerprints, total count (mod 2^64) of the
 * current table (host array). */
int qf_stats(qf_t *f, uint64_t *out, void *stream);

/* The stored multiset as <fingerprint, count> pairs sorted by fingerprint:
 * d_fp / d_cnt are device arrays of cap uint64 each; *n (host) gets the number
 * of pairs (the distinct fingerprints).  cap == 0 only sets *n (the arrays
 * may be NULL); 0 < cap < *n returns QF_ERR_ARG and writes nothing. */
int qf_enumerate(qf_t *f, uint64_t *d_fp, uint64_t *d_cnt, uint64_t cap, uint64_t *n, void *stream);

/* Union (subtract = 0: dst gets the multiset sum) or saturating difference
 * (subtract = 1: for each fingerprint, min(count in dst, count in src) copies
 * are removed from dst and the shortfall is ADDED to *d_not_found, device, one
 * uint64, may be NULL) of two filters whose fingerprints have the same length
 * (dst.q + dst.r == src.q + src.r, QF_ERR_ARG otherwise); src is unchanged
 * (src == dst doubles or empties the counts).  The source's pairs go through
 * dst's bulk merge as an already reduced batch: all or nothing, errors
 * (QF_ERR_FULL, QF_ERR_COUNT_OVERFLOW) deferred to qf_sync(dst).  A count of
 * 2^32 or more for one fingerprint of src returns QF_ERR_ARG. */
int qf_merge_into(qf_t *dst, qf_t *src, int subtract, uint64_t *d_not_found, void *stream);

/* A new filter with q quotient bits and r-bit remainders (q + r equal to the
 * source's, r in {8, 16}) holding the same fingerprint multiset as src: for
 * example 2^20 quotients with 16-bit remainders into 2^28 quotients with
 * 8-bit remainders, or back.  NULL on error (qf_last_error; QF_ERR_FULL when
 * the multiset does not fit the new table). */
qf_t *qf_resize(qf_t *src, uint32_t q, uint32_t r, void *stream);

/* ---- value association --------------------------------------------------
 * The paper names value association among the CQF's features (Sec. 1, 2)
 * without describing it.  Here a filter made by qf_create_kv keeps a small
 * value with every key: the slot's r bits hold the key's remainder of
 * r - vbits bits followed by vbits value bits, so the table stores the
 * multiset of <key fingerprint (q + r - vbits bits), value> pairs, one entry
 * per distinct pair with its count, and stays the canonical table of that
 * multiset (qf_export).  A key may carry several values; the false-positive
 * rate is that of a plain filter with r - vbits remainder bits.  On such a
 * filter the plain insert / delete / query / count / point calls and filter
 * sets return QF_ERR_ARG; qf_stats, qf_enumerate (pairs as composite
 * fingerprints), qf_merge_into (both with the same vbits) and qf_resize
 * (which keeps vbits; r must exceed it) work as for plain filters. */

/* A value-associating filter: 1 <= vbits < r, r in {8, 16}, q as qf_create. */
qf_t *qf_create_kv(uint32_t q, uint32_t r, uint32_t vbits);

/* Insert / delete the pairs <d_keys[i], d_values[i] mod 2^vbits> as a batch
 * (all or nothing, errors deferred to qf_sync, as qf_insert_batch /
 * qf_delete_batch; not-found pairs ADDED to *d_not_found, may be NULL). */
int qf_kv_insert_batch(qf_t *f, const uint64_t *d_keys, const uint64_t *d_values, uint64_t n, void *stream);
int qf_kv_delete_batch(qf_t *f, const uint64_t *d_keys, const uint64_t *d_values, uint64_t n,
                       uint64_t *d_not_found, void *stream);

/* d_value[i] = the smallest value stored with key i's fingerprint, or
 * 2^64 - 1 when there is none; d_nvalues[i] (uint32, may be NULL) = how many
 * distinct values are stored with it. */
int qf_kv_lookup_batch(qf_t *f, const uint64_t *d_keys, uint64_t n, uint64_t *d_value, uint32_t *d_nvalues,
                       void *stream);

/* ---- point updates (Sec. 5.2; the point rows of the API table of Sec. 6) --
 * One lane per key, in place on the current table: the keys of one call are
 * applied concurrently and in no set order, each under region locks (4096
 * slots per lock; a lane never waits while holding one).  Each applied update
 * has exactly the effect the same key has in a bulk call, so afterwards the
 * table is the canonical table of the resulting multiset.  Unlike a bulk
 * call, a point call is NOT all or nothing: each key succeeds or fails on its
 * own, and when the table is close to full which keys fail depends on the
 * order in which they land.
 *   d_status    : device, n int32 per key, may be NULL: 0 = applied,
 *                 1 = (delete) fingerprint not stored, nothing changed,
 *                 QF_ERR_FULL / QF_ERR_COUNT_OVERFLOW / QF_ERR_STALLED = not
 *                 applied.  The first such error is also reported by the
 *                 next qf_sync.
 *   d_not_found : as for qf_delete_batch (ADDED to; may be NULL).
 * Point lookups are qf_query_batch and qf_count_batch, which look every key
 * up on its own (no sort); a lookup must not run at the same time as point
 * updates of the same filter (stream order guarantees this). */
int qf_point_insert(qf_t *f, const uint64_t *d_keys, uint64_t n, int32_t *d_status, void *stream);
int qf_point_delete(qf_t *f, const uint64_t *d_keys, uint64_t n, int32_t *d_status, uint64_t *d_not_found,
                    void *stream);

/* ---- filter sets: many filters, one pipeline of launches ------------------
 * A set groups nf existing filters with the same r (sizes may differ) so that
 * one batch of keys, each tagged with the index of its filter in the set,
 * is hashed, sorted, reduced and merged into all of them by one sequence of
 * launches (one merge launch covers every region of every filter), and one
 * lookup launch answers a mixed query batch.  Per filter the effect is that
 * of the single-filter call on the keys tagged with it, in batch order
 * (Sec. 5.3-5.4 and 6.2 per filter; grouping many filters in one launch is
 * this library's design for workloads of thousands of small filters, where
 * a loop of per-filter calls is bound by launch count).
 * Conventions: d_fid (device, n uint32) holds each key's filter index in
 * [0, nf); an index out of range drops that key (a lookup returns 0 for it)
 * and makes qf_set_sync return QF_ERR_ARG.  Errors of a filter (FULL,
 * COUNT_OVERFLOW) are all-or-nothing for that filter's share of the batch
 * and surface at qf_set_sync (or qf_sync of that filter).  The set does not
 * own its filters; they must outlive it, and per-filter calls must be stream
 * ordered with set calls.  qf_set_create is synchronous and fails with
 * QF_ERR_ARG for nf == 0, a NULL filter, the same filter listed twice, mixed
 * r, or more than 2^31 regions (NULL and repeated handles are found before
 * any handle is read). */
typedef struct qf_set qf_set_t;
qf_set_t *qf_set_create(qf_t *const *filters, uint32_t nf);
void qf_set_destroy(qf_set_t *s); /* NULL-safe; waits for the device */
int qf_set_insert_batch(qf_set_t *s, const uint32_t *d_fid, const uint64_t *d_keys, uint64_t n,
                        void *stream);
/* d_not_found: device, nf uint64 (the shortfall of filter i is ADDED to
 * d_not_found[i]), or NULL. */
int qf_set_delete_batch(qf_set_t *s, const uint32_t *d_fid, const uint64_t *d_keys, uint64_t n,
                        uint64_t *d_not_found, void *stream);
/* The same, restricted to the filters listed in h_filters (host, n_filters
 * distinct indexes in ascending order): only their regions are merged, so a
 * batch that touches few filters of a large set costs in proportion to
 * those filters.  Every key's filter must be listed; keys of unlisted
 * filters are dropped. */
int qf_set_insert_some(qf_set_t *s, const uint32_t *h_filters, uint32_t n_filters, const uint32_t *d_fid,
                       const uint64_t *d_keys, uint64_t n, void *stream);
int qf_set_delete_some(qf_set_t *s, const uint32_t *h_filters, uint32_t n_filters, const uint32_t *d_fid,
                       const uint64_t *d_keys, uint64_t n, uint64_t *d_not_found, void *stream);
int qf_set_query_batch(qf_set_t *s, const uint32_t *d_fid, const uint64_t *d_keys, uint64_t n,
                       uint8_t *d_out, void *stream);
int qf_set_count_batch(qf_set_t *s, const uint32_t *d_fid, const uint64_t *d_keys, uint64_t n,
                       uint64_t *d_out, void *stream);
/* Waits for `stream`; returns (and clears) the set's own deferred error, else
 * the first deferred error of its filters (all of them are cleared). */
int qf_set_sync(qf_set_t *s, void *stream);
/* Waits for `stream`; writes each filter's deferred error (0 = none) to
 * codes[0..nf) (host) and clears them; returns how many are nonzero. */
int qf_set_errors(qf_set_t *s, int32_t *codes, void *stream);
/* qf_reserve for the set's pipeline. */
int qf_set_reserve(qf_set_t *s, uint64_t n, void *stream);
/* info[0..7] = nf, r, total regions, largest region log2, device bytes held by
 * the set's pipeline, batches run, bits of the composite sort key, 0. */
int qf_set_info(const qf_set_t *s, uint64_t *info);
/* Kernel timing of the set's pipeline, as qf_profile_enable / _read. */
int qf_set_profile_enable(qf_set_t *s, int kinds);
int qf_set_profile_read(qf_set_t *s, double *ms, uint64_t *n);

/* ---- launch parameters ---------------------------------------------------
 * How a pipeline (a filter's own, or a set's) cuts its work into
 * work-groups.  They change speed, never results: the table is canonical.
 * 0 in a field selects the default.
 *   region_log2          slots per merge region (one work-group's share of
 *                        the table), log2 in [6, 13]; capped at the largest
 *                        region the merge's LDS holds (2^13 slots for r = 8,
 *                        2^12 for r = 16) and at q.  Default: that cap.
 *   sort_tile            keys a sort work-group orders in LDS per step:
 *                        2048 or 4096 (default).
 *   sort_chunk           fewest keys per sort work-group, a power of two in
 *                        [4096 (default), 65536]; sets the sort's grid.
 *   lookup_keys_per_lane keys one lane of a query / count launch looks up:
 *                        1 (default), 2 or 4; sets the lookup grid.
 * qf_tune / qf_set_tune check the fields (QF_ERR_ARG, nothing changed),
 * wait for the device, rebuild the pipeline (its scratch capacity is kept)
 * and switch its profiling off.  The get calls report the parameters in
 * effect, region_log2 as the largest region log2 of the pipeline. */
typedef struct qf_tuning {
  uint32_t region_log2;
  uint32_t sort_tile;
  uint32_t sort_chunk;
  uint32_t lookup_keys_per_lane;
} qf_tuning_t;
int qf_tune(qf_t *f, const qf_tuning_t *t);
int qf_get_tuning(const qf_t *f, qf_tuning_t *t);
int qf_set_tune(qf_set_t *s, const qf_tuning_t *t);
int qf_set_get_tuning(const qf_set_t *s, qf_tuning_t *t);

/* Autotuner for filter sets: picks launch parameters for a set of nf
 * filters with quotient bits qs[0..nf) (host) and remainder bits r that is
 * filled to `load` (fraction of 2^q per filter) by one set insert batch and
 * then answers set query batches of n_query keys (spread over the filters in
 * proportion to 2^q, half of them present).  It builds private filters of a
 * sample of those sizes (at most 2^26 quotients in total, every k-th
 * filter), times candidate parameters on them on the device with synthetic
 * keys (region size first, then the sort's tile and chunk, then keys per
 * lane for the lookups; each candidate's best of two runs) and writes the
 * fastest to *best.  ms (host, 2 doubles, may be NULL) receives the insert and
 * query milliseconds of the chosen parameters on the sample.  Synchronous;
 * it uses the null stream and frees what it allocated.  Results are cached
 * per process by (qs, r, load, n_query). */
int qf_autotune_set(const uint32_t *qs, uint32_t nf, uint32_t r, double load, uint64_t n_query,
                    qf_tuning_t *best, double *ms);

/* ---- stream capture ------------------------------------------------------
 * The batch calls (qf_insert_batch, qf_delete_batch, qf_query_batch,
 * qf_count_batch and the qf_set_ forms without _some) can be recorded into
 * a graph and replayed: qf_graph_begin starts capturing `stream` (not NULL;
 * thread-local capture mode), the calls enqueue as usual, qf_graph_end ends
 * the capture and instantiates it (NULL on error, see qf_last_error), and
 * each qf_graph_launch replays every recorded launch on `stream` against
 * the filters' current contents, reading the key buffers and writing the
 * outputs given at capture time.  Everything a batch keeps between launches
 * lives on the device, so replays behave like the same calls made again.
 * Before capturing, reserve scratch for the largest batch (qf_reserve /
 * qf_set_reserve) and leave profiling off: under capture a call that would
 * have to allocate, copy from host memory or time itself fails with
 * QF_ERR_ARG.  qf_sync, qf_export, qf_import, the _some calls, the tune
 * calls and the serving calls must not be used on a stream being captured.
 * Deferred device errors of replayed batches surface at qf_sync /
 * qf_set_sync as for direct calls; a delete's not-found counts are added
 * to the captured d_not_found on every replay. */
typedef struct qf_graph qf_graph_t;
int qf_graph_begin(void *stream);
qf_graph_t *qf_graph_end(void *stream);
int qf_graph_launch(qf_graph_t *g, void *stream);
void qf_graph_destroy(qf_graph_t *g); /* NULL-safe */

/* ---- serving: device-resident filters, requests batched as they arrive ----
 * A server keeps filters in HBM and answers requests submitted from any host
 * thread.  A loop thread batches whatever is waiting into rounds: per filter,
 * the leading run of its waiting requests with one operation; all filters'
 * shares of one operation (and r) run as one filter-set batch, so requests
 * that arrive while others are on the device join the next round, and the
 * next round is assembled and launched while the current one runs.  A
 * filter's updates of a round with no more keys than it has 4096-slot lock
 * regions, and no way to fill the slots past its last quotient (3 per key
 * against a bound of those in use), are applied in place by point updates,
 * at a cost that follows the keys; the others go through the bulk merge,
 * which rewrites the filter.  Both give the same table.  Per
 * filter the effects and answers are those of executing its requests one by
 * one in submission order (linearizable in admission order); requests on
 * different filters are independent.  Filters are admitted in open order
 * while the device bytes they need fit the budget (their requests wait until
 * then); a close frees its bytes once the filter's earlier requests are done.
 * Keys are host arrays copied at submission; a query (count) writes n bytes
 * (n uint64) to h_out before its completion is reported by qfs_poll.  Delete
 * shortfalls are not reported per request.  A request's status is QF_OK or its
 * filter's deferred error for the round it ran in (QF_ERR_FULL: that filter's
 * updates of the round were not applied). */
typedef struct qf_server qfs_t;
enum { QFS_INSERT = 0, QFS_DELETE = 1, QFS_QUERY = 2, QFS_COUNT = 3 };
/* max_round_keys bounds the keys of one round and of one request; the two
 * pinned staging buffers and the batch scratch it implies count against the
 * budget.  NULL on error. */
qfs_t *qfs_create(uint64_t budget_bytes, uint64_t max_round_keys);
void qfs_destroy(qfs_t *s); /* drains the queue, stops the loop, frees all */
/* Returns the filter id (>= 0), QF_ERR_BUDGET if it can never fit, or
 * QF_ERR_ARG (q, r as for qf_create). */
int qfs_open(qfs_t *s, uint32_t q, uint32_t r);
int qfs_submit(qfs_t *s, int op, int id, const uint64_t *h_keys, uint64_t n, void *h_out, uint64_t tag);
/* Closes a filter after its earlier requests; its completion is reported with
 * `tag` like a request's.  Later submissions to it fail with QF_ERR_ARG. */
int qfs_close(qfs_t *s, int id, uint64_t tag);
/* Copies filter id's table, as its requests submitted before this call left
 * it, into the caller's host arrays (as qf_export; sized for the filter's q
 * and r, kept alive until the completion with `tag` is polled; its status is
 * qf_export's result).  Later requests of the filter wait for the copy. */
int qfs_export(qfs_t *s, int id, qf_layout_t *out, uint64_t tag);
/* Writes up to max completions (tag, status); waits up to wait_us for one if
 * none is ready.  Returns how many were written. */
int qfs_poll(qfs_t *s, uint64_t *tags, int32_t *status, uint32_t max, int wait_us);
/* st[0..14] = rounds, requests completed, keys processed, filters open,
 * filters waiting for admission, bytes in use, budget, requests waiting,
 * update requests applied in place (point updates), update requests merged
 * in bulk, the loop thread's nanoseconds spent forming rounds, launching
 * them, waiting for the device and completing them, and of the launching,
 * the nanoseconds spent copying keys into the pinned staging buffers. */
int qfs_stats(qfs_t *s, uint64_t *st);

#ifdef __cplusplus
}
#endif

#endif /* QF_H */
