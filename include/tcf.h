/*
 * tcf.h -- C ABI of the two-choice filter (TCF) in libqf.so, on one MI355X.
 *
 * The filter of Sec. 4 of McCoy, Hofmeyr, Yelick and Pandey, "High-Performance
 * Filters for GPUs" (PPoPP'23):
 *   - blocks of B 16-bit fingerprints ("tags"); each item has two candidate
 *     blocks from two hashes (power of two choices): an insert goes to the
 *     candidate holding fewer tags, a query looks for the item's tag in both;
 *   - shortcut (Sec. 4.1): when the primary candidate is less than 3/4 full the
 *     insert goes there without reading the secondary;
 *   - backing table (Sec. 4.1): items that fit in neither candidate go to a
 *     table of about 1/100 of the slots;
 *   - point form (Sec. 4, Algorithm 1): unordered 16-tag blocks (32 bytes),
 *     one item per lane, a slot taken by compare-and-swap of an empty or
 *     tombstone slot, a delete writes a tombstone; the backing table is probed
 *     by double hashing, at most 20 probes;
 *   - bulk form (Sec. 4.2): sorted 128-tag blocks (256 bytes); a batch is
 *     sorted, and each block merges the tags it holds, the batch items
 *     shortcut into it and the batch items the two choices gave it; the
 *     backing table is a sorted array; lookups binary-search.
 * The hash, tag encoding, backing-table identity and the exact bulk rules are
 * this library's readings of what the paper leaves open:
 *   h = SplitMix64 finalizer of the key; tag = low 16 bits of h (0 read as 1,
 *   0xFFFF as 0xFFFE); b1 = ((h >> 32) * nblocks) >> 32;
 *   h2 = finalizer of (h xor 0x9E3779B97F4A7C15); b2 = ((h2 >> 32) * nblocks) >> 32;
 *   backing-table identity = min(b1,b2) << 40 | tag << 24 | max(b1,b2).
 *   Bulk insert: the batch sorted by b1 << 40 | tag << 24 | b2; block b takes
 *   the first max(0, 96 - held(b)) items whose primary is b; every other item
 *   takes the candidate with the smaller f = held + shortcut (tie: primary);
 *   the items a block is given fill its free slots in order of
 *   block << 40 | tag << 24 | other, the rest go to the backing table.
 *   Bulk delete: per (b1, tag) the first copies-in-b1 deletes of the sorted
 *   batch succeed in b1, the rest likewise in b2, then in the backing table.
 * A bulk result is a function of the table and the batch's multiset of keys.
 *
 * Conventions: as in qf.h (device pointers, n elements, stream as void*,
 * stream-ordered).  Error codes are qf.h's (0 ok, -1 argument, -2 full,
 * -3 out of memory, -4 device).
 */
#ifndef TCF_H
#define TCF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tcf_filter tcf_t;

enum { TCF_POINT = 0, TCF_BULK = 1 };

/* A filter of nblocks blocks (1 <= nblocks <= 2^24): kind TCF_POINT (16 tags
 * per block) or TCF_BULK (128 tags per block), and its backing table of
 * max(64, ceil(slots / 100)) entries rounded up to a power of two.  Empty.
 * NULL on error (qf_last_error()). */
tcf_t *tcf_create(uint64_t nblocks, int kind);
void tcf_destroy(tcf_t *t); /* NULL-safe; waits for the device */

/* Insert n keys.
 * TCF_POINT: one lane per key, concurrently, in no set order (which
 *   candidate an item takes can depend on that order); d_status (n int32,
 *   may be NULL) gets 0, or QF_ERR_FULL when neither candidate nor the
 *   backing table had room (that key not inserted); the first such error is
 *   also reported by tcf_sync.
 * TCF_BULK: the whole batch or nothing: QF_ERR_FULL, returned at once, when
 *   the backing table would overflow (the table is unchanged); d_status must
 *   be NULL.  Waits for the stream once (to read the overflow count). */
int tcf_insert(tcf_t *t, const uint64_t *d_keys, uint64_t n, int32_t *d_status, void *stream);

/* d_out[i] = 1 if key i's tag is in one of its candidate blocks or its
 * identity is in the backing table, else 0 (false positives possible, never
 * false negatives for inserted keys). */
int tcf_query(tcf_t *t, const uint64_t *d_keys, uint64_t n, uint8_t *d_out, void *stream);

/* Delete one copy per key (point: the tag becomes a tombstone; bulk: the
 * block is re-sorted without it).  The number of keys with no copy to remove
 * is ADDED to *d_not_found (device, one uint64; may be NULL).  A key that was
 * never inserted can remove another key's equal tag, as with any filter. */
int tcf_delete(tcf_t *t, const uint64_t *d_keys, uint64_t n, uint64_t *d_not_found, void *stream);

/* Waits for the stream; returns (and clears) the first deferred error. */
int tcf_sync(tcf_t *t, void *stream);

/* info[0..6] = kind, nblocks, tags per block, backing entries (capacity),
 * backing entries in use (bulk; point: those holding an item), tags held in
 * blocks, device bytes (host array). */
int tcf_info(tcf_t *t, uint64_t *info, void *stream);

/* Copies the table to host arrays: h_slots (nblocks * tags-per-block
 * uint16; point: 0 empty, 0xFFFF tombstone; bulk: sorted, 0xFFFF empty after
 * the tags) and h_backing (capacity uint64 entries; point: 0 empty,
 * 2^64 - 1 tombstone; bulk: the sorted identities in use, then zeros).
 * Waits for the stream. */
int tcf_export(tcf_t *t, uint16_t *h_slots, uint64_t *h_backing, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TCF_H */
