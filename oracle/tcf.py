"""Two-choice filter (TCF) by definition, in Python and numpy.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this module.  It shares no code with the HIP
library.

What the paper fixes (Sec. 4, 4.1, 4.2):
  * the table is an array of blocks of B f-bit fingerprints ("tags"); every
    item has two candidate blocks from two hashes (power of two choices); an
    insert goes to the candidate holding fewer tags, a query answers whether
    the item's tag is in either candidate;
  * shortcut: when the primary candidate is less than 3/4 full the insert goes
    there without looking at the secondary;
  * items that fit in neither candidate go to a small backing table (about
    1/100 of the main table) searched by double hashing, at most 20 probes;
  * point blocks are unordered and a slot is taken by compare-and-swap of an
    empty or tombstone slot; a delete overwrites the tag with a tombstone;
  * bulk blocks keep their tags sorted; a bulk insert sorts the batch and
    merges, per block, the tags it holds, the batch items shortcut into it and
    the batch items the two choices gave it (three sorted lists);
  * the false-positive rate of a full table is 2B / 2^f.

Readings where the paper is silent (each is a definition here and in the
library, which implement it independently):
  * f = 16.  Point blocks hold 16 tags (32 bytes: the paper's 16-slot block
    with 16-bit tags), bulk blocks hold 128 sorted tags (256 bytes: the
    paper's bulk block of 128 16-bit slots).
  * Hash: h = fin64(key) (SplitMix64 finalizer); tag = low 16 bits of h with 0
    read as 1 and 0xFFFF as 0xFFFE; b1 = ((h >> 32) * nblocks) >> 32;
    h2 = fin64(h xor 0x9E3779B97F4A7C15); b2 = ((h2 >> 32) * nblocks) >> 32.
    nblocks <= 2^24.  Point slots: 0 empty, 0xFFFF tombstone.  Bulk slots:
    0xFFFF empty, kept after the tags so a block is sorted throughout.
  * An item's backing-table identity is its pair key
    min(b1, b2) << 40 | tag << 24 | max(b1, b2) (never 0 or 2^64 - 1).
  * Point insert: shortcut when the primary holds fewer than 12 tags; else
    the candidate with fewer tags (a tie goes to the primary).  The tag takes
    the lowest-index empty or tombstone slot; if that block has none, the
    other candidate is tried, then the backing table.  Point backing table:
    nbt = the power of two >= max(64, ceil(slots / 100)) 64-bit entries
    (0 empty, 2^64 - 1 tombstone), probe k at (a + k * s) mod nbt with
    a = h2 mod nbt, s = ((h2 >> 16) mod nbt) | 1, k < 20; an insert takes the
    first empty or tombstone entry, a lookup stops at the first empty entry.
  * Point delete: the lowest-index slot holding the tag in b1, else in b2,
    becomes a tombstone; else the first backing entry equal to the pair key.
  * Bulk insert of a batch (a function of the multiset of keys and the table):
      1. the items sorted by c = b1 << 40 | tag << 24 | b2;
      2. block b takes the first max(0, 96 - held(b)) items whose primary is b
         (in that order) as its shortcut list; f(b) = held(b) + shortcut(b);
      3. every other item chooses b1 if f(b1) <= f(b2), else b2;
      4. the chosen items of block b, sorted by chosen << 40 | tag << 24 |
         other, fill its 128 - f(b) free slots in that order; the rest go to
         the backing list;
      5. each block is the sorted union of its three lists; the bulk backing
         table is the sorted array of the pair keys of every item it holds,
         of at most nbt entries (same nbt rule); a batch that would exceed it
         fails and changes nothing.
  * Bulk delete of a batch: the items sorted by c; in each run of equal
    (b1, tag) the first k succeed in block b1, k = copies of the tag there;
    the others, sorted by b2 << 40 | tag << 24 | b1, do the same in b2 (as it
    is after the first step); the rest remove equal pair keys from the backing
    table; what remains is not found.
  * Bulk query: the tag in block b1 or in block b2, or the pair key in the
    backing table.
"""
from __future__ import annotations

import numpy as np

from .brute import fin64

U64 = np.uint64
PB = 16      # tags per point block
BB = 128     # tags per bulk block
SHORT_P = 12  # 3/4 of a point block
SHORT_B = 96  # 3/4 of a bulk block
EMPTY_P = 0
TOMB = 0xFFFF
EMPTY_B = 0xFFFF
BK_EMPTY = 0
BK_TOMB = (1 << 64) - 1
MAX_PROBES = 20
GOLDEN = 0x9E3779B97F4A7C15


class TableFull(Exception):
    pass


def backing_entries(slots: int) -> int:
    """Entries of the backing table of a table with `slots` slots."""
    need = max(64, -(-slots // 100))
    n = 1
    while n < need:
        n <<= 1
    return n


def tcf_hash(keys, nblocks: int):
    """(b1, b2, tag, h2) of each key, as uint64 arrays."""
    assert 1 <= nblocks <= (1 << 24)
    h = fin64(np.asarray(keys, dtype=U64))
    tag = h & U64(0xFFFF)
    tag = np.where(tag == U64(0), U64(1), np.where(tag == U64(0xFFFF), U64(0xFFFE), tag))
    nb = U64(nblocks)
    with np.errstate(over="ignore"):
        b1 = ((h >> U64(32)) * nb) >> U64(32)
        h2 = fin64(h ^ U64(GOLDEN))
        b2 = ((h2 >> U64(32)) * nb) >> U64(32)
    return b1, b2, tag, h2


def pair_key(b1, b2, tag):
    lo = np.minimum(b1, b2)
    hi = np.maximum(b1, b2)
    return (lo << U64(40)) | (tag << U64(24)) | hi


# ------------------------------------------------------------ point TCF ----
class PointTCF:
    """The point TCF applied one key at a time, in call order."""

    def __init__(self, nblocks: int):
        self.nb = nblocks
        self.blocks = np.zeros((nblocks, PB), dtype=np.uint16)
        self.nbt = backing_entries(nblocks * PB)
        self.backing = np.zeros(self.nbt, dtype=U64)

    def _held(self, b: int) -> int:
        row = self.blocks[b]
        return int(((row != EMPTY_P) & (row != TOMB)).sum())

    def _put(self, b: int, tag: int) -> bool:
        row = self.blocks[b]
        for i in range(PB):
            if row[i] == EMPTY_P or row[i] == TOMB:
                row[i] = tag
                return True
        return False

    def _probes(self, h2: int):
        a = h2 & (self.nbt - 1)
        s = ((h2 >> 16) & (self.nbt - 1)) | 1
        return [(a + k * s) & (self.nbt - 1) for k in range(MAX_PROBES)]

    def insert(self, key: int) -> bool:
        """False when the key fits neither candidate nor the backing table."""
        b1, b2, tag, h2 = (int(v[0]) for v in tcf_hash(np.array([key], dtype=U64), self.nb))
        if self._held(b1) < SHORT_P:
            order = (b1, b2)
        else:
            order = (b1, b2) if self._held(b1) <= self._held(b2) else (b2, b1)
        for b in order:
            if self._put(b, tag):
                return True
        pk = int(pair_key(U64(b1), U64(b2), U64(tag)))
        for pos in self._probes(h2):
            if self.backing[pos] in (U64(BK_EMPTY), U64(BK_TOMB)):
                self.backing[pos] = U64(pk)
                return True
        return False

    def delete(self, key: int) -> bool:
        b1, b2, tag, h2 = (int(v[0]) for v in tcf_hash(np.array([key], dtype=U64), self.nb))
        for b in (b1, b2):
            row = self.blocks[b]
            for i in range(PB):
                if row[i] == tag:
                    row[i] = TOMB
                    return True
        pk = U64(int(pair_key(U64(b1), U64(b2), U64(tag))))
        for pos in self._probes(h2):
            v = self.backing[pos]
            if v == U64(BK_EMPTY):
                return False
            if v == pk:
                self.backing[pos] = U64(BK_TOMB)
                return True
        return False

    def query(self, keys) -> np.ndarray:
        return point_query(self.blocks, self.backing, keys)


def point_query(blocks: np.ndarray, backing: np.ndarray, keys) -> np.ndarray:
    """Answers of point-TCF lookups (one bool per key) on a given table."""
    nb = blocks.shape[0]
    nbt = len(backing)
    b1, b2, tag, h2 = tcf_hash(keys, nb)
    t16 = tag.astype(np.uint16)
    hit = (blocks[b1.astype(np.int64)] == t16[:, None]).any(1) | (blocks[b2.astype(np.int64)] == t16[:, None]).any(1)
    pk = pair_key(b1, b2, tag)
    for i in np.nonzero(~hit)[0]:
        h = int(h2[i])
        a = h & (nbt - 1)
        s = ((h >> 16) & (nbt - 1)) | 1
        for k in range(MAX_PROBES):
            v = backing[(a + k * s) & (nbt - 1)]
            if v == U64(BK_EMPTY):
                break
            if v == pk[i]:
                hit[i] = True
                break
    return hit


def point_table_valid(blocks: np.ndarray, backing: np.ndarray, keys) -> str | None:
    """None if the table can hold exactly the multiset of `keys` under the
    point rules of placement (every tag in one of its item's two candidate
    blocks, every backing entry an item's pair key, nothing else), else the
    first reason it cannot.  Which candidate an item took depends on the
    order of concurrent inserts, so this checks for a valid assignment
    (a matching of items to stored tags, per tag value)."""
    nb = blocks.shape[0]
    b1, b2, tag, _ = tcf_hash(keys, nb)
    pk = pair_key(b1, b2, tag)
    # the backing table's entries are a sub-multiset of the items' pair keys
    bk = backing[(backing != U64(BK_EMPTY)) & (backing != U64(BK_TOMB))]
    from collections import Counter

    need = Counter(pk.tolist())
    used = Counter(bk.tolist())
    for v, c in used.items():
        if need.get(v, 0) < c:
            return f"backing entry {v:#x} held {c} times, items with that pair key: {need.get(v, 0)}"
    # items left for the blocks: drop one item per backing entry (items with
    # equal pair keys are interchangeable)
    left = np.ones(len(pk), dtype=bool)
    order = np.argsort(pk, kind="stable")
    spk = pk[order]
    for v, c in used.items():
        i0 = int(np.searchsorted(spk, U64(v)))
        left[order[i0:i0 + c]] = False
    # stored tags per (tag, block)
    flat = blocks.astype(np.int64)
    bid = np.repeat(np.arange(nb, dtype=np.int64), blocks.shape[1])
    val = flat.reshape(-1)
    keep = (val != EMPTY_P) & (val != TOMB)
    slots = Counter(zip(val[keep].tolist(), bid[keep].tolist()))
    stored_per_tag = Counter()
    for (t, b), c in slots.items():
        stored_per_tag[t] += c
    items_per_tag: dict[int, list[tuple[int, int]]] = {}
    for i in np.nonzero(left)[0]:
        items_per_tag.setdefault(int(tag[i]), []).append((int(b1[i]), int(b2[i])))
    for t in set(stored_per_tag) | set(items_per_tag):
        its = items_per_tag.get(t, [])
        if stored_per_tag.get(t, 0) != len(its):
            return f"tag {t}: {stored_per_tag.get(t, 0)} stored, {len(its)} items"
        cap = {b: slots[(t, b)] for b in {b for pair in its for b in pair} if (t, b) in slots}
        if sum(cap.values()) != len(its):
            return f"tag {t}: stored outside its items' candidate blocks"
        # Kuhn's augmenting paths, blocks with capacities
        owner: dict[int, list[int]] = {b: [] for b in cap}

        def place(i, seen):
            for b in its[i]:
                if b not in cap or b in seen:
                    continue
                seen.add(b)
                if len(owner[b]) < cap[b]:
                    owner[b].append(i)
                    return True
                for j in list(owner[b]):
                    if place(j, seen):
                        owner[b].remove(j)
                        owner[b].append(i)
                        return True
            return False

        for i in range(len(its)):
            if not place(i, set()):
                return f"tag {t}: no assignment of its {len(its)} items to their candidate blocks"
    return None


# ------------------------------------------------------------- bulk TCF ----
class BulkTCF:
    """The bulk TCF: sorted blocks, batches applied as the definition says."""

    def __init__(self, nblocks: int):
        self.nb = nblocks
        self.blocks = np.full((nblocks, BB), EMPTY_B, dtype=np.uint16)
        self.cap = backing_entries(nblocks * BB)
        self.backing = np.zeros(0, dtype=U64)  # sorted pair keys

    def held(self) -> np.ndarray:
        return (self.blocks != EMPTY_B).sum(1).astype(np.int64)

    def _rebuild(self, bid: np.ndarray, tags: np.ndarray) -> np.ndarray:
        """Blocks holding exactly the (block, tag) pairs given, sorted."""
        out = np.full((self.nb, BB), EMPTY_B, dtype=np.uint16)
        if len(bid) == 0:
            return out
        o = np.lexsort((tags, bid))
        bid, tags = bid[o], tags[o]
        start = np.searchsorted(bid, np.arange(self.nb))
        rank = np.arange(len(bid)) - start[bid]
        assert rank.max() < BB
        out[bid, rank] = tags.astype(np.uint16)
        return out

    def _contents(self):
        held = self.blocks != EMPTY_B
        bid = np.nonzero(held)[0].astype(np.int64)
        tags = self.blocks[held].astype(np.int64)
        return bid, tags

    def insert(self, keys) -> None:
        """Raises TableFull (table unchanged) when the backing list overflows."""
        keys = np.asarray(keys, dtype=U64)
        if len(keys) == 0:
            return
        b1, b2, tag, _ = tcf_hash(keys, self.nb)
        c = np.sort((b1 << U64(40)) | (tag << U64(24)) | b2)
        b1 = (c >> U64(40)).astype(np.int64)
        tag = ((c >> U64(24)) & U64(0xFFFF)).astype(np.int64)
        b2 = (c & U64(0xFFFFFF)).astype(np.int64)
        held = self.held()
        start = np.searchsorted(b1, np.arange(self.nb))
        rank = np.arange(len(c)) - start[b1]
        cnt = np.bincount(b1, minlength=self.nb)
        s = np.minimum(np.maximum(0, SHORT_B - held), cnt)
        short = rank < s[b1]
        f = held + s
        p = ~short
        pb1, pb2, ptag = b1[p], b2[p], tag[p]
        ch = np.where(f[pb1] <= f[pb2], pb1, pb2)
        ot = np.where(ch == pb1, pb2, pb1)
        k2 = np.sort((ch.astype(U64) << U64(40)) | (ptag.astype(U64) << U64(24)) | ot.astype(U64))
        ch2 = (k2 >> U64(40)).astype(np.int64)
        tag2 = ((k2 >> U64(24)) & U64(0xFFFF)).astype(np.int64)
        ot2 = (k2 & U64(0xFFFFFF)).astype(np.int64)
        start2 = np.searchsorted(ch2, np.arange(self.nb))
        rank2 = np.arange(len(k2)) - start2[ch2]
        placed = rank2 < (BB - f)[ch2]
        over = pair_key(ch2[~placed].astype(U64), ot2[~placed].astype(U64), tag2[~placed].astype(U64))
        if len(self.backing) + len(over) > self.cap:
            raise TableFull(f"backing table would hold {len(self.backing) + len(over)} > {self.cap}")
        obid, otags = self._contents()
        bid = np.concatenate([obid, b1[short], ch2[placed]])
        tags = np.concatenate([otags, tag[short], tag2[placed]])
        self.blocks = self._rebuild(bid, tags)
        self.backing = np.sort(np.concatenate([self.backing, over]))

    def delete(self, keys) -> int:
        """Returns the number of keys not found."""
        keys = np.asarray(keys, dtype=U64)
        if len(keys) == 0:
            return 0
        b1, b2, tag, _ = tcf_hash(keys, self.nb)
        left = np.sort((b1 << U64(40)) | (tag << U64(24)) | b2)
        for step in (0, 1):
            if step == 1:
                # the rest, keyed by the secondary block
                lb1 = left >> U64(40)
                lt = (left >> U64(24)) & U64(0xFFFF)
                lb2 = left & U64(0xFFFFFF)
                left = np.sort((lb2 << U64(40)) | (lt << U64(24)) | lb1)
            if len(left) == 0:
                break
            blk = (left >> U64(40)).astype(np.int64)
            t = ((left >> U64(24)) & U64(0xFFFF)).astype(np.int64)
            bid, tags = self._contents()
            have = np.sort(bid * 65536 + tags)
            want = blk * 65536 + t
            copies = np.searchsorted(have, want, "right") - np.searchsorted(have, want, "left")
            gstart = np.searchsorted(want, want, "left")
            rank = np.arange(len(want)) - gstart
            ok = rank < copies
            # remove one stored copy per successful delete
            rm = np.sort(want[ok])
            hv, hc = np.unique(have, return_counts=True)
            if len(rm):
                rv, rc = np.unique(rm, return_counts=True)
                idx = np.searchsorted(hv, rv)
                hc[idx] -= rc
            kept = np.repeat(hv, hc)
            self.blocks = self._rebuild(kept // 65536, kept % 65536)
            rest = left[~ok]
            if step == 1:
                # back to the primary orientation
                rb2 = rest >> U64(40)
                rt = (rest >> U64(24)) & U64(0xFFFF)
                rb1 = rest & U64(0xFFFFFF)
                rest = (rb1 << U64(40)) | (rt << U64(24)) | rb2
            left = rest
        if len(left) == 0:
            return 0
        lb1 = left >> U64(40)
        lt = (left >> U64(24)) & U64(0xFFFF)
        lb2 = left & U64(0xFFFFFF)
        pk = np.sort(pair_key(lb1, lb2, lt))
        bv, bc = np.unique(self.backing, return_counts=True)
        dv, dc = np.unique(pk, return_counts=True)
        idx = np.searchsorted(bv, dv)
        idx_c = np.minimum(idx, max(len(bv) - 1, 0))
        hit = (idx < len(bv)) & (bv[idx_c] == dv) if len(bv) else np.zeros(len(dv), dtype=bool)
        take = np.zeros(len(dv), dtype=np.int64)
        take[hit] = np.minimum(bc[idx_c[hit]], dc[hit])
        if len(bv):
            np.subtract.at(bc, idx_c[hit], take[hit])
            self.backing = np.repeat(bv, bc)
        return int(dc.sum() - take.sum())

    def query(self, keys) -> np.ndarray:
        return bulk_query(self.blocks, self.backing, keys)


def bulk_query(blocks: np.ndarray, backing: np.ndarray, keys) -> np.ndarray:
    nb = blocks.shape[0]
    b1, b2, tag, _ = tcf_hash(keys, nb)
    t16 = tag.astype(np.uint16)
    hit = (blocks[b1.astype(np.int64)] == t16[:, None]).any(1) | (blocks[b2.astype(np.int64)] == t16[:, None]).any(1)
    if len(backing):
        pk = pair_key(b1, b2, tag)
        pos = np.minimum(np.searchsorted(backing, pk), len(backing) - 1)
        hit |= backing[pos] == pk
    return hit
