"""Brute-force set model of the partition plan (test infrastructure only).

Everything is computed on explicit Python sets of row indices along the
partitioned dimension (dim 0), so tiny cases can be checked exhaustively
against the runtime's interval arithmetic.

Readings of the paper used here:
* Equal division of the parallel dimension among devices (Sec. "Division of
  Multidimensional Arrays"): owner block p of extent E split K ways is
  [floor(p*E/K), floor((p+1)*E/K)).
* Each device updates only the data range it owns (Sec. "Predicate-Based
  Filtering": every array write is guarded by the device's [lb, ub]).  For a
  loop that writes element i of dim 0 from outer iteration i, the guard keeps
  exactly the iterations whose write row lies in the owner block, so the
  filtered iteration set is {i in [lb, ub) : i in B_p}.
* Reads feed only guarded writes, so a device reads only the rows its kept
  iterations touch: [I.lo + off_lo, I.hi + off_hi) clipped to the array, or
  the whole array for an argument declared WHOLE.
* The paper sends updated data to every other device after each kernel; the
  lazy alternative modelled here copies, before a partition runs, exactly the
  rows it reads that its slab does not hold in their latest version, each
  from the partition that wrote it last.  Both leave every read row fresh.
* When several arguments update one array their ranges are merged to the
  widest (same section); the model merges every argument range of one array
  into its hull.
"""


def block(E, K, p):
    return (p * E // K, (p + 1) * E // K)


def slab(E, K, p, halo_lo, halo_hi, whole=False):
    if whole:
        return (0, E)
    lo, hi = block(E, K, p)
    return (max(0, lo - halo_lo), min(E, hi + halo_hi))


def iter_range(lb, ub, blk):
    """Iterations of [lb, ub) whose (identity-mapped) write row is in blk."""
    rows = set(range(lb, ub)) & set(range(*blk))
    return rows


def arg_rows(I, off_lo, off_hi, E, whole=False):
    """Rows read or written by the iterations I with offsets [off_lo, off_hi]."""
    if not I:
        return set()
    if whole:
        return set(range(E))
    rows = set()
    for i in I:
        for o in range(off_lo, off_hi + 1):
            if 0 <= i + o < E:
                rows.add(i + o)
    return rows


def hull(rows):
    return (min(rows), max(rows) + 1) if rows else (0, 0)


def runs(rows_with_src):
    """Group (row, src) pairs into maximal runs of consecutive rows with the
    same source: list of (src, lo, hi)."""
    out = []
    for r, s in sorted(rows_with_src):
        if out and out[-1][0] == s and out[-1][2] == r:
            out[-1] = (s, out[-1][1], r + 1)
        else:
            out.append((s, r, r + 1))
    return out


class ArrayState:
    """Latest writer per row (None: the host's data, valid everywhere) and
    the set of rows each partition's slab holds in their latest version."""

    def __init__(self, E, K, halo_lo, halo_hi, whole=False):
        self.E, self.K, self.whole = E, K, whole
        self.halo = (halo_lo, halo_hi)
        self.slabs = [set(range(*slab(E, K, p, halo_lo, halo_hi, whole))) for p in range(K)]
        self.writer = [None] * E
        self.valid = [set(s) for s in self.slabs]


def plan_loop(arrays, lb, ub, args, refresh="pull", max_holders=2):
    """Plan one loop nest.

    arrays: dict name -> ArrayState (all partitioned arrays share E and K).
    args: list of (name, mode, off_lo, off_hi, whole) with mode 'r' or 'w'.
    refresh: "pull" copies stale rows before a read; "holders" has every
    write also refresh the other slabs that hold the written rows (the
    paper's send-updated-data-after-the-kernel, restricted to the holders),
    as long as at most `max_holders` other slabs hold any of them (a halo
    no deeper than the blocks reaches one neighbour block on each side);
    a write reaching more holders invalidates them instead, and their
    readers pull.
    Returns a list, per partition p, of dicts with keys I (set), reads
    {name: rows}, writes {name: rows}, copies [(name, src, lo, hi)], and
    updates the states.  Raises ValueError on a range violation.
    """
    any_state = next(iter(arrays.values()))
    K = any_state.K
    E = any_state.E
    plans = []
    for p in range(K):
        I = iter_range(lb, ub, block(E, K, p))
        reads, writes = {}, {}
        for name, mode, lo, hi, whole in args:
            st = arrays[name]
            rows = arg_rows(I, lo, hi, st.E, whole or st.whole)
            d = reads if mode == "r" else writes
            d[name] = d.get(name, set()) | rows
        for d in (reads, writes):
            for name in d:
                if d[name]:
                    lo_, hi_ = hull(d[name])
                    d[name] = set(range(lo_, hi_))
        for name, rows in writes.items():
            st = arrays[name]
            if not rows <= set(range(*block(st.E, K, p))) and not st.whole:
                raise ValueError("write outside owner block")
        for name, rows in list(reads.items()) + list(writes.items()):
            if not rows <= arrays[name].slabs[p]:
                raise ValueError("access outside slab")
        plans.append({"I": I, "reads": reads, "writes": writes, "copies": []})
    # cross-partition overlap of a read of an array with another partition's
    # write of the same array (aliasing within one loop) is rejected
    for p in range(K):
        for q in range(K):
            if p == q:
                continue
            for name, rows in plans[p]["reads"].items():
                if rows & plans[q]["writes"].get(name, set()):
                    raise ValueError("read/write overlap across partitions")
            for name, rows in plans[p]["writes"].items():
                if rows & plans[q]["writes"].get(name, set()):
                    raise ValueError("overlapping writes")
    # copies: rows read that the slab does not hold fresh, from the last writer
    for p in range(K):
        for name, rows in sorted(plans[p]["reads"].items()):
            st = arrays[name]
            missing = rows - st.valid[p]
            pairs = []
            for r in missing:
                src = st.writer[r]
                assert src is not None and r in st.valid[src]
                pairs.append((r, src))
            for src, lo, hi in runs(pairs):
                plans[p]["copies"].append((name, src, lo, hi))
            st.valid[p] |= missing
    # apply writes
    for p in range(K):
        for name, rows in plans[p]["writes"].items():
            st = arrays[name]
            for r in rows:
                st.writer[r] = p
            st.valid[p] |= rows
            holders = [q for q in range(K) if q != p and rows & st.slabs[q]]
            mirror = refresh == "holders" and len(holders) <= max_holders
            for q in range(K):
                if q != p:
                    if mirror:
                        st.valid[q] |= rows & st.slabs[q]
                    else:
                        st.valid[q] -= rows
    return plans


def parallel_dim(par, seq, column_major=False):
    """Parallel dimension of an updated array (Sec. "Division of
    Multidimensional Arrays"): among the dimensions indexed by at least one
    parallel iterator, those with the most parallel iterators; among them
    those with the fewest sequential iterators; then the leftmost (C) or the
    rightmost (Fortran) one.  None when no dimension qualifies."""
    cands = [d for d in range(len(par)) if par[d] > 0]
    if not cands:
        return None
    most = max(par[d] for d in cands)
    cands = [d for d in cands if par[d] == most]
    fewest = min(seq[d] for d in cands)
    cands = [d for d in cands if seq[d] == fewest]
    return max(cands) if column_major else min(cands)
