"""Checks over the runtime's operation trace (host-side, no GPU).

* race_check: happens-before race detector.  Ops on one stream are ordered;
  a WAIT orders the waiting stream after the awaited op; a host SYNC orders
  every later op after the synchronised stream; a JOIN orders every later op
  after every earlier one.  Two accesses to the same
  rows of the same slab from different streams, at least one a write, must
  be ordered, otherwise the trace has a race.
* freshness_check: replays the trace in issue order with symbolic versions
  and checks that every row a kernel reads holds the latest value written
  to that row of the array (by any partition or the host).  A private write
  (a filtered loop's write outside the partition's owner block) leaves a
  value that is never the latest; a duplicated loop's later partitions write
  the value its first partition wrote; a POISON fill leaves invalid values.
"""
from collections import defaultdict

OPS_WITH_SEQ = {"COPY", "KERNEL", "H2D", "D2H", "COMBINE", "POISON"}


def _max(a, b):
    return {k: max(a.get(k, 0), b.get(k, 0)) for k in set(a) | set(b)}


def race_check(trace, skip_wait=None):
    """Returns a list of race descriptions (empty if none).  skip_wait:
    index (into the list of WAIT entries) of one wait to ignore."""
    vc = defaultdict(dict)      # stream -> vector clock for its next op
    host = {}
    op_vc = {}
    pending = defaultdict(list)  # (stream, seq) -> accesses
    hist = defaultdict(list)    # (array, slab, row) -> [(stream, seq, mode)]
    races = []
    wait_i = -1
    for t in trace:
        op = t["op"]
        if op == "WAIT":
            wait_i += 1
            if skip_wait is not None and wait_i == skip_wait:
                continue
            d, q, m = t["stream"], t["src"], t["seq"]
            vc[d] = _max(vc[d], op_vc.get((q, m), {q: m}))  # ops before the trace started: only q's clock
        elif op == "SYNC":
            s, m = t["stream"], t["seq"]
            if (s, m) in op_vc:
                host = _max(host, op_vc[(s, m)])
        elif op == "JOIN":
            for v in op_vc.values():
                host = _max(host, v)
        elif op == "ACCESS":
            pending[(t["stream"], t["seq"])].append(t)
        elif op in OPS_WITH_SEQ:
            d, n = t["stream"], t["seq"]
            v = _max(vc[d], host)
            v[d] = n
            vc[d] = dict(v)
            op_vc[(d, n)] = dict(v)
            for a in pending.pop((d, n), []):
                mode = "w" if a["kind"] in (2, 3, 4, 5) else "r"
                for row in range(a["lo"], a["hi"]):
                    key = (a["array"], a["dst"], row)
                    for (ps, pn, pm) in hist[key]:
                        if ps == d or (pm == "r" and mode == "r"):
                            continue
                        if v.get(ps, 0) < pn:
                            races.append(f"{op}@s{d}#{n} {mode} array {a['array']} slab {a['dst']} row {row} "
                                         f"unordered with s{ps}#{pn} {pm}")
                    hist[key].append((d, n, mode))
    return races


def freshness_check(trace):
    """Returns a list of stale reads (empty if every kernel read is fresh)."""
    logical = {}               # (array, row) -> version
    stored = {}                # (array, slab, row) -> version
    pending = defaultdict(list)
    stale = []
    counter = [0]
    epoch = [0]   # host data changes only between kernels

    def new_version():
        counter[0] += 1
        return counter[0]

    for t in trace:
        op = t["op"]
        if op == "ALLOC":
            for row in range(t["lo"], t["hi"]):
                stored[(t["array"], t["dst"], row)] = ("created", t["array"])
                logical.setdefault((t["array"], row), ("created", t["array"]))
        elif op == "ACCESS":
            pending[(t["stream"], t["seq"])].append(t)
        elif op == "H2D":
            for row in range(t["lo"], t["hi"]):
                logical[(t["array"], row)] = ("host", epoch[0])
                stored[(t["array"], t["dst"], row)] = ("host", epoch[0])
            pending.pop((t["stream"], t["seq"]), None)
        elif op == "COPY":
            for row in range(t["lo"], t["hi"]):
                stored[(t["array"], t["dst"], row)] = stored[(t["array"], t["src"], row)]
            pending.pop((t["stream"], t["seq"]), None)
        elif op == "KERNEL":
            epoch[0] += 1
            acc = pending.pop((t["stream"], t["seq"]), [])
            for a in acc:
                if a["kind"] == 1:
                    for row in range(a["lo"], a["hi"]):
                        want = logical.get((a["array"], row))
                        have = stored.get((a["array"], a["dst"], row))
                        if have != want:
                            stale.append(f"kernel s{t['stream']}#{t['seq']} reads array {a['array']} row {row} "
                                         f"in slab {a['dst']}: version {have}, latest {want}")
            written = {}   # one new value per (array, row), whichever slabs receive it
            for a in acc:
                if a["kind"] == 3:  # private values: never the array's latest
                    for row in range(a["lo"], a["hi"]):
                        stored[(a["array"], a["dst"], row)] = ("private", new_version())
                elif a["kind"] == 4:  # a duplicated loop: the value its first partition wrote
                    for row in range(a["lo"], a["hi"]):
                        stored[(a["array"], a["dst"], row)] = logical.get((a["array"], row))
            for a in acc:
                if a["kind"] == 2:
                    for row in range(a["lo"], a["hi"]):
                        key = (a["array"], row)
                        if key not in written:
                            written[key] = new_version()
                        logical[key] = written[key]
                        stored[(a["array"], a["dst"], row)] = written[key]
        elif op == "POISON":
            for row in range(t["lo"], t["hi"]):
                stored[(t["array"], t["dst"], row)] = ("poison", new_version())
            pending.pop((t["stream"], t["seq"]), None)
        elif op == "D2H":
            for row in range(t["lo"], t["hi"]):
                want = logical.get((t["array"], row))
                have = stored.get((t["array"], t["src"], row))
                if have != want:
                    stale.append(f"gather of array {t['array']} row {row} from slab {t['src']} is stale")
            pending.pop((t["stream"], t["seq"]), None)
    return stale
