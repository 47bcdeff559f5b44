// Runtime core of the K-partitioned loop-nest library: present table,
// partition planner (owner blocks, iteration sub-ranges, access ranges),
// coherence tracker and copy planner, stream/event scheduler with hazard
// tracking, reduction combine, graph batches with persistent task groups,
// the loop timer used by the autotuner, and the C ABI of jacc.h.
//
// Paper: JACC (Matsumura, Garcia De Gonzalo, Pena; HiPC 2021).  The data
// model follows its data-region routines and present table (Sec. "JACC",
// Sec. "Automated Asynchronous Execution"); the split follows the equal
// division of the parallel dimension and the per-device write ranges of
// predicate-based filtering (Sec. "Predicate-Based Filtering", Sec.
// "Division of Multidimensional Arrays"); cross-queue synchronisation only
// where a data dependency exists, skipping dependencies already solved by an
// earlier synchronisation, follows Sec. "Automated Asynchronous Execution".
#include "jacc.h"

#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "ctx_internal.h"
#include "kernels.h"

namespace {

constexpr int kMaxK = 64;
constexpr int kSlots = 4096;
constexpr int kEventRing = 16;
constexpr int64_t kWgCapacity = 1 << 16;  // workgroup partials per stream
constexpr int kTaskCapacity = 4096;       // persistent tasks per batch
constexpr int64_t kBandedMinCols = 1 << 20;  // SpMV x length from which the banded form is the default

thread_local std::string g_init_err;  // message of the last failed context-free call (jacc_init, no-alloc step)

struct Range {
    int64_t lo = 0, hi = 0;
    bool empty() const { return hi <= lo; }
};
inline Range isect(Range a, Range b) { return {std::max(a.lo, b.lo), std::min(a.hi, b.hi)}; }

// Sorted set of disjoint half-open intervals.  Updates build the new list in
// a buffer kept per thread and swap it in, so steady-state planning does not
// allocate.
struct IntervalSet {
    std::vector<Range> v;
    static std::vector<Range> &scratch() {
        static thread_local std::vector<Range> buf;
        buf.clear();
        return buf;
    }
    void add(Range r) {
        if (r.empty()) return;
        std::vector<Range> &out = scratch();
        bool placed = false;
        for (const Range &x : v) {
            if (x.hi < r.lo) {
                out.push_back(x);
            } else if (r.hi < x.lo) {
                if (!placed) {
                    out.push_back(r);
                    placed = true;
                }
                out.push_back(x);
            } else {
                r = {std::min(r.lo, x.lo), std::max(r.hi, x.hi)};
            }
        }
        if (!placed) out.push_back(r);
        v.swap(out);
    }
    void sub(Range r) {
        if (r.empty()) return;
        std::vector<Range> &out = scratch();
        for (const Range &x : v) {
            if (x.hi <= r.lo || r.hi <= x.lo) {
                out.push_back(x);
                continue;
            }
            if (x.lo < r.lo) out.push_back({x.lo, r.lo});
            if (r.hi < x.hi) out.push_back({r.hi, x.hi});
        }
        v.swap(out);
    }
    std::vector<Range> missing(Range r) const {  // r minus the set
        std::vector<Range> out;
        int64_t cur = r.lo;
        for (const Range &x : v) {
            if (x.hi <= cur) continue;
            if (x.lo >= r.hi) break;
            if (x.lo > cur) out.push_back({cur, std::min(x.lo, r.hi)});
            cur = std::max(cur, x.hi);
            if (cur >= r.hi) break;
        }
        if (cur < r.hi) out.push_back({cur, r.hi});
        return out;
    }
};

// Piecewise-constant map over a row range.
template <class T>
struct IntervalMap {
    struct Piece {
        int64_t lo, hi;
        T val;
    };
    std::vector<Piece> v;
    void init(int64_t lo, int64_t hi, const T &val) { v.assign(1, Piece{lo, hi, val}); }
    size_t split(int64_t x) {  // index of the piece starting at x (v.size() at the end)
        for (size_t i = 0; i < v.size(); ++i) {
            if (v[i].lo == x) return i;
            if (v[i].lo < x && x < v[i].hi) {
                Piece right = v[i];
                right.lo = x;
                v[i].hi = x;
                v.insert(v.begin() + (long)i + 1, right);
                return i + 1;
            }
        }
        return v.size();
    }
    template <class F>
    void for_range(Range r, F f) {  // f(Piece&) over the pieces inside r (split at its ends)
        if (r.empty() || v.empty()) return;
        r = isect(r, Range{v.front().lo, v.back().hi});
        if (r.empty()) return;
        size_t a = split(r.lo);
        size_t b = split(r.hi);
        for (size_t i = a; i < b; ++i) f(v[i]);
    }
    void assign(Range r, const T &val) {
        for_range(r, [&](Piece &p) { p.val = val; });
        coalesce();
    }
    void coalesce() {  // merges equal neighbours in place
        size_t w = 0;
        for (size_t i = 0; i < v.size(); ++i) {
            if (w > 0 && v[w - 1].hi == v[i].lo && v[w - 1].val == v[i].val) {
                v[w - 1].hi = v[i].hi;
            } else {
                if (w != i) v[w] = std::move(v[i]);
                ++w;
            }
        }
        v.resize(w);
    }
};

// A short list kept inline (no heap allocation up to N elements).
template <class T, int N>
struct SmallVec {
    T inl[N];
    int n = 0;
    std::vector<T> spill;  // elements N, N+1, ...
    int size() const { return n; }
    T &operator[](int i) { return i < N ? inl[i] : spill[(size_t)(i - N)]; }
    const T &operator[](int i) const { return i < N ? inl[i] : spill[(size_t)(i - N)]; }
    void push_back(const T &x) {
        if (n < N)
            inl[n] = x;
        else
            spill.push_back(x);
        ++n;
    }
    void clear() {
        n = 0;
        spill.clear();
    }
    bool operator==(const SmallVec &o) const {
        if (n != o.n) return false;
        for (int i = 0; i < n; ++i)
            if ((*this)[i] != o[i]) return false;
        return true;
    }
};

// Access history of a row interval of one slab: last writer (stream, seq)
// and, per other stream, the latest read since that write.
struct Access {
    int32_t ws = -1;
    int64_t wseq = 0;
    SmallVec<std::pair<int32_t, int64_t>, 4> reads;
    bool operator==(const Access &o) const { return ws == o.ws && wseq == o.wseq && reads == o.reads; }
};

struct Slab {
    void *dev = nullptr;
    Range rows;
    // storage: rows [base, ...) from dev; a column slab (arrays split along
    // dim 1) starts at an even column and has an even pitch (elements per
    // stored row), so that even global columns sit on 16-byte boundaries
    int64_t base = 0, pitch = 0;
    IntervalMap<Access> acc;
};

struct Array {
    int id = 0;
    uintptr_t host = 0;
    size_t bytes = 0;
    jacc_array_desc d{};
    int K = 1;
    int home = 0;         // stream of partition 0 for transfers; partition p uses (home + p) mod streams
    int last_stream = -1;  // base stream of the last loop that wrote this array
    int64_t E = 0, row_elems = 1;   // rows along the partitioned dimension; elements per row
    size_t esize = 8, row_bytes = 8;
    int pdim = 0;  // partitioned dimension: 0, or 1 (a 2-D array split into column blocks)
    int refs = 1;
    bool whole = false;
    bool shared = false;  // whole == 2: one device copy that every partition reads (never written by loops)
    std::vector<Slab> slabs;
    IntervalMap<int32_t> writer;  // -1: host data, valid in every holder
    std::vector<IntervalSet> valid;
    uint64_t version = 0;  // bumped by every device write (kernels, copies from the host)
    Range block(int p) const {
        return {(int64_t)((__int128)p * E / K), (int64_t)((__int128)(p + 1) * E / K)};
    }
};

// Coherence and hazard state of one array (for the replay check of batches).
struct ArraySnap {
    IntervalMap<int32_t> writer;
    std::vector<IntervalSet> valid;
    std::vector<IntervalMap<Access>> acc;
};

struct EvEntry {
    hipEvent_t ev = nullptr;
    int64_t covers = -1;
    std::vector<int64_t> waited;  // snapshot of the stream's waited[] at record time
};

struct StreamState {
    hipStream_t s = nullptr;
    int64_t seq = 0;
    int64_t recorded = 0;
    std::vector<EvEntry> ring;
    int ring_next = 0;
    std::vector<int64_t> waited;  // waited[q]: ops of stream q known complete before our next op
    hipEvent_t join_ev = nullptr;
    int64_t last_use = 0;  // loop tick of the last loop issued on this stream
};

struct SeqRef {
    int s = 0;
    int64_t seq = 0;
};

struct LoopCall {
    int kind;
    jacc_bounds b;
    std::vector<jacc_arg> args;
    std::vector<double> scalars;
    int slot;
    bool has_cfg;
    jacc_config cfg;
};

struct PendingAccess {
    Array *A;
    int p;
    Range r;
    bool write;
};

struct Batch {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<LoopCall> calls;
    std::vector<jacc_trace_op> captured;  // ops planned while capturing
    bool replay_safe = false;
    // arrays whose device slabs the graph's nodes address; when one of them
    // leaves the data region the graph is stale and is never replayed again
    std::vector<int> array_ids;
    bool stale = false;
    jk::PTask *dev_tasks = nullptr;   // kTaskCapacity device task records
    jk::PTask *host_tasks = nullptr;  // pinned staging of the same size
    int tasks_used = 0;
    int groups = 0;
};

// The column-banded copy of one partition's rows of a CSR matrix, built on
// the device at its first banded product and kept while row_ptr, col and val
// are unchanged (their versions).
struct BandCache {
    int rp_id = -1, col_id = -1, val_id = -1, p = 0, bands = 0;
    int64_t lo = 0, hi = 0;
    uint64_t v_rp = 0, v_col = 0, v_val = 0;
    bool built = false;
    jk::BandBufs bb{};
    void *mem[5] = {};
};

size_t dtype_size(int dt) {
    switch (dt) {
        case JACC_F64: return 8;
        case JACC_F32: return 4;
        case JACC_I32: return 4;
        case JACC_I64: return 8;
        default: return 0;
    }
}

}  // namespace

struct jacc_ctx {
    int K = 1;
    unsigned flags = 0;
    bool dry = false, tracing = false, serialize = false;
    bool lazy = false;       // pull halo rows before reads instead of mirroring them at writes
    bool split = false;      // stencil partitions: own-block rows first, edge rows after (any K)
    bool no_split = false;   // never split (default: split at K <= 4)
    bool no_pack = false;    // a launch per partition for eager stencil loops (default: one packed launch)
    bool eager = false;      // broadcast written rows to every holder after each loop
    bool fork_capture = false;  // plan batches with every partition on its own stream (dry run only)
    bool plan_only = false;  // planning pass without device work (batch replay check)
    bool poison = false;     // fill the rows a loop leaves stale with NaN bytes (debug)
    bool markers = false;    // roctx ranges around the host phases of each call
    int tune_mode = 0;       // loops without a configuration: 0 model pick, 1 defaults, 2 tuned
    std::string tune_db;     // timing database of tune_mode 2 (empty: none)
    std::map<std::vector<int64_t>, jacc_config> tuned;  // tune_mode 2 picks per loop signature
    // per-loop records (JACC_LOG): JSON lines; with JACC_LOG_TIMES a loop
    // that runs on one stream is timed by events around its work, read back
    // at the next synchronisation (or when many are pending)
    FILE *log = nullptr;
    bool log_times = false;
    int64_t log_seq = 0;
    int64_t log_copies = 0, log_copy_bytes = 0;  // running totals of device copies
    struct LogRec {
        std::string json;  // the record without its timing fields and closing brace
        double work = 0;   // algorithmic bytes (or flop when flop)
        bool flop = false;
        hipEvent_t e0 = nullptr, e1 = nullptr;
    };
    std::vector<LogRec> log_pending;
    jacc_allocator alloc{};
    bool use_hipmalloc = true;
    bool own_streams = false;
    std::vector<StreamState> st;
    std::map<uintptr_t, Array *> present;
    int next_id = 0;
    int next_home = 0;
    int64_t tick = 0;
    int status = JACC_OK;
    std::string err;
    std::vector<jacc_trace_op> trace;
    std::vector<jacc_trace_op> *oplog = nullptr;
    uintptr_t fake_next = (uintptr_t)1 << 44;
    // reductions (buffers indexed by stream)
    double *slots = nullptr;             // kSlots doubles
    double *partials = nullptr;          // kSlots * kMaxK doubles: per slot, one per partition
    double *wg = nullptr;                // streams * kWgCapacity doubles
    std::vector<SeqRef> partial_reader;  // last combine that read partials[slot][p]
    std::vector<SeqRef> slot_src;        // op that produced each slot
    // batches
    std::vector<Batch *> batches;
    Batch *cur = nullptr;
    std::vector<jk::PTask> ptasks;  // pending persistent group
    std::vector<PendingAccess> paccs;
    std::vector<Array *> parrays;
    hipEvent_t fork_ev = nullptr, t0 = nullptr, t1 = nullptr;
    // per-partition kernel timing (jacc_time_loop_parts): events around each
    // partition's launch; kev[2p] before, kev[2p+1] after
    bool time_parts = false;
    std::vector<hipEvent_t> kev;
    uint64_t kev_used = 0;  // bit p: partition p launched in the timed call
    // banded SpMV copies, per partition and matrix
    std::vector<BandCache> bands;
    // cost model attached by jacc_model_load (owned; released at finalize)
    void *model = nullptr;
    void (*model_release)(void *) = nullptr;
    // fault injection (tests): fail the n-th op of a kind
    int fault_kind = 0;  // 1 copy, 2 launch
    int64_t fault_n = -1, fault_count = 0;
};

namespace {

bool live(const jacc_ctx *c) { return !c->dry && !c->plan_only; }

// roctx ranges (JACC_INIT_MARKERS): the marker library is opened on first
// use, so contexts without markers never load it.
struct RoctxApi {
    int (*push)(const char *) = nullptr;
    int (*pop)() = nullptr;
    bool ok = false;
};
const RoctxApi &roctx_api() {
    static const RoctxApi api = [] {
        RoctxApi a;
        void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
        if (!h) return a;
        a.push = (int (*)(const char *))dlsym(h, "roctxRangePushA");
        a.pop = (int (*)())dlsym(h, "roctxRangePop");
        a.ok = a.push && a.pop;
        return a;
    }();
    return api;
}
// A named host range for the lifetime of the object.
class Marker {
  public:
    Marker(const jacc_ctx *c, const char *fmt, ...) {
        if (!c || !c->markers || !roctx_api().ok) return;
        char buf[96];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        roctx_api().push(buf);
        on_ = true;
    }
    ~Marker() {
        if (on_) roctx_api().pop();
    }
    Marker(const Marker &) = delete;
    Marker &operator=(const Marker &) = delete;

  private:
    bool on_ = false;
};

int set_err(jacc_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
    return code;
}

int dev_fail(jacc_ctx *c, hipError_t e, const char *what) {
    c->status = JACC_ERR_DEVICE;
    return set_err(c, JACC_ERR_DEVICE, "%s failed: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIPCHK(c, expr, what)                               \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return dev_fail(c, e_, what); \
    } while (0)

void trace(jacc_ctx *c, int op, int stream, int array, int src, int dst, int kind, int64_t lo, int64_t hi,
           int64_t seq) {
    if (!c->tracing && !c->oplog) return;
    jacc_trace_op t;
    t.op = op;
    t.stream = stream;
    t.array = array;
    t.src = src;
    t.dst = dst;
    t.kind = kind;
    t.lo = lo;
    t.hi = hi;
    t.seq = seq;
    if (c->tracing && !c->plan_only) c->trace.push_back(t);
    if (c->oplog) c->oplog->push_back(t);
}

int nstreams(const jacc_ctx *c) { return (int)c->st.size(); }
int stream_of(const jacc_ctx *c, const Array *A, int p) { return c->serialize ? 0 : (A->home + p) % nstreams(c); }

// ---- device memory ------------------------------------------------------
int dev_alloc(jacc_ctx *c, size_t bytes, void **out) {
    if (bytes == 0) bytes = 256;
    if (c->dry && c->use_hipmalloc) {
        *out = (void *)c->fake_next;
        c->fake_next += (bytes + 4095) & ~(size_t)4095;
        return JACC_OK;
    }
    void *p = nullptr;
    if (c->use_hipmalloc) {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_err(c, JACC_ERR_ALLOC, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        }
    } else {
        p = c->alloc.alloc(bytes, c->alloc.user);
        if (!p) return set_err(c, JACC_ERR_ALLOC, "allocator returned NULL for %zu bytes", bytes);
    }
    *out = p;
    return JACC_OK;
}

void dev_free(jacc_ctx *c, void *p) {
    if (!p || (c->dry && c->use_hipmalloc)) return;
    if (c->use_hipmalloc)
        (void)hipFree(p);
    else
        c->alloc.free(p, c->alloc.user);
}

// ---- streams, events, waits ----------------------------------------------
int post_op(jacc_ctx *c) {
    if (c->serialize && live(c) && !c->cur) HIPCHK(c, hipDeviceSynchronize(), "hipDeviceSynchronize");
    return JACC_OK;
}

// Make sure an event on stream q covers its op `n`; returns the ring index.
int ensure_event(jacc_ctx *c, int q, int64_t n, int *idx) {
    StreamState &S = c->st[q];
    if (S.recorded < n) {
        EvEntry &E = S.ring[S.ring_next];
        if (live(c)) HIPCHK(c, hipEventRecord(E.ev, S.s), "hipEventRecord");
        E.covers = S.seq;
        E.waited = S.waited;
        S.recorded = S.seq;
        trace(c, JACC_OP_RECORD, q, -1, -1, -1, 0, 0, 0, S.seq);
        S.ring_next = (S.ring_next + 1) % kEventRing;
    }
    int best = -1;
    for (int i = 0; i < kEventRing; ++i) {
        const EvEntry &E = S.ring[i];
        if (E.covers >= n && (best < 0 || E.covers < S.ring[best].covers)) best = i;
    }
    *idx = best;
    return JACC_OK;
}

// Stream d must not run its next op before op n of stream q completed.
int ensure_wait(jacc_ctx *c, int d, int q, int64_t n) {
    if (d == q || n <= 0) return JACC_OK;
    StreamState &D = c->st[d];
    if (D.waited[q] >= n) return JACC_OK;
    int idx = -1;
    int rc = ensure_event(c, q, n, &idx);
    if (rc) return rc;
    if (idx < 0)
        return set_err(c, JACC_ERR_INVALID, "internal: no event of stream %d covers op %lld (recorded %lld)", q,
                       (long long)n, (long long)c->st[q].recorded);
    const EvEntry &E = c->st[q].ring[idx];
    if (live(c)) HIPCHK(c, hipStreamWaitEvent(D.s, E.ev, 0), "hipStreamWaitEvent");
    trace(c, JACC_OP_WAIT, d, -1, q, -1, 0, 0, 0, E.covers);
    D.waited[q] = std::max(D.waited[q], E.covers);
    for (size_t k = 0; k < E.waited.size(); ++k) D.waited[k] = std::max(D.waited[k], E.waited[k]);
    return JACC_OK;
}

// After a full join (around a graph launch, or at the start of a capture)
// every stream knows every op issued so far is complete, and no event
// recorded before the join is waited on afterwards.
void assume_joined(jacc_ctx *c) {
    trace(c, JACC_OP_JOIN, -1, -1, -1, -1, 0, 0, 0, 0);
    for (auto &S : c->st) S.seq++;
    for (auto &S : c->st) {
        for (size_t q = 0; q < c->st.size(); ++q) S.waited[q] = c->st[q].seq;
        for (auto &E : S.ring) E.covers = -1;
        S.recorded = S.seq;
    }
}

// Stream 0 waits for all other streams (eager events).
int join_into0(jacc_ctx *c) {
    if (!live(c)) return JACC_OK;
    for (int s = 1; s < nstreams(c); ++s) {
        HIPCHK(c, hipEventRecord(c->st[s].join_ev, c->st[s].s), "hipEventRecord");
        HIPCHK(c, hipStreamWaitEvent(c->st[0].s, c->st[s].join_ev, 0), "hipStreamWaitEvent");
    }
    return JACC_OK;
}

// All other streams wait for stream 0's current position.
int fork_from0(jacc_ctx *c) {
    if (!live(c)) return JACC_OK;
    HIPCHK(c, hipEventRecord(c->fork_ev, c->st[0].s), "hipEventRecord");
    for (int s = 1; s < nstreams(c); ++s)
        HIPCHK(c, hipStreamWaitEvent(c->st[s].s, c->fork_ev, 0), "hipStreamWaitEvent");
    return JACC_OK;
}

// Hazard bookkeeping for an access by stream s (its next op, seq+1) to rows r
// of slab p of array A.  write: RAW+WAW+WAR waits, then becomes last writer.
// wkind: how a write is traced — 2 a write, 3 values private to the slab (a
// filtered loop's writes outside the partition's owner block), 4 the value
// the same loop computes in every replica (a duplicated loop's partitions
// after the first).
int hazard(jacc_ctx *c, Array *A, int p, Range r, bool write, int s, int wkind = 2) {
    if (r.empty()) return JACC_OK;
    if (A->shared) p = 0;  // every partition's slab is the one copy
    Slab &sl = A->slabs[p];
    static thread_local std::vector<std::pair<int, int64_t>> need;  // (stream, op) to wait for
    need.clear();
    sl.acc.for_range(r, [&](IntervalMap<Access>::Piece &pc) {
        if (pc.val.ws >= 0 && pc.val.ws != s) need.push_back({pc.val.ws, pc.val.wseq});
        if (write)
            for (int k = 0; k < pc.val.reads.size(); ++k) {
                const auto &rd = pc.val.reads[k];
                if (rd.first != s) need.push_back({rd.first, rd.second});
            }
    });
    for (auto &w : need) {
        int rc = ensure_wait(c, s, w.first, w.second);
        if (rc) return rc;
    }
    const int64_t next = c->st[s].seq + 1;
    sl.acc.for_range(r, [&](IntervalMap<Access>::Piece &pc) {
        if (write) {
            pc.val.ws = s;
            pc.val.wseq = next;
            pc.val.reads.clear();
        } else {
            // recorded even when s is the last writer: a later write from
            // another stream (a mirror store) must still wait for this read
            bool found = false;
            for (int k = 0; k < pc.val.reads.size(); ++k) {
                auto &rd = pc.val.reads[k];
                if (rd.first == s) {
                    rd.second = next;
                    found = true;
                }
            }
            if (!found) pc.val.reads.push_back({s, next});
        }
    });
    sl.acc.coalesce();
    trace(c, JACC_OP_ACCESS, s, A->id, -1, p, write ? wkind : 1, r.lo, r.hi, next);
    return JACC_OK;
}

bool inject_fault(jacc_ctx *c, int kind) {
    if (c->fault_kind != kind || c->plan_only) return false;
    return ++c->fault_count == c->fault_n;
}

// ---- present table --------------------------------------------------------
Array *lookup(jacc_ctx *c, const void *host) {
    uintptr_t a = (uintptr_t)host;
    auto it = c->present.upper_bound(a);
    if (it == c->present.begin()) return nullptr;
    --it;
    Array *A = it->second;
    return (a >= A->host && a < A->host + A->bytes) ? A : nullptr;
}

// ---- copies ------------------------------------------------------------
// Copy rows r of array A from slab q to slab p, on stream s.
// Moves rows r between the host array and slab p (dir 1 host to device, 2
// device to host) or from slab q to slab p (dir 3) on stream s.  A part_dim
// 0 array's rows are contiguous in both; a part_dim 1 array's rows are
// columns: a strided 2-D copy of (r.hi - r.lo) elements from each of its
// extent[0] rows, with the host's row pitch and each slab's own.
int move_rows(jacc_ctx *c, Array *A, int dir, int q, int p, Range r, int s) {
    if (!live(c) || r.empty()) return JACC_OK;
    if (r.lo < 0 || r.hi > A->E) return set_err(c, JACC_ERR_INVALID, "internal: rows outside array %d", A->id);
    auto inside = [&](int pp) { return r.lo >= A->slabs[pp].rows.lo && r.hi <= A->slabs[pp].rows.hi; };
    if ((dir != 1 && !inside(q)) || (dir != 2 && !inside(p)))
        return set_err(c, JACC_ERR_INVALID, "internal: rows [%lld,%lld) outside a slab of array %d", (long long)r.lo,
                       (long long)r.hi, A->id);
    const hipMemcpyKind kind =
        dir == 1 ? hipMemcpyHostToDevice : dir == 2 ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    const size_t unit = A->pdim == 0 ? A->row_bytes : A->esize;  // bytes of a row within one line
    auto slab_ptr = [&](int pp) { return (char *)A->slabs[pp].dev + (size_t)(r.lo - A->slabs[pp].base) * unit; };
    char *host = (char *)A->host + (size_t)r.lo * unit;
    char *src = dir == 1 ? host : slab_ptr(q);
    char *dst = dir == 2 ? host : slab_ptr(p);
    if (A->pdim == 0) {
        HIPCHK(c, hipMemcpyAsync(dst, src, (size_t)(r.hi - r.lo) * unit, kind, c->st[s].s), "hipMemcpyAsync");
    } else {
        const size_t host_pitch = (size_t)A->d.extent[1] * A->esize;
        auto pitch = [&](int pp) { return (size_t)A->slabs[pp].pitch * A->esize; };
        const size_t spitch = dir == 1 ? host_pitch : pitch(q);
        const size_t dpitch = dir == 2 ? host_pitch : pitch(p);
        HIPCHK(c, hipMemcpy2DAsync(dst, dpitch, src, spitch, (size_t)(r.hi - r.lo) * A->esize, (size_t)A->d.extent[0],
                                   kind, c->st[s].s),
               "hipMemcpy2DAsync");
    }
    return JACC_OK;
}

int issue_copy(jacc_ctx *c, Array *A, int q, int p, Range r, int s) {
    int rc = hazard(c, A, q, r, false, s);
    if (rc) return rc;
    rc = hazard(c, A, p, r, true, s);
    if (rc) return rc;
    if (inject_fault(c, 1)) {
        c->status = JACC_ERR_DEVICE;
        return set_err(c, JACC_ERR_DEVICE, "injected fault in copy %lld", (long long)c->fault_count);
    }
    rc = move_rows(c, A, 3, q, p, r, s);
    if (rc) return rc;
    c->log_copies++;
    c->log_copy_bytes += (r.hi - r.lo) * (int64_t)(A->pdim == 0 ? A->row_bytes : A->esize * A->d.extent[0]);
    c->st[s].seq++;
    trace(c, JACC_OP_COPY, s, A->id, q, p, 0, r.lo, r.hi, c->st[s].seq);
    return post_op(c);
}

// Fills stale rows r of slab p with NaN bytes on stream s, ordered like a
// write to them (JACC_INIT_POISON); the rows stay stale.
int poison_rows(jacc_ctx *c, Array *A, int p, Range r, int s) {
    if (r.empty()) return JACC_OK;
    int rc = hazard(c, A, p, r, true, s, 5);
    if (rc) return rc;
    if (live(c)) {
        const Slab &S = A->slabs[p];
        const size_t unit = A->pdim == 0 ? A->row_bytes : A->esize;
        char *at = (char *)S.dev + (size_t)(r.lo - S.base) * unit;
        const size_t width = (size_t)(r.hi - r.lo) * unit;
        HIPCHK(c,
               A->pdim == 0 ? jk::launch_poison(at, width, width, 1, c->st[s].s)
                            : jk::launch_poison(at, (size_t)S.pitch * A->esize, width, A->d.extent[0], c->st[s].s),
               "poison fill");
    }
    c->st[s].seq++;
    trace(c, JACC_OP_POISON, s, A->id, -1, p, 0, r.lo, r.hi, c->st[s].seq);
    return post_op(c);
}

// Pull into slab p (on stream s) every row of `need` it does not hold fresh.
int make_fresh(jacc_ctx *c, Array *A, int p, Range need, int s) {
    if (need.empty()) return JACC_OK;
    std::vector<Range> miss = A->valid[p].missing(need);
    for (const Range &m : miss) {
        std::vector<std::pair<int, Range>> pieces;
        A->writer.for_range(m, [&](IntervalMap<int32_t>::Piece &pc) { pieces.push_back({pc.val, {pc.lo, pc.hi}}); });
        A->writer.coalesce();
        for (auto &pc : pieces) {
            int q = pc.first;
            if (q < 0 || q == p)
                return set_err(c, JACC_ERR_INVALID, "internal: rows [%lld,%lld) of array %d stale with no writer",
                               (long long)pc.second.lo, (long long)pc.second.hi, A->id);
            int rc = issue_copy(c, A, q, p, pc.second, s);
            if (rc) return rc;
        }
        A->valid[p].add(m);
    }
    return JACC_OK;
}

void note_write(Array *A, int p, Range w) {
    if (w.empty()) return;
    ++A->version;
    A->writer.assign(w, p);
    for (int q = 0; q < A->K; ++q) {
        if (q == p)
            A->valid[q].add(w);
        else
            A->valid[q].sub(w);
    }
}

// Rows every replica computed alike (a duplicated loop): valid in every
// holder, with no single latest writer.
void note_everywhere(Array *A, Range w) {
    if (w.empty()) return;
    ++A->version;
    A->writer.assign(w, -1);
    for (int q = 0; q < A->K; ++q) A->valid[q].add(w);
}

// Source of each row for gathers: the last writer, else the block owner.
template <class F>
void for_owner_pieces(Array *A, Range r, F f) {
    std::vector<std::pair<int, Range>> pieces;
    A->writer.for_range(r, [&](IntervalMap<int32_t>::Piece &pc) { pieces.push_back({pc.val, {pc.lo, pc.hi}}); });
    A->writer.coalesce();
    for (auto &pc : pieces) {
        if (pc.first >= 0) {
            f(pc.first, pc.second);
            continue;
        }
        if (A->whole) {
            f(0, pc.second);
            continue;
        }
        for (int p = 0; p < A->K; ++p) {
            Range x = isect(pc.second, A->block(p));
            if (!x.empty()) f(p, x);
        }
    }
}

int sync_stream(jacc_ctx *c, int s) {
    if (live(c)) HIPCHK(c, hipStreamSynchronize(c->st[s].s), "hipStreamSynchronize");
    trace(c, JACC_OP_SYNC, s, -1, -1, -1, 0, 0, 0, c->st[s].seq);
    return JACC_OK;
}

int sync_all(jacc_ctx *c) {
    for (int s = 0; s < nstreams(c); ++s) {
        int rc = sync_stream(c, s);
        if (rc) return rc;
    }
    return JACC_OK;
}

int h2d_rows(jacc_ctx *c, Array *A, int p, Range r) {
    const int s = stream_of(c, A, p);
    int rc = hazard(c, A, p, r, true, s);
    if (rc) return rc;
    ++A->version;
    rc = move_rows(c, A, 1, -1, p, r, s);
    if (rc) return rc;
    c->st[s].seq++;
    trace(c, JACC_OP_H2D, s, A->id, -1, p, 0, r.lo, r.hi, c->st[s].seq);
    return post_op(c);
}

int d2h_rows(jacc_ctx *c, Array *A, int p, Range r) {
    const int s = stream_of(c, A, p);
    int rc = hazard(c, A, p, r, false, s);
    if (rc) return rc;
    rc = move_rows(c, A, 2, p, -1, r, s);
    if (rc) return rc;
    c->st[s].seq++;
    trace(c, JACC_OP_D2H, s, A->id, p, -1, 0, r.lo, r.hi, c->st[s].seq);
    return post_op(c);
}

int gather(jacc_ctx *c, Array *A, Range r) {
    std::vector<char> used(c->st.size(), 0);
    int rc = JACC_OK;
    for_owner_pieces(A, r, [&](int p, Range x) {
        if (rc) return;
        rc = d2h_rows(c, A, p, x);
        used[stream_of(c, A, p)] = 1;
    });
    if (rc) return rc;
    for (size_t s = 0; s < used.size(); ++s)
        if (used[s]) {
            rc = sync_stream(c, (int)s);
            if (rc) return rc;
        }
    return JACC_OK;
}

void drop_bands(jacc_ctx *c, int array_id) {
    for (size_t i = 0; i < c->bands.size();) {
        BandCache &bc = c->bands[i];
        if (array_id < 0 || bc.rp_id == array_id || bc.col_id == array_id || bc.val_id == array_id) {
            for (void *m : bc.mem) dev_free(c, m);
            c->bands.erase(c->bands.begin() + (long)i);
        } else {
            ++i;
        }
    }
}

void free_array(jacc_ctx *c, Array *A) {
    drop_bands(c, A->id);
    for (int p = 0; p < (A->shared ? 1 : A->K); ++p) {
        trace(c, JACC_OP_FREE, -1, A->id, -1, p, 0, A->slabs[p].rows.lo, A->slabs[p].rows.hi, 0);
        dev_free(c, A->slabs[p].dev);
    }
    delete A;
}

bool desc_equal(const jacc_array_desc &a, const jacc_array_desc &b) {
    if (a.dtype != b.dtype || a.ndim != b.ndim || a.halo_lo != b.halo_lo || a.halo_hi != b.halo_hi ||
        a.whole != b.whole || a.num_partitions != b.num_partitions || a.part_dim != b.part_dim)
        return false;
    for (int i = 0; i < a.ndim; ++i)
        if (a.extent[i] != b.extent[i]) return false;
    return true;
}

// ---- persistent task groups ------------------------------------------------
// Launches the pending persistent tasks as one persistent kernel on stream 0:
// a grid sized to the chip walks all tasks' tiles, reading the task records
// from the batch's device table.
int flush_group(jacc_ctx *c) {
    if (c->ptasks.empty()) return JACC_OK;
    Batch *B = c->cur;
    const int s = 0;
    const int n = (int)c->ptasks.size();
    if (!B || B->tasks_used + n > kTaskCapacity)
        return set_err(c, JACC_ERR_UNSUPPORTED, "more than %d persistent tasks in one batch", kTaskCapacity);
    for (const PendingAccess &a : c->paccs) {
        int rc = hazard(c, a.A, a.p, a.r, a.write, s);
        if (rc) return rc;
    }
    int64_t tiles = 0;
    bool jacobi_only = true;
    for (auto &t : c->ptasks) {
        t.tile_begin = tiles;
        tiles += t.ntiles;
        jacobi_only = jacobi_only && t.kind == JACC_LOOP_JACOBI2D;
    }
    if (live(c)) {
        const int64_t grid = jk::persistent_grid(tiles, jacobi_only);
        // the table is written to pinned memory now and uploaded once when
        // the batch closes, before the graph first runs
        std::memcpy(B->host_tasks + B->tasks_used, c->ptasks.data(), (size_t)n * sizeof(jk::PTask));
        HIPCHK(c, jk::launch_persistent(B->dev_tasks + B->tasks_used, n, tiles, grid, jacobi_only, c->st[s].s),
               "persistent kernel launch");
    }
    B->tasks_used += n;
    B->groups++;
    c->st[s].seq++;
    trace(c, JACC_OP_KERNEL, s, -1, -1, -1, -n, 0, tiles, c->st[s].seq);
    c->ptasks.clear();
    c->paccs.clear();
    c->parrays.clear();
    return JACC_OK;
}

bool pending_touches(const jacc_ctx *c, const Array *A) {
    for (const Array *x : c->parrays)
        if (x == A) return true;
    return false;
}

// ---- loop kinds: argument tables --------------------------------------------
struct KindInfo {
    int nargs;
    int ndim;
    int red;  // 0 none, 1 optional, 2 required
};

bool kind_info(int kind, KindInfo *k) {
    switch (kind) {
        case JACC_LOOP_JACOBI2D: *k = {2, 2, 0}; return true;
        case JACC_LOOP_HEAT3D: *k = {2, 3, 1}; return true;
        case JACC_LOOP_SUM: *k = {1, 1, 2}; return true;
        case JACC_LOOP_GEMM: *k = {3, 2, 0}; return true;
        case JACC_LOOP_SPMV_CSR: *k = {5, 1, 0}; return true;
        case JACC_LOOP_SCATTER_SQ: *k = {3, 1, 0}; return true;
        case JACC_LOOP_PRED_CHAIN: *k = {5, 1, 0}; return true;
        default: return false;
    }
}

struct PartPlan {
    Range iters;
    std::vector<Range> rng;  // per argument
};

#define GUARD(c)                           \
    do {                                   \
        if (!(c)) return JACC_ERR_INVALID; \
        if ((c)->status) {                 \
            return JACC_ERR_DEVICE;        \
        }                                  \
    } while (0)

// Validates a loop call and builds its launch template and per-partition
// plan.  On success *primary_out is the argument whose owner blocks split
// the iterations (the written array; the read array for SUM).
int prepare_loop(jacc_ctx *c, int kind, const jacc_bounds *b, int nargs, const jacc_arg *args, const double *scalars,
                 int nscalars, bool want_red, const jacc_config *cfg, Array **arr, jk::Launch &L,
                 std::vector<PartPlan> &plan, int *primary_out, bool *dup_out) {
    KindInfo ki;
    if (!kind_info(kind, &ki)) return set_err(c, JACC_ERR_INVALID, "unknown loop kind %d", kind);
    if (!b || nargs != ki.nargs || !args)
        return set_err(c, JACC_ERR_INVALID, "loop kind %d takes %d arguments and bounds", kind, ki.nargs);
    if (b->ndim != ki.ndim) return set_err(c, JACC_ERR_INVALID, "loop kind %d takes %d-D bounds", kind, ki.ndim);
    for (int d = 0; d < b->ndim; ++d)
        if (b->lo[d] < 0 || b->hi[d] < b->lo[d]) return set_err(c, JACC_ERR_INVALID, "bad bounds in dim %d", d);
    if (nscalars < 0 || nscalars > 4 || (nscalars > 0 && !scalars)) return set_err(c, JACC_ERR_INVALID, "bad scalars");
    if (ki.red == 0 && want_red) return set_err(c, JACC_ERR_INVALID, "loop kind %d has no reduction", kind);
    if (ki.red == 2 && !want_red) return set_err(c, JACC_ERR_INVALID, "loop kind %d needs a reduction target", kind);
    if (kind == JACC_LOOP_HEAT3D && nscalars < 1) return set_err(c, JACC_ERR_INVALID, "HEAT3D needs alpha");

    int K = -1;
    for (int i = 0; i < nargs; ++i) {
        if (args[i].mode < JACC_READ || args[i].mode > (JACC_READWRITE | JACC_FILTERED) ||
            ((args[i].mode & JACC_FILTERED) && !(args[i].mode & JACC_WRITE)))
            return set_err(c, JACC_ERR_INVALID, "argument %d: bad mode", i);
        if (args[i].off_lo > args[i].off_hi) return set_err(c, JACC_ERR_INVALID, "argument %d: off_lo > off_hi", i);
        Array *A = lookup(c, args[i].host);
        if (!A) return set_err(c, JACC_ERR_NOT_PRESENT, "argument %d (%p) is not present", i, args[i].host);
        if ((uintptr_t)args[i].host != A->host)
            return set_err(c, JACC_ERR_UNSUPPORTED, "argument %d is an interior pointer of array %d", i, A->id);
        if (K < 0) K = A->K;
        if (A->K != K) return set_err(c, JACC_ERR_UNSUPPORTED, "arguments are partitioned with different K");
        if ((args[i].mode & JACC_WRITE) && A->shared)
            return set_err(c, JACC_ERR_INVALID, "argument %d writes array %d, entered as one shared read-only copy",
                           i, A->id);
        arr[i] = A;
    }
    // arrays split along dimension 1 (column blocks) take the 2-D stencil
    // only, with every argument split the same way
    const int pd = arr[0]->pdim;
    for (int i = 1; i < nargs; ++i)
        if (arr[i]->pdim != pd)
            return set_err(c, JACC_ERR_UNSUPPORTED, "arguments are partitioned along different dimensions");
    if (pd != 0 && kind != JACC_LOOP_JACOBI2D)
        return set_err(c, JACC_ERR_UNSUPPORTED, "loop kind %d does not take arrays split along dimension %d", kind, pd);
    auto is = [&](int i, int dt, int nd) { return arr[i]->d.dtype == dt && arr[i]->d.ndim == nd; };
    L = jk::Launch{};
    L.kind = kind;
    L.ndim = b->ndim;
    L.nargs = nargs;
    for (int i = 0; i < nscalars; ++i) L.scalars[i] = scalars[i];
    for (int i = 0; i < 4; ++i) L.ext[i] = arr[0]->d.ndim > i ? arr[0]->d.extent[i] : 0;
    int primary = -1;
    switch (kind) {
        case JACC_LOOP_JACOBI2D:
            if (!is(0, JACC_F64, 2) || !is(1, JACC_F64, 2) || arr[0]->d.extent[0] != arr[1]->d.extent[0] ||
                arr[0]->d.extent[1] != arr[1]->d.extent[1])
                return set_err(c, JACC_ERR_INVALID, "JACOBI2D takes two FP64 2-D arrays of equal shape");
            if (b->hi[0] > arr[0]->d.extent[0] - 1 || b->lo[0] < 1 || b->lo[1] < 1 ||
                b->hi[1] > arr[0]->d.extent[1] - 1)
                return set_err(c, JACC_ERR_RANGE, "JACOBI2D bounds must lie inside the interior");
            primary = 1;
            break;
        case JACC_LOOP_HEAT3D:
            if (!is(0, JACC_F64, 3) || !is(1, JACC_F64, 3))
                return set_err(c, JACC_ERR_INVALID, "HEAT3D takes two FP64 3-D arrays");
            for (int d = 0; d < 3; ++d)
                if (arr[0]->d.extent[d] != arr[1]->d.extent[d])
                    return set_err(c, JACC_ERR_INVALID, "HEAT3D arrays differ in shape");
            for (int d = 0; d < 3; ++d)
                if (b->lo[d] < 1 || b->hi[d] > arr[0]->d.extent[d] - 1)
                    return set_err(c, JACC_ERR_RANGE, "HEAT3D bounds must lie inside the interior");
            primary = 1;
            break;
        case JACC_LOOP_SUM:
            if (arr[0]->d.dtype != JACC_F64) return set_err(c, JACC_ERR_INVALID, "SUM takes an FP64 array");
            if (b->hi[0] > arr[0]->E) return set_err(c, JACC_ERR_RANGE, "SUM bounds exceed the array");
            primary = 0;
            break;
        case JACC_LOOP_GEMM:
            if (!is(0, JACC_F64, 2) || !is(1, JACC_F64, 2) || !is(2, JACC_F64, 2))
                return set_err(c, JACC_ERR_INVALID, "GEMM takes three FP64 2-D arrays");
            if (arr[0]->d.extent[1] != arr[1]->d.extent[0] || arr[0]->d.extent[0] != arr[2]->d.extent[0] ||
                arr[1]->d.extent[1] != arr[2]->d.extent[1])
                return set_err(c, JACC_ERR_INVALID, "GEMM shapes do not conform");
            if (b->hi[0] > arr[2]->d.extent[0] || b->hi[1] > arr[2]->d.extent[1])
                return set_err(c, JACC_ERR_RANGE, "GEMM bounds exceed C");
            primary = 2;
            break;
        case JACC_LOOP_SPMV_CSR:
            if (!is(0, JACC_I32, 1) || !is(1, JACC_I32, 1) || !is(2, JACC_F64, 1) || !is(3, JACC_F64, 1) ||
                !is(4, JACC_F64, 1))
                return set_err(c, JACC_ERR_INVALID, "SPMV_CSR takes int32 row_ptr, int32 col, f64 val, x, y");
            if (arr[0]->E != arr[4]->E + 1 || arr[1]->E != arr[2]->E)
                return set_err(c, JACC_ERR_INVALID, "SPMV_CSR: row_ptr must have n+1 entries and col/val match");
            if (b->hi[0] > arr[4]->E) return set_err(c, JACC_ERR_RANGE, "SPMV_CSR bounds exceed y");
            primary = 4;
            break;
        case JACC_LOOP_SCATTER_SQ:
            if (!is(0, JACC_F64, 1) || !is(1, JACC_I32, 1) || !is(2, JACC_F64, 1))
                return set_err(c, JACC_ERR_INVALID, "SCATTER_SQ takes f64 in, int32 idx, f64 out");
            if (arr[0]->E != arr[1]->E) return set_err(c, JACC_ERR_INVALID, "SCATTER_SQ: in and idx differ in length");
            if (!(args[2].mode & JACC_FILTERED))
                return set_err(c, JACC_ERR_INVALID, "SCATTER_SQ writes out through indices: declare it FILTERED");
            if (!args[0].whole || !args[1].whole)
                return set_err(c, JACC_ERR_INVALID, "SCATTER_SQ reads in and idx whole");
            if (b->hi[0] > arr[0]->E) return set_err(c, JACC_ERR_RANGE, "SCATTER_SQ bounds exceed in");
            primary = 2;
            break;
        case JACC_LOOP_PRED_CHAIN:
            if (!is(0, JACC_F64, 1) || !is(1, JACC_F64, 1) || !is(2, JACC_F64, 1) || !is(3, JACC_I32, 2) ||
                !is(4, JACC_F64, 1) || arr[3]->d.extent[1] != 3)
                return set_err(c, JACC_ERR_INVALID, "PRED_CHAIN takes f64 a, b, c, int32 idx (T x 3) and f64 xs (T)");
            if (arr[3]->E != arr[4]->E) return set_err(c, JACC_ERR_INVALID, "PRED_CHAIN: idx and xs differ in length");
            for (int i = 0; i < 2; ++i)
                if (!(args[i].mode & JACC_FILTERED) || !arr[i]->whole)
                    return set_err(c, JACC_ERR_INVALID,
                                   "PRED_CHAIN writes a and b FILTERED into arrays entered whole (replicated)");
            for (int i = 2; i < 5; ++i)
                if (!args[i].whole) return set_err(c, JACC_ERR_INVALID, "PRED_CHAIN reads c, idx and xs whole");
            if (b->hi[0] > arr[3]->E) return set_err(c, JACC_ERR_RANGE, "PRED_CHAIN bounds exceed idx");
            primary = 0;
            break;
    }
    if (!(args[primary].mode & JACC_WRITE) && kind != JACC_LOOP_SUM)
        return set_err(c, JACC_ERR_INVALID, "the output argument must be declared writable");

    Array *P = arr[primary];
    // Aliasing: one array in two argument positions, one of them written (the
    // paper's aliased pointers).  The partition ranges cannot be trusted; with
    // every array replicated the loop runs duplicated (each partition computes
    // everything on its own replicas, unfiltered, and nothing moves after it),
    // otherwise it is refused.
    bool aliased = false, all_whole = true;
    for (int i = 0; i < nargs; ++i) {
        all_whole = all_whole && arr[i]->whole;
        for (int j = 0; j < i; ++j)
            if (arr[i] == arr[j] && ((args[i].mode | args[j].mode) & JACC_WRITE)) aliased = true;
    }
    if (aliased && !all_whole)
        return set_err(c, JACC_ERR_RANGE,
                       "an argument array is aliased (read and written through two arguments) and not entered "
                       "whole: duplicated execution needs replicas");
    const bool dup = aliased;
    *dup_out = dup;
    // A filtered output is written through data-dependent indices: every
    // partition runs the whole iteration space (the write-index arithmetic is
    // duplicated) and keeps the writes that land in its owner block.  A
    // filtered output entered whole is divided into owner blocks like a
    // partitioned one; its replicas hold every row.
    const bool filtered = (args[primary].mode & JACC_FILTERED) != 0;
    if (pd != 0 && filtered)
        return set_err(c, JACC_ERR_UNSUPPORTED, "a filtered output split along dimension %d", pd);
    const Range all_iters{b->lo[pd], b->hi[pd]};  // iterations along the partitioned dimension
    plan.assign(K, PartPlan{});
    for (int p = 0; p < K; ++p) {
        Range own = (P->whole && !filtered) ? (p == 0 ? Range{0, P->E} : Range{0, 0}) : P->block(p);
        plan[p].iters = (filtered || dup) ? all_iters : isect(all_iters, own);
        if (filtered && !dup && own.empty()) plan[p].iters = Range{};
        plan[p].rng.resize(nargs);
        for (int i = 0; i < nargs; ++i) {
            Range r{};
            if (!plan[p].iters.empty()) {
                if (args[i].whole || dup)
                    r = {0, arr[i]->E};
                else if (args[i].mode & JACC_FILTERED)
                    r = arr[i]->block(p);
                else
                    r = isect({plan[p].iters.lo + args[i].off_lo, plan[p].iters.hi - 1 + args[i].off_hi + 1},
                              {0, arr[i]->E});
            }
            plan[p].rng[i] = r;
            if (r.empty()) continue;
            const Range sl = arr[i]->slabs[p].rows;
            if (r.lo < sl.lo || r.hi > sl.hi)
                return set_err(c, JACC_ERR_RANGE,
                               "partition %d: argument %d touches rows [%lld,%lld) outside its slab [%lld,%lld)", p, i,
                               (long long)r.lo, (long long)r.hi, (long long)sl.lo, (long long)sl.hi);
            if ((args[i].mode & JACC_WRITE) && !arr[i]->whole) {
                Range own_i = arr[i]->block(p);
                if (r.lo < own_i.lo || r.hi > own_i.hi)
                    return set_err(c, JACC_ERR_RANGE,
                                   "partition %d: argument %d writes rows [%lld,%lld) outside its owner block", p, i,
                                   (long long)r.lo, (long long)r.hi);
            }
        }
    }
    // one array written by two partitions, or read by one partition where
    // another writes it in the same loop (the paper duplicates such loops)
    for (int i = 0; i < nargs && !dup; ++i) {
        if (!(args[i].mode & JACC_WRITE)) continue;
        for (int j = 0; j < nargs; ++j) {
            if (arr[j] != arr[i]) continue;
            for (int p = 0; p < K; ++p)
                for (int q = 0; q < K; ++q) {
                    if (p == q) continue;
                    if (!isect(plan[p].rng[i], plan[q].rng[j]).empty())
                        return set_err(c, JACC_ERR_RANGE,
                                       "partitions %d and %d overlap on array %d (aliased write ranges)", p, q,
                                       arr[i]->id);
                }
        }
    }
    jk::Cfg cf{0, 0, 0, 0, 0, 0, 0, 0};
    L.part_rows = 0;
    for (const PartPlan &pp : plan)
        L.part_rows = std::max(L.part_rows, pd == 0 ? pp.iters.hi - pp.iters.lo
                                                    : (pp.iters.empty() ? 0 : b->hi[0] - b->lo[0]));
    if (cfg) cf = {cfg->bx, cfg->by, cfg->tile, cfg->vec, cfg->persistent, cfg->order, cfg->march, cfg->rows};
    if (pd != 0 && cf.persistent)
        return set_err(c, JACC_ERR_UNSUPPORTED, "persistent execution of arrays split along dimension 1");
    L.cfg = jk::default_config(kind, L, cf);
    if (kind == JACC_LOOP_SPMV_CSR && !cf.order && !c->cur && arr[3]->E >= kBandedMinCols) {
        // x far larger than an XCD's L2: the column-banded form, one band
        // per XCD, two lanes per row and band (measured at 2^22 columns)
        L.cfg.order = 4;
        if (!cf.tile) L.cfg.tile = 2;
        if (!cf.by) L.cfg.by = 1;
    }
    if (jk::check_config(L) != 0)
        return set_err(c, JACC_ERR_INVALID,
                       "configuration bx=%d by=%d tile=%d vec=%d persistent=%d order=%d march=%d rows=%d not valid for kind %d",
                       L.cfg.bx, L.cfg.by, L.cfg.tile, L.cfg.vec, L.cfg.persistent, L.cfg.order, L.cfg.march,
                       L.cfg.rows, kind);
    if (kind == JACC_LOOP_SPMV_CSR && L.cfg.order == 4 && c->cur)
        return set_err(c, JACC_ERR_UNSUPPORTED, "the column-banded SpMV form is not captured in batches");
    if (L.cfg.persistent) {
        if (!c->cur) return set_err(c, JACC_ERR_INVALID, "persistent execution needs an open batch");
        if (want_red) return set_err(c, JACC_ERR_UNSUPPORTED, "persistent execution of a reduction");
        if (args[primary].mode & JACC_FILTERED)
            return set_err(c, JACC_ERR_UNSUPPORTED, "persistent execution of a filtered loop");
    }
    *primary_out = primary;
    return JACC_OK;
}

// The banded copy of partition p's rows of the CSR matrix in arr[0..2]
// (row_ptr, col, val) for x = arr[3]: found, marked for a rebuild when the
// matrix changed since it was built, or allocated.
int band_cache(jacc_ctx *c, Array **arr, int p, Range rows, int bands, BandCache **out) {
    Array *rp = arr[0], *col = arr[1], *val = arr[2];
    for (BandCache &bc : c->bands)
        if (bc.rp_id == rp->id && bc.col_id == col->id && bc.val_id == val->id && bc.p == p && bc.lo == rows.lo &&
            bc.hi == rows.hi && bc.bands == bands) {
            if (bc.v_rp != rp->version || bc.v_col != col->version || bc.v_val != val->version) {
                bc.built = false;
                bc.v_rp = rp->version;
                bc.v_col = col->version;
                bc.v_val = val->version;
            }
            *out = &bc;
            return JACC_OK;
        }
    const int64_t n = rows.hi - rows.lo, len = (int64_t)bands * n;
    const int64_t nb = jk::band_scan_blocks(len);
    if (nb > 8192) return set_err(c, JACC_ERR_UNSUPPORTED, "banded SpMV: %lld band rows exceed the scan", (long long)len);
    BandCache bc;
    bc.rp_id = rp->id;
    bc.col_id = col->id;
    bc.val_id = val->id;
    bc.p = p;
    bc.bands = bands;
    bc.lo = rows.lo;
    bc.hi = rows.hi;
    bc.v_rp = rp->version;
    bc.v_col = col->version;
    bc.v_val = val->version;
    const size_t sizes[5] = {(size_t)(len + 1) * 4, (size_t)(nb + 1) * 4, (size_t)col->E * 4, (size_t)col->E * 8,
                             (size_t)len * 8};
    for (int i = 0; i < 5; ++i) {
        int rc = dev_alloc(c, sizes[i], &bc.mem[i]);
        if (rc) {
            for (int j = 0; j < i; ++j) dev_free(c, bc.mem[j]);
            return rc;
        }
    }
    bc.bb.bands = bands;
    bc.bb.ncols = arr[3]->E;
    bc.bb.bptr = (int32_t *)bc.mem[0];
    bc.bb.sums = (int32_t *)bc.mem[1];
    bc.bb.bcol = (int32_t *)bc.mem[2];
    bc.bb.bval = (double *)bc.mem[3];
    bc.bb.part = (double *)bc.mem[4];
    c->bands.push_back(bc);
    *out = &c->bands.back();
    return JACC_OK;
}

// What a loop call did, for its JACC_LOG record.
struct LoopNote {
    int K = 0, nrun = 0;
    bool packed = false;
    jk::Cfg cfg{};
    double cells = 0;  // iterations of the box
    double work = 0;   // algorithmic bytes (flop for GEMM); 0 where none is defined
    bool flop = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;  // around the loop's work on its one stream
};

int loop_impl(jacc_ctx *c, int kind, const jacc_bounds *b, int nargs, const jacc_arg *args, const double *scalars,
              int nscalars, int slot, double *red_host, const jacc_config *cfg, LoopNote *note = nullptr) {
    const bool want_red = slot >= 0 || red_host;
    jacc_config picked;
    if (!cfg && c->tune_mode != 1 && (kind == JACC_LOOP_JACOBI2D || kind == JACC_LOOP_HEAT3D) && nargs == 2 &&
        args) {
        // no configuration given: the attached cost model's pick for this
        // loop on its arrays' partitions, or (JACC_TUNE=exhaustive) the
        // tuner's, each cached per loop signature; arrays split along
        // dimension 1 keep the defaults
        Array *W = lookup(c, args[1].host);
        if (W && W->host == (uintptr_t)args[1].host && W->pdim == 0) {
            if (c->tune_mode == 2) {
                if (jr::tuned_config(c, kind, b, nargs, args, scalars, nscalars, &picked)) cfg = &picked;
            } else if (c->model && jr::model_config(c, kind, W->d.extent, W->d.ndim, W->K, &picked)) {
                cfg = &picked;
            }
        }
    }
    if (slot >= kSlots) return set_err(c, JACC_ERR_INVALID, "reduction slot %d out of range", slot);
    if (red_host && c->cur) return set_err(c, JACC_ERR_INVALID, "a synchronous reduction inside a batch");
    Array *arr[8];
    jk::Launch L;
    std::vector<PartPlan> plan;
    int primary = -1;
    bool dup = false;
    int rc;
    {
        Marker mk(c, "jacc plan kind=%d", kind);
        rc = prepare_loop(c, kind, b, nargs, args, scalars, nscalars, want_red, cfg, arr, L, plan, &primary, &dup);
    }
    if (rc) return rc;
    Marker mk_issue(c, "jacc issue kind=%d K=%d", kind, arr[0]->K);
    const bool persistent = L.cfg.persistent != 0;
    // a pending persistent group is launched before anything that touches
    // its arrays; loops on other arrays (persistent or not) go ahead of it,
    // so the small loops of a batch gather into few launches whatever the
    // order they are issued in
    bool conflict = false;
    for (int i = 0; i < nargs && !conflict; ++i) conflict = pending_touches(c, arr[i]);
    if (conflict) {
        rc = flush_group(c);
        if (rc) return rc;
    }
    if (c->cur && !c->plan_only) {
        for (int i = 0; i < nargs; ++i)
            if (std::find(c->cur->array_ids.begin(), c->cur->array_ids.end(), arr[i]->id) == c->cur->array_ids.end())
                c->cur->array_ids.push_back(arr[i]->id);
        LoopCall lc;
        lc.kind = kind;
        lc.b = *b;
        lc.args.assign(args, args + nargs);
        lc.scalars.assign(scalars, scalars + nscalars);
        lc.slot = slot;
        lc.has_cfg = cfg != nullptr;
        if (cfg) lc.cfg = *cfg;
        c->cur->calls.push_back(lc);
    }
    Array *P = arr[primary];
    const int K = P->K;
    // Streams: with one partition per stream, partition p runs on stream p.
    // With fewer partitions than streams the loop goes where its data was
    // last produced (a dependent loop stays on the same queue), and a loop
    // with no device-side producer takes the least recently used stream —
    // the queue choice of the paper's automated asynchronous execution.
    int base = 0;
    const int ns = nstreams(c);
    if (K < ns && !c->serialize) {
        base = -1;
        for (int i = 0; i < nargs && base < 0; ++i)
            if ((args[i].mode & JACC_READ) && arr[i]->last_stream >= 0) base = arr[i]->last_stream;
        if (base < 0) base = P->last_stream;
        if (base < 0) {
            base = 0;
            for (int s = 1; s < ns; ++s)
                if (c->st[s].last_use < c->st[base].last_use) base = s;
        }
    }
    // inside a batch everything is captured on stream 0 (a single-stream
    // graph); the partitions of a stencil step become tiles of one
    // persistent launch when the configuration asks for it
    const bool one_stream = c->serialize || (c->cur != nullptr && !c->fork_capture);
    // packed: outside batches, the partitions of a stencil loop run in one
    // launch on one stream, each partition's tiles a run of its workgroups
    // (measured on 8192^2 Jacobi at K = 8: 5.9-6.0 TB/s, against 4.9-5.6
    // for a launch per partition on K streams, whose kernels contend for the
    // device's hardware queues); a residual's workgroup partials of all
    // partitions must fit the stream's partial buffer
    bool packed = !c->cur && !c->no_pack && !c->serialize && !c->time_parts && !c->split && K > 1 &&
                  K <= jk::kMaxPack && !persistent && !dup &&
                  (kind == JACC_LOOP_JACOBI2D || kind == JACC_LOOP_HEAT3D || kind == JACC_LOOP_SUM ||
                   (kind == JACC_LOOP_SPMV_CSR && L.cfg.order == 4 && L.cfg.rows <= 1)) &&
                  !(args[primary].mode & JACC_FILTERED) && (P->pdim == 0 || kind == JACC_LOOP_JACOBI2D) &&
                  !P->whole;
    if (packed && want_red) {
        int64_t total = 0;
        for (int p = 0; p < K; ++p) {
            if (plan[p].iters.empty()) continue;
            jk::Launch T = L;
            for (int d = 0; d < b->ndim; ++d) {
                T.lo[d] = b->lo[d];
                T.hi[d] = b->hi[d];
            }
            T.lo[0] = plan[p].iters.lo;
            T.hi[0] = plan[p].iters.hi;
            total += jk::reduction_workgroups(T);
        }
        packed = total <= kWgCapacity;
    }
    auto stream_for = [&](int p) { return (one_stream || persistent) ? 0 : (base + (packed ? 0 : p)) % ns; };
    if (note) {
        note->K = K;
        note->packed = packed;
        note->cfg = L.cfg;
        for (int p = 0; p < K; ++p) note->nrun += !plan[p].iters.empty();
        double cells = 1;
        for (int d = 0; d < b->ndim; ++d) cells *= (double)(b->hi[d] - b->lo[d]);
        note->cells = cells;
        switch (kind) {
            case JACC_LOOP_JACOBI2D:
            case JACC_LOOP_HEAT3D: note->work = 16.0 * cells; break;
            case JACC_LOOP_SUM: note->work = 8.0 * cells * (double)arr[0]->row_elems; break;
            case JACC_LOOP_GEMM:
                note->work = 2.0 * cells * (double)arr[0]->d.extent[1];
                note->flop = true;
                break;
            case JACC_LOOP_SPMV_CSR: {  // nnz of the rows from the caller's row_ptr
                const int32_t *rp = (const int32_t *)args[0].host;
                const double nnz = (double)rp[b->hi[0]] - (double)rp[b->lo[0]];
                note->work = 4.0 * (cells + 1) + 12.0 * nnz + 16.0 * cells;
                break;
            }
            case JACC_LOOP_SCATTER_SQ: note->work = 20.0 * cells; break;
            default: break;
        }
        if (c->log_times && live(c) && (packed || K == 1 || one_stream)) {
            const int s0 = stream_for(0);
            HIPCHK(c, hipEventCreate(&note->e0), "hipEventCreate");
            HIPCHK(c, hipEventCreate(&note->e1), "hipEventCreate");
            HIPCHK(c, hipEventRecord(note->e0, c->st[s0].s), "hipEventRecord");
        }
    }
    // rows of its slab a partition may write: a filtered output entered
    // whole takes private writes anywhere in the partition's replica
    int first_run = 0;  // first partition with iterations (a duplicated loop's reference replica)
    while (first_run < K - 1 && plan[first_run].iters.empty()) ++first_run;
    auto write_span = [&](int i, const PartPlan &pp) {
        return ((args[i].mode & JACC_FILTERED) && arr[i]->whole && !pp.iters.empty()) ? Range{0, arr[i]->E}
                                                                                        : pp.rng[i];
    };
    ++c->tick;
    for (int p = 0; p < K; ++p) c->st[stream_for(p)].last_use = c->tick;
    for (int i = 0; i < nargs; ++i)
        if (args[i].mode & JACC_WRITE) arr[i]->last_stream = base;
    // mirrors: a stencil partition also writes the rows of its output that
    // other slabs hold as halo (at most one neighbour block on each side)
    // (for an array split along dim 1, the JACOBI2D kernel writes the
    // columns other slabs keep: column mirrors)
    const bool can_mirror = !c->lazy && !c->eager && (kind == JACC_LOOP_JACOBI2D || kind == JACC_LOOP_HEAT3D) &&
                            !P->whole && K > 1 && (P->pdim == 0 || kind == JACC_LOOP_JACOBI2D);
    const int red_slot = slot >= 0 ? slot : kSlots - 1;  // a synchronous-only reduction uses the last slot
    std::vector<int> order;       // partitions that reduce, in partition order
    std::vector<int> red_streams;  // their streams
    // pieces: one per partition, or (split mode) first every partition's
    // rows whose reads stay inside its own block, then the edge rows that
    // read a neighbour's rows
    struct Piece {
        int p;
        PartPlan pp;
    };
    std::vector<Piece> pieces;
    // measured: splitting pays at 2-4 partitions; at 8 the extra launches
    // make the host the bottleneck, so it is then only taken on request
    // (and only for partitions of at least 2^22 cells, whose kernels outlast
    // the host cost of the extra launches)
    int64_t part_cells = L.part_rows;
    for (int d = 1; d < b->ndim; ++d) part_cells *= std::max<int64_t>(0, b->hi[d] - b->lo[d]);
    const bool auto_split = K <= 4 && !c->no_split && part_cells >= ((int64_t)1 << 22);
    const bool split = (c->split || auto_split) && !packed && !c->time_parts && !want_red && !persistent && !one_stream &&
                       K > 1 &&
                       !(args[primary].mode & JACC_FILTERED) && P->pdim == 0 &&
                       (kind == JACC_LOOP_JACOBI2D || kind == JACC_LOOP_HEAT3D);
    if (split) {
        int e = 0;  // halo depth of the reads along dim 0
        for (int i = 0; i < nargs; ++i)
            if ((args[i].mode & JACC_READ) && !args[i].whole)
                e = std::max(e, std::max(-args[i].off_lo, args[i].off_hi));
        auto piece = [&](int p, Range it) {
            Piece pc{p, PartPlan{}};
            pc.pp.iters = it;
            pc.pp.rng.resize(nargs);
            for (int i = 0; i < nargs; ++i)
                pc.pp.rng[i] = args[i].whole ? Range{0, arr[i]->E}
                                             : isect({it.lo + args[i].off_lo, it.hi + args[i].off_hi}, {0, arr[i]->E});
            return pc;
        };
        std::vector<Piece> edges;
        for (int p = 0; p < K; ++p) {
            const Range it = plan[p].iters;
            if (it.empty()) continue;
            const int64_t top = p > 0 ? e : 0, bot = p < K - 1 ? e : 0;
            if (it.hi - it.lo < top + bot + 8) {
                edges.push_back(piece(p, it));  // too short to split: all of it waits
                continue;
            }
            pieces.push_back(piece(p, {it.lo + top, it.hi - bot}));
            if (top) edges.push_back(piece(p, {it.lo, it.lo + top}));
            if (bot) edges.push_back(piece(p, {it.hi - bot, it.hi}));
        }
        pieces.insert(pieces.end(), edges.begin(), edges.end());
    } else if (!packed) {
        for (int p = 0; p < K; ++p) pieces.push_back({p, plan[p]});
    }
    // the launch of one piece, and the other slabs' rows it also writes
    auto piece_launch = [&](int p, const PartPlan &pp, std::vector<std::pair<int, Range>> &mirrors) {
        mirrors.clear();
        if (can_mirror) {
            for (int q = 0; q < K; ++q) {
                if (q == p) continue;
                Range x = isect(pp.rng[primary], P->slabs[q].rows);
                if (!x.empty()) mirrors.push_back({q, x});
            }
            if (mirrors.size() > 2) mirrors.clear();  // then the readers pull instead
        }
        jk::Launch LP = L;
        for (int d = 0; d < b->ndim; ++d) {
            LP.lo[d] = b->lo[d];
            LP.hi[d] = b->hi[d];
        }
        LP.lo[P->pdim] = pp.iters.lo;
        LP.hi[P->pdim] = pp.iters.hi;
        LP.part_dim = P->pdim;
        for (int i = 0; i < nargs; ++i) {
            // biased so that global indices address the slab: by whole rows,
            // or by elements for column slabs (whose width is the row pitch)
            const Slab &sl = arr[i]->slabs[p];
            const bool cols = arr[i]->pdim != 0;
            const size_t unit = cols ? arr[i]->esize : arr[i]->row_bytes;
            LP.a[i].ptr = (const char *)sl.dev - (intptr_t)((size_t)sl.base * unit);
            LP.a[i].slab_lo = sl.rows.lo;
            LP.a[i].slab_hi = sl.rows.hi;
            LP.a[i].row_elems = cols ? sl.pitch : arr[i]->row_elems;
        }
        if (args[primary].mode & JACC_FILTERED) {
            LP.own_lo = pp.rng[primary].lo;
            LP.own_hi = pp.rng[primary].hi;
        }
        if (kind == JACC_LOOP_PRED_CHAIN) {
            LP.own2_lo = pp.rng[1].lo;
            LP.own2_hi = pp.rng[1].hi;
        }
        if (P->pdim == 0) {
            LP.mir.n = (int)mirrors.size();
            for (size_t k = 0; k < mirrors.size(); ++k) {
                const Slab &sq = P->slabs[mirrors[k].first];
                LP.mir.m[k].ptr = (double *)((char *)sq.dev - (intptr_t)((size_t)sq.rows.lo * P->row_bytes));
                LP.mir.m[k].lo = mirrors[k].second.lo;
                LP.mir.m[k].hi = mirrors[k].second.hi;
            }
        } else {  // column slabs, each biased by its first stored column
            LP.mir.n = 0;
            LP.cmir.n = (int)mirrors.size();
            for (size_t k = 0; k < mirrors.size(); ++k) {
                const Slab &sq = P->slabs[mirrors[k].first];
                LP.cmir.m[k].ptr = (double *)sq.dev - sq.base;
                LP.cmir.m[k].pitch = sq.pitch;
                LP.cmir.m[k].lo = mirrors[k].second.lo;
                LP.cmir.m[k].hi = mirrors[k].second.hi;
            }
        }
        return LP;
    };
    if (packed) {
        // pulls first (copies on the one stream), then every partition's
        // accesses, all attributed to the one launch that follows
        const int s = stream_for(0);
        for (int p = 0; p < K; ++p) {
            if (plan[p].iters.empty()) continue;
            for (int i = 0; i < nargs; ++i)
                if (args[i].mode & JACC_READ) {
                    rc = make_fresh(c, arr[i], p, plan[p].rng[i], s);
                    if (rc) return rc;
                }
        }
        std::vector<jk::Launch> lps;
        std::vector<jk::BandBufs> bbs;  // banded SpMV: each partition's band-major copy
        std::vector<std::vector<std::pair<int, Range>>> mirs((size_t)K);
        for (int p = 0; p < K; ++p) {
            const PartPlan &pp = plan[p];
            if (pp.iters.empty()) continue;
            jk::Launch LP = piece_launch(p, pp, mirs[(size_t)p]);
            for (int i = 0; i < nargs; ++i) {
                if (args[i].mode & JACC_READ) {
                    rc = hazard(c, arr[i], p, pp.rng[i], false, s);
                    if (rc) return rc;
                }
                if (args[i].mode & JACC_WRITE) {
                    rc = hazard(c, arr[i], p, pp.rng[i], true, s);
                    if (rc) return rc;
                }
            }
            for (auto &m : mirs[(size_t)p]) {
                rc = hazard(c, P, m.first, m.second, true, s);
                if (rc) return rc;
            }
            if (want_red) {  // as in a launch per partition: partials[slot][p] free, sum written there
                const size_t pi = (size_t)red_slot * kMaxK + p;
                rc = ensure_wait(c, s, c->partial_reader[pi].s, c->partial_reader[pi].seq);
                if (rc) return rc;
                LP.part_out = c->partials + pi;
                order.push_back(p);
                red_streams.push_back(s);
            }
            if (kind == JACC_LOOP_SPMV_CSR) {
                BandCache *bc = nullptr;
                rc = band_cache(c, arr, p, pp.iters, 8 * LP.cfg.by, &bc);
                if (rc) return rc;
                if (live(c) && !bc->built) HIPCHK(c, jk::build_bands(LP, bc->bb, c->st[s].s), "banded SpMV build");
                bc->built = true;
                bbs.push_back(bc->bb);
            }
            lps.push_back(LP);
        }
        if (inject_fault(c, 2)) {
            c->status = JACC_ERR_DEVICE;
            return set_err(c, JACC_ERR_DEVICE, "injected fault in launch %lld", (long long)c->fault_count);
        }
        if (live(c))
            HIPCHK(c,
                   kind == JACC_LOOP_SPMV_CSR
                       ? jk::launch_spmv_banded_parts(lps.data(), bbs.data(), (int)lps.size(), c->st[s].s)
                       : jk::launch_parts(lps.data(), (int)lps.size(), c->wg + (size_t)s * kWgCapacity, kWgCapacity,
                                          c->st[s].s),
                   "kernel launch");
        c->st[s].seq++;
        for (int p = 0; p < K; ++p)
            if (!plan[p].iters.empty())
                trace(c, JACC_OP_KERNEL, s, -1, -1, p, kind, plan[p].iters.lo, plan[p].iters.hi, c->st[s].seq);
        rc = post_op(c);
        if (rc) return rc;
        // no event is recorded here: the packed launch's stream carries the
        // loop's every partition, and a later wait on it records one then
        // (ensure_wait), covering at least this launch
        for (int p = 0; p < K; ++p) {
            if (plan[p].iters.empty()) continue;
            for (int i = 0; i < nargs; ++i)
                if (args[i].mode & JACC_WRITE) note_write(arr[i], p, plan[p].rng[i]);
            for (auto &m : mirs[(size_t)p]) P->valid[m.first].add(m.second);
        }
    }
    if (nstreams(c) > 1 && !one_stream && !persistent && K > 1) {
        // the pieces below issue on several streams and wait on earlier work
        // of each other's streams: a stream whose last op carries no event
        // yet (a packed launch, a loop of one partition) gets one now, before
        // this loop adds its own ops there, so a wait on it does not also
        // cover them
        for (const Piece &pc : pieces) {
            if (pc.pp.iters.empty()) continue;
            const int s = stream_for(pc.p);
            if (c->st[s].recorded < c->st[s].seq) {
                int idx;
                rc = ensure_event(c, s, c->st[s].seq, &idx);
                if (rc) return rc;
            }
        }
    }
    for (const Piece &piece_ : pieces) {
        const int p = piece_.p;
        const PartPlan &pp = piece_.pp;
        if (pp.iters.empty()) continue;
        const int s = stream_for(p);
        std::vector<std::pair<int, Range>> mirrors;
        for (int i = 0; i < nargs; ++i)
            if (args[i].mode & JACC_READ) {
                rc = make_fresh(c, arr[i], p, pp.rng[i], s);
                if (rc) return rc;
            }
        jk::Launch LP = piece_launch(p, pp, mirrors);
        auto note_mirrors = [&]() {
            for (auto &m : mirrors) P->valid[m.first].add(m.second);
        };
        if (persistent) {
            jk::PTask t;
            if (!jk::make_task(LP, &t))
                return set_err(c, JACC_ERR_UNSUPPORTED, "loop kind %d cannot run persistent", kind);
            if (t.ntiles > 0) c->ptasks.push_back(t);
            for (int i = 0; i < nargs; ++i) {
                if (args[i].mode & JACC_READ) c->paccs.push_back({arr[i], p, pp.rng[i], false});
                if (args[i].mode & JACC_WRITE) c->paccs.push_back({arr[i], p, write_span(i, pp), true});
                c->parrays.push_back(arr[i]);
            }
            for (auto &m : mirrors) c->paccs.push_back({P, m.first, m.second, true});
            for (int i = 0; i < nargs; ++i)
                if (args[i].mode & JACC_WRITE) {
                    if (dup)
                        note_everywhere(arr[i], pp.rng[i]);
                    else
                        note_write(arr[i], p, pp.rng[i]);
                }
            note_mirrors();
            continue;
        }
        for (int i = 0; i < nargs; ++i) {
            if (args[i].mode & JACC_READ) {
                rc = hazard(c, arr[i], p, pp.rng[i], false, s);
                if (rc) return rc;
            }
            if (args[i].mode & JACC_WRITE) {
                const Range span = write_span(i, pp);
                rc = hazard(c, arr[i], p, pp.rng[i], true, s, (dup && p != first_run) ? 4 : 2);
                if (rc) return rc;
                // private writes of a filtered output outside the owner block
                for (const Range &x : {Range{span.lo, std::min(span.hi, pp.rng[i].lo)},
                                       Range{std::max(span.lo, pp.rng[i].hi), span.hi}}) {
                    if (x.empty() || pp.rng[i].empty()) continue;
                    rc = hazard(c, arr[i], p, x, true, s, 3);
                    if (rc) return rc;
                }
            }
        }
        for (auto &m : mirrors) {  // writes into another partition's slab
            rc = hazard(c, P, m.first, m.second, true, s);
            if (rc) return rc;
        }
        if (want_red) {
            // partials[slot][p] is read by the last combine of that slot
            // (loops reducing into different slots never wait on each
            // other's combines); the workgroup scratch of stream s is
            // consumed by the finaliser that follows the kernel on the same
            // stream
            const size_t pi = (size_t)red_slot * kMaxK + p;
            rc = ensure_wait(c, s, c->partial_reader[pi].s, c->partial_reader[pi].seq);
            if (rc) return rc;
            LP.wg_partials = c->wg + (size_t)s * kWgCapacity;
            LP.wg_capacity = kWgCapacity;
            LP.part_out = c->partials + pi;
            if (jk::reduction_workgroups(LP) > kWgCapacity)
                return set_err(c, JACC_ERR_UNSUPPORTED, "reduction needs more than %lld workgroups",
                               (long long)kWgCapacity);
            order.push_back(p);
            red_streams.push_back(s);
        }
        if (inject_fault(c, 2)) {
            c->status = JACC_ERR_DEVICE;
            return set_err(c, JACC_ERR_DEVICE, "injected fault in launch %lld", (long long)c->fault_count);
        }
        const bool timed = c->time_parts && live(c) && p < kMaxK;
        if (timed) HIPCHK(c, hipEventRecord(c->kev[2 * p], c->st[s].s), "hipEventRecord");
        if (kind == JACC_LOOP_SPMV_CSR && LP.cfg.order == 4) {  // column-banded product
            BandCache *bc = nullptr;
            rc = band_cache(c, arr, p, pp.iters, 8 * LP.cfg.by, &bc);
            if (rc) return rc;
            if (live(c)) {
                if (!bc->built) HIPCHK(c, jk::build_bands(LP, bc->bb, c->st[s].s), "banded SpMV build");
                HIPCHK(c, jk::launch_spmv_banded(LP, bc->bb, c->st[s].s), "kernel launch");
            }
            bc->built = true;
        } else if (live(c)) {
            HIPCHK(c, jk::launch_loop(LP, c->st[s].s), "kernel launch");
        }
        if (timed) {
            HIPCHK(c, hipEventRecord(c->kev[2 * p + 1], c->st[s].s), "hipEventRecord");
            c->kev_used |= (uint64_t)1 << p;
        }
        c->st[s].seq++;
        trace(c, JACC_OP_KERNEL, s, -1, -1, p, kind, pp.iters.lo, pp.iters.hi, c->st[s].seq);
        rc = post_op(c);
        if (rc) return rc;
        // a precise event for the other partitions, which read these rows in
        // the next loop from their own streams; a loop of one partition
        // records none (a later wait on this stream records one then)
        if (nstreams(c) > 1 && !one_stream && K > 1) {
            int idx;
            rc = ensure_event(c, s, c->st[s].seq, &idx);
            if (rc) return rc;
        }
        for (int i = 0; i < nargs; ++i)
            if (args[i].mode & JACC_WRITE) {
                if (dup)
                    note_everywhere(arr[i], pp.rng[i]);
                else
                    note_write(arr[i], p, pp.rng[i]);
            }
        note_mirrors();
    }
    // the paper's coherence: every partition sends the rows it wrote to every
    // other slab that holds them, on its own stream after its kernel
    if (c->eager && !dup && !persistent) {
        for (int p = 0; p < K; ++p) {
            if (plan[p].iters.empty()) continue;
            for (int i = 0; i < nargs; ++i) {
                if (!(args[i].mode & JACC_WRITE)) continue;
                Array *A = arr[i];
                for (int q = 0; q < K; ++q) {
                    if (q == p) continue;
                    const Range x = isect(plan[p].rng[i], A->slabs[q].rows);
                    if (x.empty()) continue;
                    rc = issue_copy(c, A, p, q, x, stream_for(p));
                    if (rc) return rc;
                    A->valid[q].add(x);
                }
            }
        }
    }
    // debug: rows of floating-point slabs this loop left stale are filled
    // with NaN, so a read that skipped its pull shows in the results
    if (c->poison && !persistent && !dup) {
        Marker mk(c, "jacc poison");
        for (int i = 0; i < nargs; ++i) {
            Array *A = arr[i];
            if (!(args[i].mode & JACC_WRITE) || (A->d.dtype != JACC_F64 && A->d.dtype != JACC_F32)) continue;
            for (int p = 0; p < K; ++p) {
                if (plan[p].iters.empty()) continue;
                for (int q = 0; q < K; ++q) {
                    const Range x = isect(plan[p].rng[i], A->slabs[q].rows);
                    if (x.empty()) continue;
                    for (const Range &m : A->valid[q].missing(x)) {
                        rc = poison_rows(c, A, q, m, stream_for(q));
                        if (rc) return rc;
                    }
                }
            }
        }
    }
    if (want_red) {
        Marker mk(c, "jacc combine slot=%d", red_slot);
        const int s0 = one_stream ? 0 : base % ns;
        for (int s : red_streams) {
            rc = ensure_wait(c, s0, s, c->st[s].seq);
            if (rc) return rc;
        }
        const int sl = red_slot;
        rc = ensure_wait(c, s0, c->slot_src[sl].s, c->slot_src[sl].seq);  // earlier writer of the slot
        if (rc) return rc;
        if (live(c)) {
            jk::CombineList cl{};
            cl.n = (int)order.size();
            for (size_t k = 0; k < order.size(); ++k) cl.idx[k] = order[k];
            HIPCHK(c, jk::launch_combine(c->partials + (size_t)sl * kMaxK, cl, c->slots + sl, c->st[s0].s),
                   "combine launch");
        }
        c->st[s0].seq++;
        for (int q : order) c->partial_reader[(size_t)sl * kMaxK + q] = {s0, c->st[s0].seq};
        c->slot_src[sl] = {s0, c->st[s0].seq};
        trace(c, JACC_OP_COMBINE, s0, -1, -1, -1, sl, 0, 0, c->st[s0].seq);
        rc = post_op(c);
        if (rc) return rc;
        if (red_host) {
            rc = sync_stream(c, s0);
            if (rc) return rc;
            if (live(c))
                HIPCHK(c, hipMemcpy(red_host, c->slots + sl, sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy(D2H)");
            else
                *red_host = 0.0;
        }
    }
    if (note && note->e1) HIPCHK(c, hipEventRecord(note->e1, c->st[stream_for(0)].s), "hipEventRecord");
    return JACC_OK;
}

const char *kind_name(int kind) {
    switch (kind) {
        case JACC_LOOP_JACOBI2D: return "JACOBI2D";
        case JACC_LOOP_HEAT3D: return "HEAT3D";
        case JACC_LOOP_SUM: return "SUM";
        case JACC_LOOP_GEMM: return "GEMM";
        case JACC_LOOP_SPMV_CSR: return "SPMV_CSR";
        case JACC_LOOP_SCATTER_SQ: return "SCATTER_SQ";
        case JACC_LOOP_PRED_CHAIN: return "PRED_CHAIN";
        default: return "?";
    }
}

// Writes one JSON line: the record's fields plus its timing (ms < 0: none).
void log_write(jacc_ctx *c, const jacc_ctx::LogRec &r, double ms) {
    std::string line = r.json;
    char buf[160];
    if (ms < 0 || r.work <= 0) {
        snprintf(buf, sizeof buf, ", \"ms\": %s}\n", ms < 0 ? "null" : std::to_string(ms).c_str());
    } else if (r.flop) {
        snprintf(buf, sizeof buf, ", \"ms\": %.6f, \"tflops\": %.3f}\n", ms, r.work / (ms * 1e-3) / 1e12);
    } else {
        const double gbps = r.work / (ms * 1e-3) / 1e9;
        snprintf(buf, sizeof buf, ", \"ms\": %.6f, \"gbps\": %.1f, \"frac_hbm_peak\": %.4f}\n", ms, gbps,
                 gbps / 8000.0);
    }
    line += buf;
    fputs(line.c_str(), c->log);
}

// Resolves and writes the pending timed records (their events complete).
void log_flush(jacc_ctx *c) {
    if (!c->log) return;
    for (auto &r : c->log_pending) {
        float ms = -1.0f;
        if (r.e1 && hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess)
            ms = -1.0f;
        log_write(c, r, ms);
        if (r.e0) (void)hipEventDestroy(r.e0);
        if (r.e1) (void)hipEventDestroy(r.e1);
    }
    c->log_pending.clear();
    fflush(c->log);
}

void log_loop(jacc_ctx *c, int kind, const LoopNote &n, int64_t copies, int64_t copy_bytes, double issue_us) {
    char buf[512];
    snprintf(buf, sizeof buf,
             "{\"loop\": %lld, \"kind\": \"%s\", \"K\": %d, \"partitions_run\": %d, \"packed\": %s, "
             "\"cfg\": {\"bx\": %d, \"by\": %d, \"tile\": %d, \"vec\": %d, \"order\": %d, \"march\": %d, "
             "\"rows\": %d, \"persistent\": %d}, \"cells\": %.0f, \"copies\": %lld, \"copy_bytes\": %lld, "
             "\"%s\": %.0f, \"issue_us\": %.2f",
             (long long)c->log_seq++, kind_name(kind), n.K, n.nrun, n.packed ? "true" : "false", n.cfg.bx, n.cfg.by,
             n.cfg.tile, n.cfg.vec, n.cfg.order, n.cfg.march, n.cfg.rows, n.cfg.persistent, n.cells,
             (long long)copies, (long long)copy_bytes, n.flop ? "flop" : "algorithmic_bytes", n.work, issue_us);
    jacc_ctx::LogRec r;
    r.json = buf;
    r.work = n.work;
    r.flop = n.flop;
    r.e0 = n.e0;
    r.e1 = n.e1;
    if (!r.e1) {
        log_write(c, r, -1.0);
        return;
    }
    c->log_pending.push_back(r);
    if (c->log_pending.size() >= 256) log_flush(c);
}

// ---- batches ----------------------------------------------------------------
void snapshot(jacc_ctx *c, std::map<Array *, ArraySnap> &snap) {
    snap.clear();
    for (auto &kv : c->present) {
        ArraySnap s;
        s.writer = kv.second->writer;
        s.valid = kv.second->valid;
        for (auto &sl : kv.second->slabs) s.acc.push_back(sl.acc);
        snap[kv.second] = s;
    }
}

void restore(jacc_ctx *c, std::map<Array *, ArraySnap> &snap) {
    for (auto &kv : snap) {
        kv.first->writer = kv.second.writer;
        kv.first->valid = kv.second.valid;
        for (size_t p = 0; p < kv.second.acc.size(); ++p) kv.first->slabs[p].acc = kv.second.acc[p];
    }
}

// Structural form of an op list (what is copied or launched where), without
// sequence numbers.
std::vector<std::vector<int64_t>> structure(const std::vector<jacc_trace_op> &ops) {
    std::vector<std::vector<int64_t>> out;
    for (const auto &t : ops) {
        if (t.op == JACC_OP_RECORD || t.op == JACC_OP_SYNC || t.op == JACC_OP_JOIN) continue;
        if (t.op == JACC_OP_WAIT)
            out.push_back({t.op, t.stream, t.src});
        else
            out.push_back({t.op, t.stream, t.array, t.src, t.dst, t.kind, t.lo, t.hi});
    }
    return out;
}

// Plans the recorded calls of batch B once more without device work, from
// the current state, logging the ops into *log.
int replan(jacc_ctx *c, Batch *B, std::vector<jacc_trace_op> *log) {
    Batch probe;
    Batch *saved = c->cur;
    c->plan_only = true;
    c->oplog = log;
    c->cur = &probe;
    assume_joined(c);
    int rc = JACC_OK;
    for (auto &lc : B->calls) {
        rc = loop_impl(c, lc.kind, &lc.b, (int)lc.args.size(), lc.args.data(), lc.scalars.data(),
                       (int)lc.scalars.size(), lc.slot, nullptr, lc.has_cfg ? &lc.cfg : nullptr);
        if (rc) break;
    }
    if (!rc) rc = flush_group(c);
    c->cur = saved;
    c->plan_only = false;
    c->oplog = nullptr;
    return rc;
}

int launch_graph(jacc_ctx *c, Batch *B, int repeats) {
    int rc = join_into0(c);
    if (rc) return rc;
    if (live(c))
        for (int r = 0; r < repeats; ++r) HIPCHK(c, hipGraphLaunch(B->exec, c->st[0].s), "hipGraphLaunch");
    rc = fork_from0(c);
    if (rc) return rc;
    assume_joined(c);
    return JACC_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char *jacc_version(void) { return "jacc-mi355x 0.2 (gfx950)"; }

int jacc_init(jacc_ctx **out, int K, void *const *streams, const jacc_allocator *alloc, unsigned flags) {
    g_init_err.clear();
    if (!out) return JACC_ERR_INVALID;
    *out = nullptr;
    // environment defaults; the caller's flags win
    auto env_on = [](const char *name) {
        const char *v = getenv(name);
        return v && *v && strcmp(v, "0") != 0;
    };
    if (K == 0) {
        const char *v = getenv("JACC_K");
        char *end = nullptr;
        const long k = (v && *v) ? strtol(v, &end, 10) : 0;
        if (!v || !*v || *end || k < 1 || k > kMaxK) {
            g_init_err = "K = 0 takes JACC_K, which must be an integer in [1, 64]";
            return JACC_ERR_INVALID;
        }
        K = (int)k;
    }
    if (K < 1 || K > kMaxK) {
        g_init_err = "K must lie in [1, 64]";
        return JACC_ERR_INVALID;
    }
    if (env_on("JACC_SERIALIZE")) flags |= JACC_INIT_SERIALIZE;
    if (env_on("JACC_TRACE")) flags |= JACC_INIT_TRACE;
    if (env_on("JACC_DEBUG_POISON")) flags |= JACC_INIT_POISON;
    if (env_on("JACC_ROCTX")) flags |= JACC_INIT_MARKERS;
    if (const char *v = getenv("JACC_COHERENCE")) {
        const bool lz = !strcmp(v, "lazy"), eg = !strcmp(v, "eager");
        if (!lz && !eg && strcmp(v, "mirror") != 0) {
            g_init_err = "JACC_COHERENCE must be mirror, lazy or eager";
            return JACC_ERR_INVALID;
        }
        if (!(flags & (JACC_INIT_LAZY | JACC_INIT_EAGER))) flags |= lz ? JACC_INIT_LAZY : eg ? JACC_INIT_EAGER : 0u;
    }
    int tune_mode = 0;
    if (const char *v = getenv("JACC_TUNE")) {
        if (!strcmp(v, "off"))
            tune_mode = 1;
        else if (!strcmp(v, "exhaustive"))
            tune_mode = 2;
        else if (strcmp(v, "model") != 0) {
            g_init_err = "JACC_TUNE must be model, off or exhaustive";
            return JACC_ERR_INVALID;
        }
    }
    if (alloc && (!alloc->alloc || !alloc->free)) {
        g_init_err = "allocator without alloc/free";
        return JACC_ERR_INVALID;
    }
    if ((flags & JACC_INIT_FORK_CAPTURE) && !(flags & JACC_INIT_DRYRUN)) {
        g_init_err = "JACC_INIT_FORK_CAPTURE plans batches only (dry run): captured graphs run on one stream";
        return JACC_ERR_UNSUPPORTED;
    }
    if ((flags & JACC_INIT_EAGER) && (flags & JACC_INIT_LAZY)) {
        g_init_err = "JACC_INIT_EAGER and JACC_INIT_LAZY exclude each other";
        return JACC_ERR_INVALID;
    }
    jacc_ctx *c = nullptr;
    try {
        c = new jacc_ctx();
        c->K = K;
        c->flags = flags;
        c->dry = (flags & JACC_INIT_DRYRUN) != 0;
        c->tracing = (flags & JACC_INIT_TRACE) != 0;
        c->serialize = (flags & JACC_INIT_SERIALIZE) != 0;
        c->lazy = (flags & JACC_INIT_LAZY) != 0;
        c->split = (flags & JACC_INIT_SPLIT) != 0;
        c->no_split = (flags & JACC_INIT_NO_SPLIT) != 0;
        c->no_pack = (flags & JACC_INIT_NO_PACK) != 0;
        c->eager = (flags & JACC_INIT_EAGER) != 0;
        c->fork_capture = (flags & JACC_INIT_FORK_CAPTURE) != 0;
        c->poison = (flags & JACC_INIT_POISON) != 0;
        c->markers = (flags & JACC_INIT_MARKERS) != 0;
        c->tune_mode = tune_mode;
        if (const char *db = getenv("JACC_TUNE_DB")) c->tune_db = db;
        if (const char *lp = getenv("JACC_LOG")) {
            if (*lp) {
                c->log = fopen(lp, "a");
                if (!c->log) {
                    g_init_err = std::string("cannot open JACC_LOG file ") + lp;
                    delete c;
                    return JACC_ERR_INVALID;
                }
            }
        }
        c->log_times = env_on("JACC_LOG_TIMES");
        if (alloc) {
            c->alloc = *alloc;
            c->use_hipmalloc = false;
        }
        if (const char *f = getenv("JACC_FAULT_INJECT")) {  // "<copy|launch>:<n>"
            const char *colon = strchr(f, ':');
            if (colon) {
                if (!strncmp(f, "copy", 4)) c->fault_kind = 1;
                if (!strncmp(f, "launch", 6)) c->fault_kind = 2;
                c->fault_n = atoll(colon + 1);
            }
        }
        const int ns = c->serialize ? 1 : K;
        c->st.resize(ns);
        c->own_streams = (streams == nullptr);
        c->partial_reader.assign((size_t)kSlots * kMaxK, SeqRef{});
        c->slot_src.assign(kSlots, SeqRef{});
        int rc = JACC_OK;
        for (int s = 0; s < ns && !rc; ++s) {
            StreamState &S = c->st[s];
            S.waited.assign(ns, 0);
            S.ring.resize(kEventRing);
            if (c->dry) continue;
            hipError_t e = hipSuccess;
            if (streams)
                S.s = (hipStream_t)streams[s];
            else
                e = hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking);
            for (auto &E : S.ring)
                if (e == hipSuccess) e = hipEventCreateWithFlags(&E.ev, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&S.join_ev, hipEventDisableTiming);
            if (e != hipSuccess) rc = dev_fail(c, e, "stream/event creation");
        }
        if (!rc && !c->dry) {
            hipError_t e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreate(&c->t0);
            if (e == hipSuccess) e = hipEventCreate(&c->t1);
            if (e != hipSuccess) rc = dev_fail(c, e, "event creation");
        }
        if (!rc) rc = dev_alloc(c, kSlots * sizeof(double), (void **)&c->slots);
        if (!rc) rc = dev_alloc(c, (size_t)kSlots * kMaxK * sizeof(double), (void **)&c->partials);
        if (!rc) rc = dev_alloc(c, (size_t)ns * kWgCapacity * sizeof(double), (void **)&c->wg);
        if (!rc && !c->dry) {
            hipError_t e = hipMemset(c->slots, 0, kSlots * sizeof(double));
            if (e == hipSuccess) e = hipDeviceSynchronize();
            if (e != hipSuccess) rc = dev_fail(c, e, "hipMemset");
        }
        if (rc) {
            g_init_err = c->err;
            c->status = JACC_OK;
            jacc_finalize(c);
            return rc;
        }
        // a model file named by the environment: attached when it loads
        // (a file that does not leaves its reason in jacc_last_error)
        const char *mp = getenv("JACC_MODEL_PATH");
        if (mp && *mp && !c->dry) (void)jacc_model_load(c, mp);
    } catch (const std::bad_alloc &) {
        delete c;
        g_init_err = "host allocation failed";
        return JACC_ERR_ALLOC;
    } catch (...) {
        delete c;
        g_init_err = "internal error";
        return JACC_ERR_INVALID;
    }
    *out = c;
    return JACC_OK;
}

int jacc_finalize(jacc_ctx *c) {
    if (!c) return JACC_ERR_INVALID;
    int status = c->status;
    try {
        if (c->log) {
            if (!c->status && !c->dry)
                for (auto &S : c->st)
                    if (S.s) (void)hipStreamSynchronize(S.s);
            log_flush(c);
            fclose(c->log);
            c->log = nullptr;
        }
        if (c->model && c->model_release) c->model_release(c->model);  // its buffers come from this context
        c->model = nullptr;
        if (c->cur) {  // abandon an open capture (its op log goes with it)
            c->oplog = nullptr;
            if (live(c)) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(c->st[0].s, &g);
                if (g) (void)hipGraphDestroy(g);
            }
            c->batches.push_back(c->cur);
            c->cur = nullptr;
        }
        if (!c->dry)
            for (auto &S : c->st)
                if (S.s) (void)hipStreamSynchronize(S.s);
        for (Batch *B : c->batches) {
            if (!B) continue;
            if (!c->dry) {
                if (B->exec) (void)hipGraphExecDestroy(B->exec);
                if (B->graph) (void)hipGraphDestroy(B->graph);
                if (B->host_tasks) (void)hipHostFree(B->host_tasks);
            }
            dev_free(c, B->dev_tasks);
            delete B;
        }
        c->batches.clear();
        for (auto &kv : c->present) free_array(c, kv.second);
        c->present.clear();
        dev_free(c, c->slots);
        dev_free(c, c->partials);
        dev_free(c, c->wg);
        if (!c->dry) {
            for (auto &S : c->st) {
                for (auto &E : S.ring)
                    if (E.ev) (void)hipEventDestroy(E.ev);
                if (S.join_ev) (void)hipEventDestroy(S.join_ev);
                if (c->own_streams && S.s) (void)hipStreamDestroy(S.s);
            }
            for (hipEvent_t e : c->kev)
                if (e) (void)hipEventDestroy(e);
            if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
            if (c->t0) (void)hipEventDestroy(c->t0);
            if (c->t1) (void)hipEventDestroy(c->t1);
        }
    } catch (...) {
    }
    delete c;
    return status;
}

int jacc_data_enter(jacc_ctx *c, void *host, const jacc_array_desc *d, int clause) {
    GUARD(c);
    Marker mk(c, "jacc enter");
    try {
        if (c->cur) return set_err(c, JACC_ERR_INVALID, "data regions cannot change inside a batch");
        if (!host || !d) return set_err(c, JACC_ERR_INVALID, "NULL host pointer or descriptor");
        if (clause != JACC_COPYIN && clause != JACC_CREATE && clause != JACC_COPY)
            return set_err(c, JACC_ERR_INVALID, "bad clause %d", clause);
        size_t es = dtype_size(d->dtype);
        if (!es || d->ndim < 1 || d->ndim > 4) return set_err(c, JACC_ERR_INVALID, "bad dtype or ndim");
        int64_t row = 1;
        for (int i = 0; i < d->ndim; ++i) {
            if (d->extent[i] < 1) return set_err(c, JACC_ERR_INVALID, "extent[%d] < 1", i);
            if (i > 0) row *= d->extent[i];
        }
        if (d->halo_lo < 0 || d->halo_hi < 0) return set_err(c, JACC_ERR_INVALID, "negative halo");
        if (d->reserved != 0) return set_err(c, JACC_ERR_INVALID, "reserved descriptor field not 0");
        if (d->part_dim != 0 && d->part_dim != 1) return set_err(c, JACC_ERR_INVALID, "part_dim must be 0 or 1");
        if (d->part_dim == 1 && d->ndim != 2)
            return set_err(c, JACC_ERR_UNSUPPORTED, "arrays are split along dimension 1 only when they are 2-D");
        if (d->whole < 0 || d->whole > 2) return set_err(c, JACC_ERR_INVALID, "whole must be 0, 1 or 2");
        if (d->part_dim != 0 && d->whole)
            return set_err(c, JACC_ERR_INVALID, "an array entered whole is not split: part_dim must be 0");
        const int64_t E = d->extent[d->part_dim];
        int K = d->num_partitions ? d->num_partitions : c->K;
        // more partitions than streams is allowed: partition p then runs on
        // stream p mod the stream count
        if (K < 1 || K > kMaxK) return set_err(c, JACC_ERR_INVALID, "num_partitions %d not in [1,%d]", K, kMaxK);
        if (!d->whole && K > E)
            return set_err(c, JACC_ERR_INVALID, "K=%d exceeds the %lld rows of dimension %d", K, (long long)E,
                           d->part_dim);
        size_t bytes = (size_t)d->extent[0] * (size_t)row * es;
        if (Array *A = lookup(c, host)) {
            if (A->host == (uintptr_t)host && A->bytes == bytes && desc_equal(A->d, *d)) {
                A->refs++;
                return JACC_OK;
            }
            return set_err(c, JACC_ERR_ALREADY_PRESENT, "host range overlaps array %d with another descriptor", A->id);
        }
        {  // a new range must not overlap a later array either
            auto it = c->present.lower_bound((uintptr_t)host);
            if (it != c->present.end() && it->first < (uintptr_t)host + bytes)
                return set_err(c, JACC_ERR_ALREADY_PRESENT, "host range overlaps array %d", it->second->id);
        }
        Array *A = new Array();
        A->id = c->next_id++;
        A->host = (uintptr_t)host;
        A->bytes = bytes;
        A->d = *d;
        A->K = K;
        A->home = (K == nstreams(c) || c->serialize) ? 0 : (c->next_home++ % nstreams(c));
        A->pdim = d->part_dim;
        A->E = E;
        A->row_elems = A->pdim == 0 ? row : d->extent[0];  // a row of dimension 1 is a column
        A->esize = es;
        A->row_bytes = (size_t)A->row_elems * es;
        A->whole = d->whole != 0;
        A->shared = d->whole == 2;
        A->slabs.resize(K);
        A->valid.resize(K);
        A->writer.init(0, A->E, -1);
        int rc = JACC_OK;
        for (int p = 0; p < K && !rc; ++p) {
            Range sl{0, A->E};
            if (!A->whole) {
                Range bl = A->block(p);
                sl = {std::max<int64_t>(0, bl.lo - d->halo_lo), std::min<int64_t>(A->E, bl.hi + d->halo_hi)};
            }
            Slab &S = A->slabs[p];
            S.rows = sl;
            S.base = A->pdim == 0 ? sl.lo : (sl.lo & ~(int64_t)1);
            S.pitch = A->pdim == 0 ? A->row_elems : ((sl.hi - S.base + 1) & ~(int64_t)1);
            S.acc.init(sl.lo, sl.hi, Access{});
            A->valid[p].add(sl);
            if (A->shared && p > 0) {  // the same device copy as partition 0
                S.dev = A->slabs[0].dev;
                continue;
            }
            const size_t stored = A->pdim == 0 ? (size_t)(sl.hi - sl.lo) * A->row_bytes
                                               : (size_t)S.pitch * (size_t)d->extent[0] * A->esize;
            rc = dev_alloc(c, stored, &S.dev);
            if (!rc) trace(c, JACC_OP_ALLOC, -1, A->id, -1, p, 0, sl.lo, sl.hi, 0);
        }
        if (rc) {
            for (int p = 0; p < (A->shared ? 1 : K); ++p) dev_free(c, A->slabs[p].dev);
            delete A;
            return rc;
        }
        c->present[A->host] = A;
        if (clause == JACC_COPYIN || clause == JACC_COPY) {
            for (int p = 0; p < (A->shared ? 1 : K); ++p) {
                rc = h2d_rows(c, A, p, A->slabs[p].rows);
                if (rc) return rc;
            }
        }
        return JACC_OK;
    } catch (const std::bad_alloc &) {
        return set_err(c, JACC_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return set_err(c, JACC_ERR_INVALID, "internal error");
    }
}

int jacc_data_exit(jacc_ctx *c, void *host, int clause) {
    GUARD(c);
    Marker mk(c, "jacc exit");
    try {
        if (c->cur) return set_err(c, JACC_ERR_INVALID, "data regions cannot change inside a batch");
        if (clause != JACC_COPYOUT && clause != JACC_DELETE) return set_err(c, JACC_ERR_INVALID, "bad clause %d", clause);
        Array *A = lookup(c, host);
        if (!A) return set_err(c, JACC_ERR_NOT_PRESENT, "%p is not present", host);
        int rc = JACC_OK;
        if (clause == JACC_COPYOUT) {
            rc = gather(c, A, {0, A->E});
            if (rc) return rc;
        }
        if (--A->refs > 0) return JACC_OK;
        rc = sync_all(c);
        if (rc) return rc;
        for (Batch *B : c->batches)
            if (B && std::find(B->array_ids.begin(), B->array_ids.end(), A->id) != B->array_ids.end()) B->stale = true;
        c->present.erase(A->host);
        free_array(c, A);
        return JACC_OK;
    } catch (...) {
        return set_err(c, JACC_ERR_INVALID, "internal error");
    }
}

int jacc_update(jacc_ctx *c, void *host, int dir, int64_t row_lo, int64_t row_hi) {
    GUARD(c);
    Marker mk(c, "jacc update dir=%d", dir);
    try {
        if (c->cur) return set_err(c, JACC_ERR_INVALID, "updates cannot run inside a batch");
        Array *A = lookup(c, host);
        if (!A) return set_err(c, JACC_ERR_NOT_PRESENT, "%p is not present", host);
        if (row_hi < 0) row_hi = A->E;
        if (row_lo < 0 || row_lo > row_hi || row_hi > A->E)
            return set_err(c, JACC_ERR_INVALID, "bad row range [%lld,%lld)", (long long)row_lo, (long long)row_hi);
        Range r{row_lo, row_hi};
        if (r.empty()) return JACC_OK;
        if (dir == JACC_UPDATE_HOST) {
            const int rc = gather(c, A, r);
            if (!rc) log_flush(c);
            return rc;
        }
        if (dir != JACC_UPDATE_DEVICE) return set_err(c, JACC_ERR_INVALID, "bad direction %d", dir);
        for (int p = 0; p < A->K; ++p) {
            Range x = isect(r, A->slabs[p].rows);
            if (x.empty()) continue;
            if (!A->shared || p == 0) {
                int rc = h2d_rows(c, A, p, x);
                if (rc) return rc;
            }
            A->valid[p].add(x);
        }
        A->writer.assign(r, -1);
        return JACC_OK;
    } catch (...) {
        return set_err(c, JACC_ERR_INVALID, "internal error");
    }
}

int jacc_parallel_loop(jacc_ctx *c, int kind, const jacc_bounds *b, int nargs, const jacc_arg *args,
                       const double *scalars, int nscalars, int reduce_slot, double *reduce_host,
                       const jacc_config *cfg) {
    GUARD(c);
    try {
        if (!c->log || c->cur) return loop_impl(c, kind, b, nargs, args, scalars, nscalars, reduce_slot, reduce_host, cfg);
        LoopNote note;
        const int64_t c0 = c->log_copies, b0 = c->log_copy_bytes;
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = loop_impl(c, kind, b, nargs, args, scalars, nscalars, reduce_slot, reduce_host, cfg, &note);
        const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
        if (rc != JACC_OK) {
            if (note.e0) (void)hipEventDestroy(note.e0);
            if (note.e1) (void)hipEventDestroy(note.e1);
            return rc;
        }
        log_loop(c, kind, note, c->log_copies - c0, c->log_copy_bytes - b0, us);
        return rc;
    } catch (const std::bad_alloc &) {
        return set_err(c, JACC_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return set_err(c, JACC_ERR_INVALID, "internal error");
    }
}

int jacc_wait(jacc_ctx *c) {
    GUARD(c);
    Marker mk(c, "jacc wait");
    if (c->cur) return set_err(c, JACC_ERR_INVALID, "jacc_wait inside a batch");
    const int rc = sync_all(c);
    if (!rc) log_flush(c);
    return rc;
}

int jacc_reduction_get(jacc_ctx *c, int slot, double *out) {
    GUARD(c);
    if (slot < 0 || slot >= kSlots || !out) return set_err(c, JACC_ERR_INVALID, "bad slot or output");
    if (c->cur) return set_err(c, JACC_ERR_INVALID, "reduction readback inside a batch");
    int rc = sync_stream(c, c->slot_src[slot].s);
    if (rc) return rc;
    if (!live(c)) {
        *out = 0.0;
        return JACC_OK;
    }
    HIPCHK(c, hipMemcpy(out, c->slots + slot, sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy(D2H)");
    return JACC_OK;
}

int jacc_reduction_read(jacc_ctx *c, int first, int count, double *out) {
    GUARD(c);
    if (first < 0 || count < 0 || first + count > kSlots || (count && !out))
        return set_err(c, JACC_ERR_INVALID, "bad slot range");
    if (c->cur) return set_err(c, JACC_ERR_INVALID, "reduction readback inside a batch");
    int rc = sync_all(c);
    if (rc) return rc;
    if (!count) return JACC_OK;
    if (!live(c)) {
        memset(out, 0, (size_t)count * sizeof(double));
        return JACC_OK;
    }
    HIPCHK(c, hipMemcpy(out, c->slots + first, (size_t)count * sizeof(double), hipMemcpyDeviceToHost),
           "hipMemcpy(D2H)");
    return JACC_OK;
}

int jacc_batch_begin(jacc_ctx *c) {
    GUARD(c);
    Marker mk(c, "jacc batch begin");
    if (c->cur) return set_err(c, JACC_ERR_INVALID, "a batch is already open");
    Batch *B = new Batch();
    int rc = dev_alloc(c, kTaskCapacity * sizeof(jk::PTask), (void **)&B->dev_tasks);
    if (rc) {
        delete B;
        return rc;
    }
    if (!c->dry) {
        hipError_t e = hipHostMalloc((void **)&B->host_tasks, kTaskCapacity * sizeof(jk::PTask), hipHostMallocDefault);
        if (e != hipSuccess) {
            dev_free(c, B->dev_tasks);
            delete B;
            return dev_fail(c, e, "hipHostMalloc");
        }
    }
    // everything issued before the batch completes before the graph runs:
    // each launch joins every stream into stream 0 first
    rc = join_into0(c);
    if (rc) return rc;
    if (live(c)) HIPCHK(c, hipStreamBeginCapture(c->st[0].s, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    c->cur = B;
    assume_joined(c);
    c->oplog = &B->captured;
    return JACC_OK;
}

int jacc_batch_end(jacc_ctx *c, int *graph_id) {
    GUARD(c);
    Marker mk(c, "jacc batch end");
    if (!c->cur) return set_err(c, JACC_ERR_INVALID, "no open batch");
    if (!graph_id) return set_err(c, JACC_ERR_INVALID, "NULL graph id");
    Batch *B = c->cur;
    int rc = flush_group(c);
    c->oplog = nullptr;
    if (rc) return rc;
    if (live(c)) {
        HIPCHK(c, hipStreamEndCapture(c->st[0].s, &B->graph), "hipStreamEndCapture");
        HIPCHK(c, hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        if (B->tasks_used > 0)
            HIPCHK(c, hipMemcpy(B->dev_tasks, B->host_tasks, (size_t)B->tasks_used * sizeof(jk::PTask),
                                hipMemcpyHostToDevice),
                   "hipMemcpy(task tables)");
    }
    c->cur = nullptr;
    c->batches.push_back(B);
    *graph_id = (int)c->batches.size() - 1;
    // Replay check.  The graph holds the ops planned from the state before the
    // batch; the coherence state now is the state after one execution.  If
    // planning the same calls from this state gives the same copies, waits
    // and launches, a replay re-executes exactly what a second execution
    // needs, and the state after it is unchanged (the written rows and the
    // copied rows are the same), so every later replay is correct too.
    try {
        std::map<Array *, ArraySnap> s1;
        snapshot(c, s1);
        std::vector<jacc_trace_op> second;
        int rc2 = replan(c, B, &second);
        B->replay_safe = (rc2 == JACC_OK && structure(second) == structure(B->captured));
        restore(c, s1);
        if (!B->replay_safe) c->err = "batch is not replay-safe";
    } catch (...) {
        c->plan_only = false;
        c->oplog = nullptr;
        c->cur = nullptr;
        B->replay_safe = false;
    }
    assume_joined(c);
    // the batch's calls take effect now: the graph runs once
    return launch_graph(c, B, 1);
}

int jacc_batch_launch(jacc_ctx *c, int graph_id, int repeats) {
    GUARD(c);
    Marker mk(c, "jacc batch launch graph=%d x%d", graph_id, repeats);
    if (c->cur) return set_err(c, JACC_ERR_INVALID, "batch launch inside an open batch");
    if (graph_id < 0 || graph_id >= (int)c->batches.size() || !c->batches[graph_id])
        return set_err(c, JACC_ERR_INVALID, "unknown graph %d", graph_id);
    if (repeats < 0) return set_err(c, JACC_ERR_INVALID, "negative repeats");
    Batch *B = c->batches[graph_id];
    if (B->stale)
        return set_err(c, JACC_ERR_INVALID, "graph %d uses an array that has left the data region", graph_id);
    if (!B->replay_safe)
        return set_err(c, JACC_ERR_UNSUPPORTED, "graph %d is not replay-safe (a later pass plans other copies)",
                       graph_id);
    if (repeats == 0) return JACC_OK;
    return launch_graph(c, B, repeats);
}

int jacc_batch_info(jacc_ctx *c, int graph_id, int *loops, int *persistent_groups, int *replay_safe) {
    GUARD(c);
    if (graph_id < 0 || graph_id >= (int)c->batches.size() || !c->batches[graph_id])
        return set_err(c, JACC_ERR_INVALID, "unknown graph %d", graph_id);
    Batch *B = c->batches[graph_id];
    if (loops) *loops = (int)B->calls.size();
    if (persistent_groups) *persistent_groups = B->groups;
    if (replay_safe) *replay_safe = (B->replay_safe && !B->stale) ? 1 : 0;
    return JACC_OK;
}

int jacc_batch_destroy(jacc_ctx *c, int graph_id) {
    GUARD(c);
    if (c->cur) return set_err(c, JACC_ERR_INVALID, "batch destroy inside an open batch");
    if (graph_id < 0 || graph_id >= (int)c->batches.size() || !c->batches[graph_id])
        return set_err(c, JACC_ERR_INVALID, "unknown graph %d", graph_id);
    Batch *B = c->batches[graph_id];
    int rc = sync_all(c);
    if (rc) return rc;
    if (!c->dry) {
        if (B->exec) (void)hipGraphExecDestroy(B->exec);
        if (B->graph) (void)hipGraphDestroy(B->graph);
        if (B->host_tasks) (void)hipHostFree(B->host_tasks);
    }
    dev_free(c, B->dev_tasks);
    delete B;
    c->batches[graph_id] = nullptr;
    return JACC_OK;
}

int jacc_batch_time(jacc_ctx *c, int graph_id, int warmup, int reps, double *ms) {
    GUARD(c);
    if (c->dry) return set_err(c, JACC_ERR_UNSUPPORTED, "timing needs the device");
    if (reps < 1 || !ms || warmup < 0) return set_err(c, JACC_ERR_INVALID, "bad repetition count");
    int rc = jacc_batch_launch(c, graph_id, warmup);
    if (rc) return rc;
    Batch *B = c->batches[graph_id];
    rc = join_into0(c);
    if (rc) return rc;
    for (int r = 0; r < reps; ++r) {
        HIPCHK(c, hipEventRecord(c->t0, c->st[0].s), "hipEventRecord");
        HIPCHK(c, hipGraphLaunch(B->exec, c->st[0].s), "hipGraphLaunch");
        HIPCHK(c, hipEventRecord(c->t1, c->st[0].s), "hipEventRecord");
        HIPCHK(c, hipEventSynchronize(c->t1), "hipEventSynchronize");
        float f = 0.f;
        HIPCHK(c, hipEventElapsedTime(&f, c->t0, c->t1), "hipEventElapsedTime");
        ms[r] = f;
    }
    rc = fork_from0(c);
    if (rc) return rc;
    assume_joined(c);
    return JACC_OK;
}

int jacc_time_loop(jacc_ctx *c, int kind, const jacc_bounds *b, int nargs, const jacc_arg *args,
                   const double *scalars, int nscalars, const jacc_config *cfg, int warmup, int reps, double *ms) {
    GUARD(c);
    if (c->dry) return set_err(c, JACC_ERR_UNSUPPORTED, "timing needs the device");
    if (c->cur) return set_err(c, JACC_ERR_INVALID, "timing inside an open batch");
    if (reps < 1 || !ms || warmup < 0) return set_err(c, JACC_ERR_INVALID, "bad repetition count");
    try {
        if (cfg && cfg->persistent) {  // persistent configurations run as a one-loop graph
            int rc = jacc_batch_begin(c);
            if (rc) return rc;
            rc = loop_impl(c, kind, b, nargs, args, scalars, nscalars, -1, nullptr, cfg);
            int g = -1;
            int rc_end = jacc_batch_end(c, &g);
            if (!rc) rc = rc_end;
            if (!rc) rc = jacc_batch_time(c, g, warmup, reps, ms);
            if (g >= 0) {
                int rc2 = jacc_batch_destroy(c, g);
                if (!rc) rc = rc2;
            }
            return rc;
        }
        const int slot = kind == JACC_LOOP_SUM ? kSlots - 2 : -1;
        for (int r = 0; r < warmup; ++r) {
            int rc = loop_impl(c, kind, b, nargs, args, scalars, nscalars, slot, nullptr, cfg);
            if (rc) return rc;
        }
        for (int r = 0; r < reps; ++r) {
            int rc = join_into0(c);
            if (rc) return rc;
            HIPCHK(c, hipEventRecord(c->t0, c->st[0].s), "hipEventRecord");
            rc = fork_from0(c);
            if (rc) return rc;
            assume_joined(c);
            rc = loop_impl(c, kind, b, nargs, args, scalars, nscalars, slot, nullptr, cfg);
            if (rc) return rc;
            rc = join_into0(c);
            if (rc) return rc;
            HIPCHK(c, hipEventRecord(c->t1, c->st[0].s), "hipEventRecord");
            HIPCHK(c, hipEventSynchronize(c->t1), "hipEventSynchronize");
            float f = 0.f;
            HIPCHK(c, hipEventElapsedTime(&f, c->t0, c->t1), "hipEventElapsedTime");
            ms[r] = f;
            assume_joined(c);
        }
        return JACC_OK;
    } catch (...) {
        return set_err(c, JACC_ERR_INVALID, "internal error");
    }
}

int jacc_time_loop_parts(jacc_ctx *c, int kind, const jacc_bounds *b, int nargs, const jacc_arg *args,
                         const double *scalars, int nscalars, const jacc_config *cfg, double *step_ms,
                         double *kernel_ms, int nkernel) {
    GUARD(c);
    if (c->dry) return set_err(c, JACC_ERR_UNSUPPORTED, "timing needs the device");
    if (c->cur) return set_err(c, JACC_ERR_INVALID, "timing inside an open batch");
    if (!step_ms || nkernel < 0 || (nkernel && !kernel_ms) || nkernel > kMaxK)
        return set_err(c, JACC_ERR_INVALID, "bad timing outputs");
    if (cfg && cfg->persistent) return set_err(c, JACC_ERR_UNSUPPORTED, "per-partition timing of a persistent loop");
    try {
        if (c->kev.empty()) {
            c->kev.assign(2 * kMaxK, nullptr);
            for (auto &e : c->kev) HIPCHK(c, hipEventCreate(&e), "hipEventCreate");
        }
        const int slot = kind == JACC_LOOP_SUM ? kSlots - 2 : -1;
        int rc = join_into0(c);
        if (rc) return rc;
        HIPCHK(c, hipEventRecord(c->t0, c->st[0].s), "hipEventRecord");
        rc = fork_from0(c);
        if (rc) return rc;
        assume_joined(c);
        c->time_parts = true;
        c->kev_used = 0;
        rc = loop_impl(c, kind, b, nargs, args, scalars, nscalars, slot, nullptr, cfg);
        c->time_parts = false;
        if (rc) return rc;
        rc = join_into0(c);
        if (rc) return rc;
        HIPCHK(c, hipEventRecord(c->t1, c->st[0].s), "hipEventRecord");
        HIPCHK(c, hipEventSynchronize(c->t1), "hipEventSynchronize");
        float f = 0.f;
        HIPCHK(c, hipEventElapsedTime(&f, c->t0, c->t1), "hipEventElapsedTime");
        *step_ms = f;
        for (int p = 0; p < nkernel; ++p) {
            kernel_ms[p] = 0.0;
            if (!(c->kev_used >> p & 1)) continue;
            HIPCHK(c, hipEventElapsedTime(&f, c->kev[2 * p], c->kev[2 * p + 1]), "hipEventElapsedTime");
            kernel_ms[p] = f;
        }
        assume_joined(c);
        return JACC_OK;
    } catch (...) {
        c->time_parts = false;
        return set_err(c, JACC_ERR_INVALID, "internal error");
    }
}

const char *jacc_last_error(const jacc_ctx *c) { return c ? c->err.c_str() : g_init_err.c_str(); }

int jacc_slab_info(jacc_ctx *c, void *host, int p, void **dev, int64_t *row_lo, int64_t *row_hi) {
    if (!c) return JACC_ERR_INVALID;
    Array *A = lookup(c, host);
    if (!A) return set_err(c, JACC_ERR_NOT_PRESENT, "%p is not present", host);
    if (p < 0 || p >= A->K) return set_err(c, JACC_ERR_INVALID, "bad partition %d", p);
    if (dev) *dev = A->slabs[p].dev;
    if (row_lo) *row_lo = A->slabs[p].rows.lo;
    if (row_hi) *row_hi = A->slabs[p].rows.hi;
    return JACC_OK;
}

int jacc_trace_len(const jacc_ctx *c) { return c ? (int)c->trace.size() : 0; }

int jacc_trace_get(const jacc_ctx *c, int i, jacc_trace_op *out) {
    if (!c || !out || i < 0 || i >= (int)c->trace.size()) return JACC_ERR_INVALID;
    *out = c->trace[(size_t)i];
    return JACC_OK;
}

int jacc_trace_clear(jacc_ctx *c) {
    if (!c) return JACC_ERR_INVALID;
    c->trace.clear();
    return JACC_OK;
}

}  // extern "C"

// ---- internal access for other library modules -------------------------------

namespace jr {
bool dry(const jacc_ctx *c) { return c->dry; }
bool failed(const jacc_ctx *c) { return c->status != JACC_OK; }
bool in_batch(const jacc_ctx *c) { return c->cur != nullptr || c->plan_only; }
hipStream_t stream0(const jacc_ctx *c) { return c->st[0].s; }
int alloc(jacc_ctx *c, size_t bytes, void **out) { return dev_alloc(c, bytes, out); }
void release(jacc_ctx *c, void *p) { dev_free(c, p); }
int device_error(jacc_ctx *c, hipError_t e, const char *what) { return dev_fail(c, e, what); }
int error(jacc_ctx *c, int code, const char *msg) { return set_err(c, code, "%s", msg); }
int array_info(jacc_ctx *c, const void *host, jacc_array_desc *d, size_t *bytes, int *K) {
    Array *A = lookup(c, host);
    if (!A) return set_err(c, JACC_ERR_NOT_PRESENT, "%p is not present", host);
    if (d) *d = A->d;
    if (bytes) *bytes = A->bytes;
    if (K) *K = A->K;
    return JACC_OK;
}
void set_thread_error(const char *msg) { g_init_err = msg ? msg : ""; }
void *attached_model(const jacc_ctx *c) { return c->model; }
std::map<std::vector<int64_t>, jacc_config> &tuned_picks(jacc_ctx *c) { return c->tuned; }
const char *tune_db(const jacc_ctx *c) { return c->tune_db.c_str(); }
void attach_model(jacc_ctx *c, void *model, void (*release_model)(void *)) {
    if (c->model && c->model_release) c->model_release(c->model);
    c->model = model;
    c->model_release = release_model;
}
}  // namespace jr
