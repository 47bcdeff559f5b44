"""ctypes binding of libjacc.so (the C ABI in include/jacc.h).

Argument marshalling only: every step of every loop runs in the library's
HIP kernels and C++ runtime.  PyTorch supplies device memory (through the
allocator callback) and the K HIP streams.  The library must be built
in-tree (``python -m paper_2110_14340_amd.build``); loading fails loudly
when it is missing — there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# JACC_LIB names another build of the library (e.g. the sanitizer build of
# `python -m paper_2110_14340_amd.build --asan`)
LIB_PATH = os.environ.get("JACC_LIB") or os.path.join(HERE, "libjacc.so")

# ---- constants mirrored from jacc.h --------------------------------------
OK, ERR_INVALID, ERR_NOT_PRESENT, ERR_ALREADY_PRESENT, ERR_RANGE, ERR_ALLOC, ERR_DEVICE, ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
F64, F32, I32, I64 = 0, 1, 2, 3
COPYIN, CREATE, COPY = 1, 2, 3
COPYOUT, DELETE = 1, 2
UPDATE_HOST, UPDATE_DEVICE = 1, 2
READ, WRITE, READWRITE, FILTERED = 1, 2, 3, 4
JACOBI2D, HEAT3D, SUM, GEMM, SPMV_CSR, SCATTER_SQ, PRED_CHAIN = 1, 2, 3, 4, 5, 6, 7
INIT_DRYRUN, INIT_TRACE, INIT_SERIALIZE, INIT_LAZY, INIT_SPLIT, INIT_NO_SPLIT, INIT_EAGER = 1, 2, 4, 8, 16, 32, 64
INIT_FORK_CAPTURE, INIT_POISON, INIT_MARKERS, INIT_NO_PACK = 128, 256, 512, 1024
SHARED = 2  # jacc_array_desc.whole: one read-only copy for every partition
OP_NAMES = {1: "ALLOC", 2: "FREE", 3: "H2D", 4: "D2H", 5: "COPY", 6: "KERNEL", 7: "RECORD", 8: "WAIT",
            9: "SYNC", 10: "COMBINE", 11: "ACCESS", 12: "JOIN", 13: "POISON"}
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "NOT_PRESENT", -3: "ALREADY_PRESENT", -4: "RANGE", -5: "ALLOC",
                -6: "DEVICE", -7: "UNSUPPORTED"}

_DTYPES = {np.dtype(np.float64): F64, np.dtype(np.float32): F32, np.dtype(np.int32): I32,
           np.dtype(np.int64): I64}


class ArrayDesc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("ndim", ctypes.c_int32), ("extent", ctypes.c_int64 * 4),
                ("halo_lo", ctypes.c_int32), ("halo_hi", ctypes.c_int32), ("whole", ctypes.c_int32),
                ("num_partitions", ctypes.c_int32), ("part_dim", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Arg(ctypes.Structure):
    _fields_ = [("host", ctypes.c_void_p), ("mode", ctypes.c_int32), ("off_lo", ctypes.c_int32),
                ("off_hi", ctypes.c_int32), ("whole", ctypes.c_int32)]


class Bounds(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("pad_", ctypes.c_int32), ("lo", ctypes.c_int64 * 3),
                ("hi", ctypes.c_int64 * 3)]


class Config(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("vec", ctypes.c_int32), ("persistent", ctypes.c_int32), ("order", ctypes.c_int32),
                ("march", ctypes.c_int32), ("rows", ctypes.c_int32)]


class Candidate(ctypes.Structure):
    _fields_ = [("cfg", Config), ("K", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class TuneOpts(ctypes.Structure):
    _fields_ = [("warmup", ctypes.c_int32), ("reps", ctypes.c_int32), ("nks", ctypes.c_int32),
                ("ks", ctypes.c_int32 * 8), ("db_path", ctypes.c_char_p)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("members", ctypes.c_int32), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("lr", ctypes.c_float), ("seed", ctypes.c_uint64), ("holdout", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class TrainReport(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("signatures", ctypes.c_int32), ("loss_first", ctypes.c_float),
                ("loss_last", ctypes.c_float), ("heldout_mse", ctypes.c_float), ("pad_", ctypes.c_int32)]


class Allocator(ctypes.Structure):
    ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
    FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
    _fields_ = [("alloc", ALLOC), ("free", FREE), ("user", ctypes.c_void_p)]


class TraceOp(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("stream", ctypes.c_int32), ("array", ctypes.c_int32),
                ("src", ctypes.c_int32), ("dst", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("lo", ctypes.c_int64), ("hi", ctypes.c_int64), ("seq", ctypes.c_int64)]


_lib = None


def lib():
    """Load libjacc.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2110_14340_amd.build` "
                           "(there is no non-HIP fallback)")
    # PyTorch ships its own HIP runtime; it must be loaded before libjacc.so
    # so that the library binds to the same runtime instead of loading a
    # second one (two runtimes in one process cannot share streams).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.jacc_version.restype = ctypes.c_char_p
    L.jacc_init.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(Allocator), ctypes.c_uint]
    L.jacc_finalize.argtypes = [vp]
    L.jacc_data_enter.argtypes = [vp, vp, ctypes.POINTER(ArrayDesc), i32]
    L.jacc_data_exit.argtypes = [vp, vp, i32]
    L.jacc_update.argtypes = [vp, vp, i32, i64, i64]
    L.jacc_parallel_loop.argtypes = [vp, i32, ctypes.POINTER(Bounds), i32, ctypes.POINTER(Arg),
                                     ctypes.POINTER(ctypes.c_double), i32, i32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(Config)]
    L.jacc_wait.argtypes = [vp]
    L.jacc_reduction_get.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    L.jacc_reduction_read.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double)]
    L.jacc_last_error.argtypes = [vp]
    L.jacc_last_error.restype = ctypes.c_char_p
    L.jacc_slab_info.argtypes = [vp, vp, i32, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.jacc_batch_begin.argtypes = [vp]
    L.jacc_batch_end.argtypes = [vp, ctypes.POINTER(i32)]
    L.jacc_batch_launch.argtypes = [vp, i32, i32]
    L.jacc_batch_info.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.jacc_batch_destroy.argtypes = [vp, i32]
    L.jacc_batch_time.argtypes = [vp, i32, i32, i32, ctypes.POINTER(ctypes.c_double)]
    L.jacc_time_loop.argtypes = [vp, i32, ctypes.POINTER(Bounds), i32, ctypes.POINTER(Arg),
                                 ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(Config), i32, i32,
                                 ctypes.POINTER(ctypes.c_double)]
    L.jacc_time_loop_parts.argtypes = [vp, i32, ctypes.POINTER(Bounds), i32, ctypes.POINTER(Arg),
                                       ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(Config),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), i32]
    fp = ctypes.POINTER(ctypes.c_float)
    L.jacc_model_nparams.argtypes = [i32]
    L.jacc_model_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.jacc_model_destroy.argtypes = [vp]
    L.jacc_model_set_params.argtypes = [vp, fp, i32]
    L.jacc_model_get_params.argtypes = [vp, fp, i32]
    L.jacc_model_set_scaler.argtypes = [vp, fp, fp]
    L.jacc_model_predict.argtypes = [vp, fp, i32, fp]
    L.jacc_model_gradients.argtypes = [vp, fp, fp, i32, fp, fp]
    L.jacc_model_adam_step.argtypes = [vp, ctypes.c_float]
    L.jacc_model_fit.argtypes = [vp, fp, fp, i32, i32, i32, ctypes.c_float, ctypes.c_uint64, fp]
    CP = ctypes.POINTER(Candidate)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int)
    L.jacc_candidates.argtypes = [i32, i64p, i32, i32p, i32, CP, i32, i32p]
    L.jacc_features.argtypes = [i32, i64p, i32, CP, fp]
    L.jacc_build_key.argtypes = [vp]
    L.jacc_build_key.restype = ctypes.c_char_p
    L.jacc_median.argtypes = [ctypes.POINTER(ctypes.c_double), i32]
    L.jacc_median.restype = ctypes.c_double
    L.jacc_argmin.argtypes = [ctypes.POINTER(ctypes.c_double), i32]
    L.jacc_tune.argtypes = [vp, i32, ctypes.POINTER(Bounds), i32, ctypes.POINTER(Arg), ctypes.POINTER(ctypes.c_double),
                            i32, ctypes.POINTER(TuneOpts), CP, ctypes.POINTER(ctypes.c_double), i32, i32p]
    L.jacc_model_train.argtypes = [vp, ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(TrainOpts),
                                   ctypes.POINTER(TrainReport)]
    L.jacc_model_load.argtypes = [vp, ctypes.c_char_p]
    L.jacc_model_unload.argtypes = [vp]
    L.jacc_model_pick.argtypes = [vp, i32, i64p, i32, i32p, i32, CP, fp, i32, i32p]
    L.jacc_choose.argtypes = [vp, i32, ctypes.POINTER(Bounds), i32, ctypes.POINTER(Arg),
                              ctypes.POINTER(ctypes.c_double), i32, ctypes.c_char_p, ctypes.POINTER(TuneOpts), CP, i32p]
    L.jacc_trace_len.argtypes = [vp]
    L.jacc_trace_get.argtypes = [vp, i32, ctypes.POINTER(TraceOp)]
    L.jacc_trace_clear.argtypes = [vp]
    d = ctypes.c_double
    L.jacc_adapt_create.argtypes = [ctypes.POINTER(vp), i32, d]
    L.jacc_adapt_destroy.argtypes = [vp]
    L.jacc_adapt_observe.argtypes = [vp, d, d, d, ctypes.POINTER(i32)]
    L.jacc_adapt_state.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(d), ctypes.POINTER(ctypes.c_longlong)]
    L.jacc_adapt_mean_diff.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_longlong)]
    L.jacc_parallel_dim.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
    L.jacc_heat3d_noalloc.argtypes = [vp, vp, i64, i64, i64, d, vp, vp]
    _lib = L
    return L


class JaccError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def config(bx=0, by=0, tile=0, vec=0, persistent=0, order=0, march=0, rows=0):
    return Config(bx, by, tile, vec, persistent, order, march, rows)


def bounds(*pairs):
    b = Bounds()
    b.ndim = len(pairs)
    for d, (lo, hi) in enumerate(pairs):
        b.lo[d] = lo
        b.hi[d] = hi
    return b


CHOICE_MODEL, CHOICE_TUNER, CHOICE_DEFAULT = 1, 2, 3
NFEATURES = 13
MAX_CANDIDATES = 1024
_CAND_FIELDS = ("bx", "by", "tile", "vec", "persistent", "rows")


def cand_dict(c):
    """A jacc_candidate as a dict of its configuration fields and K."""
    d = {k: int(getattr(c.cfg, k)) for k in _CAND_FIELDS}
    d["K"] = int(c.K)
    return d


def cand_struct(d):
    c = Candidate()
    c.cfg = config(bx=d["bx"], by=d["by"], tile=d["tile"], vec=d["vec"], persistent=d.get("persistent", 0),
                   rows=d.get("rows", 1))
    c.K = d["K"]
    return c


def _i64s(v):
    return (ctypes.c_int64 * len(v))(*[int(x) for x in v])


def _i32s(v):
    return (ctypes.c_int * max(1, len(v)))(*[int(x) for x in v])


def stencil_kind(shape):
    return JACOBI2D if len(shape) == 2 else HEAT3D


def candidates(shape, ks):
    """jacc_candidates: the tuner's candidates (dicts) in their tie-break order."""
    L = lib()
    n = ctypes.c_int(0)
    out = (Candidate * MAX_CANDIDATES)()
    rc = L.jacc_candidates(stencil_kind(shape), _i64s(shape), len(shape), _i32s(ks), len(ks), out, MAX_CANDIDATES,
                           ctypes.byref(n))
    if rc != OK:
        raise JaccError(rc, "jacc_candidates")
    return [cand_dict(out[i]) for i in range(min(n.value, MAX_CANDIDATES))]


def features(shape, cand):
    """jacc_features: the cost model's input for one candidate."""
    out = np.zeros(NFEATURES, dtype=np.float32)
    c = cand_struct(cand)
    rc = lib().jacc_features(stencil_kind(shape), _i64s(shape), len(shape), ctypes.byref(c),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    if rc != OK:
        raise JaccError(rc, "jacc_features")
    return out


def median(samples):
    v = np.ascontiguousarray(samples, dtype=np.float64)
    return float(lib().jacc_median(v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), v.size))


def argmin(values):
    v = np.ascontiguousarray(values, dtype=np.float64)
    rc = lib().jacc_argmin(v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), v.size)
    if rc < 0:
        raise JaccError(rc, "jacc_argmin")
    return rc


def tune_opts(ks=(), db_path=None, warmup=0, reps=0):
    o = TuneOpts()
    o.warmup, o.reps, o.nks = warmup, reps, len(ks)
    for i, k in enumerate(ks):
        o.ks[i] = k
    o.db_path = db_path.encode() if db_path else None
    return o


class TorchAllocator:
    """Device memory from PyTorch's caching allocator (uint8 tensors kept
    alive until the library frees them)."""

    def __init__(self, device="cuda"):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self._a = Allocator.ALLOC(self._alloc)
        self._f = Allocator.FREE(self._free)
        self.struct = Allocator(self._a, self._f, None)

    def _alloc(self, nbytes, user):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
        except Exception:
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, user):
        self.live.pop(ptr, None)


class Context:
    """One runtime context with K partitions.

    streams: None (library-created streams), "torch" (K new torch streams,
    default priority) or a list of K torch streams.
    allocator: "torch" (PyTorch caching allocator) or "hip" (hipMalloc).
    """

    def __init__(self, K, streams="torch", allocator="torch", flags=0):
        self.L = lib()
        self.K = K
        self.flags = flags
        self._keep = []
        self.streams = None
        sp = None
        if flags & INIT_DRYRUN:
            streams = None
            if allocator == "torch":
                allocator = "hip"
        if streams == "torch":
            import torch
            self.streams = [torch.cuda.Stream() for _ in range(K)]
        elif streams is not None:
            self.streams = list(streams)
        if self.streams is not None:
            arr = (ctypes.c_void_p * K)(*[s.cuda_stream for s in self.streams])
            self._keep.append(arr)
            sp = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        ap = None
        if allocator == "torch":
            self.allocator = TorchAllocator()
            ap = ctypes.byref(self.allocator.struct)
        elif allocator != "hip":  # any object with a ctypes Allocator in .struct
            self.allocator = allocator
            ap = ctypes.byref(allocator.struct)
        self.ctx = ctypes.c_void_p()
        st = self.L.jacc_init(ctypes.byref(self.ctx), K, sp, ap, flags)
        if st != OK:
            raise JaccError(st, "jacc_init failed: " + self.L.jacc_last_error(None).decode())
        self.arrays = {}
        self._ids = {}  # id(array) -> (array, host address) of entered arrays
        self._calls = {}
        self._no_scalars = (ctypes.c_double * 1)(0.0)
        self._loop_fn = self.L.jacc_parallel_loop

    # -- helpers ---------------------------------------------------------
    def _check(self, st):
        if st != OK:
            raise JaccError(st, self.L.jacc_last_error(self.ctx).decode())
        return st

    def status(self, st):
        """Status name of a raw return code (for tests of error paths)."""
        return STATUS_NAMES.get(st, st)

    def _ptr(self, a):
        """Host address of an array; entered arrays are looked up by identity
        (the context holds them, so neither their id nor their buffer can
        change while it is open)."""
        ent = self._ids.get(id(a))
        if ent is not None and ent[0] is a:
            return ent[1]
        return a.__array_interface__["data"][0]

    def close(self):
        if self.ctx:
            st = self.L.jacc_finalize(self.ctx)
            self.ctx = ctypes.c_void_p()
            self.arrays.clear()
            self._ids.clear()
            return st
        return OK

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- data ----------------------------------------------------------------
    def enter(self, a, halo=(0, 0), whole=False, K=0, clause=COPYIN, part_dim=0, raw=False):
        """jacc_data_enter; whole: False (partitioned), True (a replica per
        partition) or SHARED (one read-only copy for every partition)."""
        assert a.flags.c_contiguous
        d = ArrayDesc()
        d.dtype = _DTYPES[a.dtype]
        d.ndim = a.ndim
        for i, e in enumerate(a.shape):
            d.extent[i] = e
        d.halo_lo, d.halo_hi = halo
        d.whole = int(whole)
        d.num_partitions = K
        d.part_dim = part_dim
        st = self.L.jacc_data_enter(self.ctx, self._ptr(a), ctypes.byref(d), clause)
        if raw:
            return st
        self._check(st)
        p = self._ptr(a)
        self.arrays[p] = a
        self._ids[id(a)] = (a, p)
        return st

    def exit(self, a, clause=COPYOUT, raw=False):
        st = self.L.jacc_data_exit(self.ctx, self._ptr(a), clause)
        return st if raw else self._check(st)

    def update(self, a, direction, lo=0, hi=-1, raw=False):
        st = self.L.jacc_update(self.ctx, self._ptr(a), direction, lo, hi)
        return st if raw else self._check(st)

    # -- loops ---------------------------------------------------------------
    def loop(self, kind, bnds, args, scalars=(), slot=-1, sync=False, cfg=None, raw=False):
        """args: list of (array, mode, off_lo, off_hi, whole)."""
        n = len(args)
        A = (Arg * n)()
        for i, (a, mode, lo, hi, whole) in enumerate(args):
            A[i] = Arg(self._ptr(a) if isinstance(a, np.ndarray) else a, mode, lo, hi, int(whole))
        S = (ctypes.c_double * max(1, len(scalars)))(*scalars)
        out = ctypes.c_double(0.0)
        st = self.L.jacc_parallel_loop(self.ctx, kind, ctypes.byref(bnds), n, A, S, len(scalars), slot,
                                       ctypes.byref(out) if sync else None,
                                       ctypes.byref(cfg) if cfg is not None else None)
        if raw:
            return st
        self._check(st)
        return out.value if sync else None

    def _stencil_call(self, kind, u_in, u_out, pairs, scalars, slot, sync, cfg, raw):
        """Marshalled arguments of a stencil call, cached per (arrays, box)
        so that a time-stepping loop pays the ctypes construction once."""
        key = (kind, self._ptr(u_in), self._ptr(u_out), pairs)
        ent = self._calls.get(key)
        if ent is None:
            if len(self._calls) > 512:
                self._calls.clear()
            A = (Arg * 2)()
            A[0] = Arg(key[1], READ, -1, 1, 0)
            A[1] = Arg(key[2], WRITE, 0, 0, 0)
            b = bounds(*pairs)
            ent = self._calls[key] = (A, b, ctypes.byref(b))
        A, _, bref = ent
        S = (ctypes.c_double * len(scalars))(*scalars) if scalars else self._no_scalars
        out = ctypes.c_double(0.0) if sync else None
        st = self._loop_fn(self.ctx, kind, bref, 2, A, S, len(scalars), slot, ctypes.byref(out) if sync else None,
                           ctypes.byref(cfg) if cfg is not None else None)
        if raw:
            return st
        self._check(st)
        return out.value if sync else None

    # convenience wrappers for the loop kinds (declared access ranges)
    def jacobi2d(self, u_in, u_out, rows=None, cols=None, cfg=None, raw=False):
        ny, nx = u_in.shape
        pairs = (tuple(rows or (1, ny - 1)), tuple(cols or (1, nx - 1)))
        return self._stencil_call(JACOBI2D, u_in, u_out, pairs, (), -1, False, cfg, raw)

    def heat3d(self, u_in, u_out, alpha, slot=-1, sync=False, cfg=None, raw=False):
        nz, ny, nx = u_in.shape
        return self._stencil_call(HEAT3D, u_in, u_out, ((1, nz - 1), (1, ny - 1), (1, nx - 1)), (alpha,), slot, sync,
                                  cfg, raw)

    def sum(self, x, squares=False, slot=-1, sync=True, rows=None, raw=False):
        b = bounds(rows or (0, x.shape[0]))
        return self.loop(SUM, b, [(x, READ, 0, 0, 0)], scalars=(1.0 if squares else 0.0,), slot=slot,
                         sync=sync, raw=raw)

    def gemm(self, A, B, C, cfg=None, raw=False):
        b = bounds((0, C.shape[0]), (0, C.shape[1]))
        return self.loop(GEMM, b, [(A, READ, 0, 0, 0), (B, READ, 0, 0, 1), (C, WRITE, 0, 0, 0)], cfg=cfg, raw=raw)

    def spmv(self, rp, col, val, x, y, cfg=None, raw=False):
        b = bounds((0, y.shape[0]))
        return self.loop(SPMV_CSR, b, [(rp, READ, 0, 1, 0), (col, READ, 0, 0, 1), (val, READ, 0, 0, 1),
                                       (x, READ, 0, 0, 1), (y, WRITE, 0, 0, 0)], cfg=cfg, raw=raw)

    def pred_chain(self, a, b, c, idx, xs, rows=None, raw=False):
        """The statement chain of the paper's filtering example over
        iterations `rows` (default all): a and b (entered whole) written
        FILTERED, c, idx (T x 3 int32) and xs read whole.  Passing the same
        array as a and b runs the loop duplicated."""
        bnd = bounds(rows or (0, xs.shape[0]))
        return self.loop(PRED_CHAIN, bnd, [(a, WRITE | FILTERED, 0, 0, 0), (b, WRITE | FILTERED, 0, 0, 0),
                                           (c, READ, 0, 0, 1), (idx, READ, 0, 0, 1), (xs, READ, 0, 0, 1)], raw=raw)

    def scatter_sq(self, x, idx, out, rows=None, raw=False):
        """out[idx[i]] = x[i]^2 with writes filtered to each partition's rows."""
        b = bounds(rows or (0, x.shape[0]))
        return self.loop(SCATTER_SQ, b, [(x, READ, 0, 0, 1), (idx, READ, 0, 0, 1),
                                         (out, WRITE | FILTERED, 0, 0, 0)], raw=raw)

    # -- batches and timing ----------------------------------------------------
    def batch_begin(self):
        return self._check(self.L.jacc_batch_begin(self.ctx))

    def batch_end(self):
        g = ctypes.c_int(-1)
        self._check(self.L.jacc_batch_end(self.ctx, ctypes.byref(g)))
        return g.value

    def batch_launch(self, graph, repeats=1, raw=False):
        st = self.L.jacc_batch_launch(self.ctx, graph, repeats)
        return st if raw else self._check(st)

    def batch_info(self, graph):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(self.L.jacc_batch_info(self.ctx, graph, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"loops": a.value, "persistent_groups": b.value, "replay_safe": bool(c.value)}

    def batch_destroy(self, graph):
        return self._check(self.L.jacc_batch_destroy(self.ctx, graph))

    def batch_time(self, graph, warmup=2, reps=10):
        out = np.zeros(reps, dtype=np.float64)
        self._check(self.L.jacc_batch_time(self.ctx, graph, warmup, reps,
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def time_loop(self, kind, bnds, args, scalars=(), cfg=None, warmup=2, reps=10, raw=False):
        """HIP-event times (ms) of `reps` runs of one loop call."""
        n = len(args)
        A = (Arg * n)()
        for i, (a, mode, lo, hi, whole) in enumerate(args):
            A[i] = Arg(self._ptr(a), mode, lo, hi, int(whole))
        S = (ctypes.c_double * max(1, len(scalars)))(*scalars)
        out = np.zeros(reps, dtype=np.float64)
        st = self.L.jacc_time_loop(self.ctx, kind, ctypes.byref(bnds), n, A, S, len(scalars),
                                   ctypes.byref(cfg) if cfg is not None else None, warmup, reps,
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if raw:
            return st, out
        self._check(st)
        return out

    def time_loop_parts(self, kind, bnds, args, scalars=(), cfg=None, nparts=None, raw=False):
        """One timed run of a loop call: (step ms, per-partition kernel ms)."""
        n = len(args)
        A = (Arg * n)()
        for i, (a, mode, lo, hi, whole) in enumerate(args):
            A[i] = Arg(self._ptr(a), mode, lo, hi, int(whole))
        S = (ctypes.c_double * max(1, len(scalars)))(*scalars)
        nk = self.K if nparts is None else nparts
        ker = np.zeros(max(1, nk), dtype=np.float64)
        step = ctypes.c_double(0.0)
        st = self.L.jacc_time_loop_parts(self.ctx, kind, ctypes.byref(bnds), n, A, S, len(scalars),
                                         ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(step),
                                         ker.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nk)
        if raw:
            return st
        self._check(st)
        return step.value, ker[:nk]

    # -- tuner and cost model ----------------------------------------------------
    def _stencil_args(self, u_in, u_out):
        A = (Arg * 2)()
        A[0] = Arg(self._ptr(u_in), READ, -1, 1, 0)
        A[1] = Arg(self._ptr(u_out), WRITE, 0, 0, 0)
        shape = u_in.shape
        b = bounds(*[(1, e - 1) for e in shape])
        scal = (ctypes.c_double * 1)(0.1)
        return A, b, scal, (1 if len(shape) == 3 else 0)

    def tune(self, u_in, u_out, ks=(), db_path=None, warmup=0, reps=0):
        """jacc_tune for the stencil sweep u_in -> u_out (JACOBI2D for 2-D,
        HEAT3D with alpha 0.1 for 3-D): (best candidate, candidates, medians)."""
        A, b, scal, ns = self._stencil_args(u_in, u_out)
        o = tune_opts(ks, db_path, warmup, reps)
        best = Candidate()
        med = np.zeros(MAX_CANDIDATES, dtype=np.float64)
        n = ctypes.c_int(0)
        self._check(self.L.jacc_tune(self.ctx, stencil_kind(u_in.shape), ctypes.byref(b), 2, A, scal, ns,
                                     ctypes.byref(o), ctypes.byref(best),
                                     med.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), MAX_CANDIDATES,
                                     ctypes.byref(n)))
        cands = candidates(u_in.shape, list(ks) if ks else [self.arrays_K(u_out)])
        assert len(cands) == n.value
        return cand_dict(best), cands, med[:n.value].copy()

    def arrays_K(self, a):
        """Partition count of a present array (from its slab table)."""
        K = 0
        while K < 64 and self.L.jacc_slab_info(self.ctx, self._ptr(a), K, None, None, None) == OK:
            K += 1
        return K

    def build_key(self):
        return self.L.jacc_build_key(self.ctx).decode()

    def model_train(self, db_path, out_path, members=3, epochs=600, batch=256, lr=1e-3, seed=0, holdout=0):
        o = TrainOpts(members, epochs, batch, lr, seed, holdout, 0)
        r = TrainReport()
        self._check(self.L.jacc_model_train(self.ctx, db_path.encode(), out_path.encode(), ctypes.byref(o),
                                            ctypes.byref(r)))
        return {"rows": r.rows, "signatures": r.signatures, "loss_first": r.loss_first, "loss_last": r.loss_last,
                "heldout_mse": r.heldout_mse}

    def model_load(self, path, raw=False):
        st = self.L.jacc_model_load(self.ctx, path.encode())
        return st if raw else self._check(st)

    def model_unload(self):
        return self._check(self.L.jacc_model_unload(self.ctx))

    def model_pick(self, shape, ks, raw=False):
        """(chosen candidate, candidates, predicted log times)."""
        best = Candidate()
        pred = np.zeros(MAX_CANDIDATES, dtype=np.float32)
        n = ctypes.c_int(0)
        st = self.L.jacc_model_pick(self.ctx, stencil_kind(shape), _i64s(shape), len(shape), _i32s(ks), len(ks),
                                    ctypes.byref(best), pred.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                    MAX_CANDIDATES, ctypes.byref(n))
        if raw:
            return st
        self._check(st)
        return cand_dict(best), candidates(shape, ks), pred[:n.value].copy()

    def choose(self, u_in, u_out, model_path=None, ks=(), db_path=None, tune=True, warmup=0, reps=0):
        """jacc_choose: (candidate, source) by the chain model -> tuner -> default."""
        A, b, scal, ns = self._stencil_args(u_in, u_out)
        o = tune_opts(ks, db_path, warmup, reps)
        out = Candidate()
        src = ctypes.c_int(0)
        self._check(self.L.jacc_choose(self.ctx, stencil_kind(u_in.shape), ctypes.byref(b), 2, A, scal, ns,
                                       model_path.encode() if model_path else None,
                                       ctypes.byref(o) if tune else None, ctypes.byref(out), ctypes.byref(src)))
        return cand_dict(out), src.value

    # -- sync / reductions -----------------------------------------------------
    def wait(self):
        return self._check(self.L.jacc_wait(self.ctx))

    def reduction(self, slot):
        out = ctypes.c_double()
        self._check(self.L.jacc_reduction_get(self.ctx, slot, ctypes.byref(out)))
        return out.value

    def reductions(self, first, count):
        out = np.zeros(count, dtype=np.float64)
        self._check(self.L.jacc_reduction_read(self.ctx, first, count,
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def slab(self, a, p):
        dev = ctypes.c_void_p()
        lo = ctypes.c_int64()
        hi = ctypes.c_int64()
        self._check(self.L.jacc_slab_info(self.ctx, self._ptr(a), p, ctypes.byref(dev), ctypes.byref(lo),
                                          ctypes.byref(hi)))
        return dev.value, lo.value, hi.value

    def last_error(self):
        return self.L.jacc_last_error(self.ctx).decode()

    # -- trace -----------------------------------------------------------------
    def trace(self):
        n = self.L.jacc_trace_len(self.ctx)
        out = []
        t = TraceOp()
        for i in range(n):
            self.L.jacc_trace_get(self.ctx, i, ctypes.byref(t))
            out.append({"op": OP_NAMES[t.op], "stream": t.stream, "array": t.array, "src": t.src, "dst": t.dst,
                        "kind": t.kind, "lo": t.lo, "hi": t.hi, "seq": t.seq})
        return out

    def trace_clear(self):
        self.L.jacc_trace_clear(self.ctx)


# ---- learned cost model -------------------------------------------------------
PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4")


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Model:
    """The FP32 cost-model network living on a context's device (its
    forward, backward and Adam run in the library's HIP kernels)."""

    H = 64

    def __init__(self, ctx, nfeat):
        self.c = ctx
        self.L = ctx.L
        self.F = nfeat
        self.P = self.L.jacc_model_nparams(nfeat)
        self.m = ctypes.c_void_p()
        ctx._check(self.L.jacc_model_create(ctx.ctx, nfeat, ctypes.byref(self.m)))

    def close(self):
        if self.m:
            self.L.jacc_model_destroy(self.m)
            self.m = ctypes.c_void_p()

    def shapes(self):
        H, F = self.H, self.F
        return {"W1": (H, F), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H, H), "b3": (H,), "w4": (H,),
                "b4": (1,)}

    def pack(self, params):
        return _f32(np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1) for k in PARAM_ORDER]))

    def unpack(self, flat):
        out, o = {}, 0
        for k in PARAM_ORDER:
            shp = self.shapes()[k]
            n = int(np.prod(shp))
            out[k] = np.asarray(flat[o:o + n]).reshape(shp)
            o += n
        return out

    def set_params(self, params):
        flat = self.pack(params) if isinstance(params, dict) else _f32(params)
        self.c._check(self.L.jacc_model_set_params(self.m, _fptr(flat), flat.size))

    def get_params(self):
        flat = np.zeros(self.P, dtype=np.float32)
        self.c._check(self.L.jacc_model_get_params(self.m, _fptr(flat), self.P))
        return self.unpack(flat)

    def set_scaler(self, mean, std):
        mu, sd = _f32(mean), _f32(std)
        self.c._check(self.L.jacc_model_set_scaler(self.m, _fptr(mu), _fptr(sd)))

    def predict(self, X):
        X = _f32(X)
        out = np.zeros(X.shape[0], dtype=np.float32)
        self.c._check(self.L.jacc_model_predict(self.m, _fptr(X), X.shape[0], _fptr(out)))
        return out

    def gradients(self, X, y):
        X, y = _f32(X), _f32(y)
        g = np.zeros(self.P, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        self.c._check(self.L.jacc_model_gradients(self.m, _fptr(X), _fptr(y), X.shape[0], _fptr(g), _fptr(loss)))
        return float(loss[0]), self.unpack(g)

    def adam_step(self, lr=1e-3):
        self.c._check(self.L.jacc_model_adam_step(self.m, ctypes.c_float(lr)))

    def train(self, X, y, epochs, batch=256, lr=1e-3, seed=0):
        X, y = _f32(X), _f32(y)
        losses = np.zeros(max(1, epochs), dtype=np.float32)
        self.c._check(self.L.jacc_model_fit(self.m, _fptr(X), _fptr(y), X.shape[0], epochs, batch,
                                            ctypes.c_float(lr), ctypes.c_uint64(seed), _fptr(losses)))
        return losses[:epochs]


ADAPT_DUPLICATE, ADAPT_PARTITION, ADAPT_DUPLICATE_FINAL = 0, 1, 2


class Adaptive:
    """Duplicate-vs-partition policy of one loop nest (jacc_adapt_*)."""

    def __init__(self, n_parts, peak_bytes_per_s):
        self.L = lib()
        h = ctypes.c_void_p()
        rc = self.L.jacc_adapt_create(ctypes.byref(h), int(n_parts), float(peak_bytes_per_s))
        if rc != OK:
            raise JaccError(rc, "jacc_adapt_create")
        self.h = h

    def observe(self, time_kernel_s, time_comm_s, write_bytes, raw=False):
        m = ctypes.c_int(-1)
        rc = self.L.jacc_adapt_observe(self.h, float(time_kernel_s), float(time_comm_s), float(write_bytes),
                                       ctypes.byref(m))
        if raw:
            return rc
        if rc != OK:
            raise JaccError(rc, "jacc_adapt_observe")
        return m.value

    def state(self):
        m = ctypes.c_int(-1)
        e = ctypes.c_double(0.0)
        cnt = (ctypes.c_longlong * 5)()
        self.L.jacc_adapt_state(self.h, ctypes.byref(m), ctypes.byref(e), cnt)
        return {"mode": m.value, "eff_dup": e.value, "n_dup": cnt[0], "eq1": cnt[1], "eq2": cnt[2], "eq3": cnt[3],
                "violations": cnt[4]}

    def mean_diff(self):
        """(mean of (t_k + t_c) - min(right sides) over the partitioned runs, their count)."""
        m = ctypes.c_double(0.0)
        n = ctypes.c_longlong(0)
        self.L.jacc_adapt_mean_diff(self.h, ctypes.byref(m), ctypes.byref(n))
        return m.value, n.value

    def close(self):
        if getattr(self, "h", None):
            self.L.jacc_adapt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def parallel_dim(parallel_iters, sequential_iters, column_major=False):
    """jacc_parallel_dim: the dimension an updated array is divided along, or
    -1 when no dimension is indexed by a parallel iterator."""
    L = lib()
    n = len(parallel_iters)
    P = (ctypes.c_int * max(1, n))(*parallel_iters)
    S = (ctypes.c_int * max(1, n))(*sequential_iters)
    out = ctypes.c_int(-2)
    rc = L.jacc_parallel_dim(n, P, S, int(bool(column_major)), ctypes.byref(out))
    if rc != OK:
        raise JaccError(rc, "jacc_parallel_dim")
    return out.value


NOALLOC_MAX_PARTIALS = 65536


def heat3d_noalloc(u_in, u_out, alpha, residual=None, stream=None):
    """jacc_heat3d_noalloc on device tensors: one heat step of the contiguous
    FP64 (nz, ny, nx) tensor `u_in` into `u_out`, the residual (a one-element
    FP64 device tensor, or None) written on the device.  `stream` is a
    torch.cuda.Stream (default: the current stream).  Raises JaccError with
    the library's reason on a nonzero status."""
    import torch
    for t in (u_in, u_out):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.dim() == 3 and t.is_contiguous()):
            raise ValueError("fields must be contiguous 3-D float64 tensors")
    if tuple(u_in.shape) != tuple(u_out.shape):
        raise ValueError("u_in and u_out differ in shape")
    res_ptr = None
    if residual is not None:
        if not (residual.dtype == torch.float64 and residual.numel() >= 1):
            raise ValueError("residual must be a float64 tensor of at least one element")
        res_ptr = residual.data_ptr()
    if stream is None:
        stream = torch.cuda.current_stream(u_in.device) if u_in.is_cuda else None
    s_ptr = stream.cuda_stream if stream is not None else None
    nz, ny, nx = u_in.shape
    rc = lib().jacc_heat3d_noalloc(u_in.data_ptr(), u_out.data_ptr(), nz, ny, nx, float(alpha), res_ptr, s_ptr)
    if rc != OK:
        raise JaccError(rc, lib().jacc_last_error(None).decode())
