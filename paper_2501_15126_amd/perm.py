"""ctypes binding of libperm_mi355x.so (include/perm.h).

Argument marshalling only: every step of the permanent (validation, the
structural check, ordering, partitioning, code generation, hipRTC, the GPU
kernels and the reduction) runs inside the C-ABI library.  If the library is
not built, importing this module raises; there is no fallback.

A matrix is a CCS tuple ``(n, colptr, rowidx, val)`` (int32, int32, float64
arrays), as produced by ``paper_2501_15126_amd.workloads``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libperm_mi355x.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libperm_mi355x.so is not built: run __graft_entry__.build() "
                      "(hipcc for gfx950) before using paper_2501_15126_amd.perm")

_lib = ctypes.CDLL(LIB_PATH)

PERM_OK, PERM_EINVAL, PERM_ETOOBIG, PERM_ENOMEM, PERM_EDEVICE, PERM_ECOMPILE, PERM_EAGAIN, \
    PERM_ENOTREADY, PERM_ECANCELED = range(9)
STATUS_NAMES = ["PERM_OK", "PERM_EINVAL", "PERM_ETOOBIG", "PERM_ENOMEM", "PERM_EDEVICE",
                "PERM_ECOMPILE", "PERM_EAGAIN", "PERM_ENOTREADY", "PERM_ECANCELED"]
MODES = {"auto": 0, "pure": 1, "hybrid": 2}
MAX_N = 64


class PermError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES[status] if 0 <= status < 9 else status, message))
        self.status = status


class PermCsc(ctypes.Structure):
    # the three arrays as plain addresses (int32, int32, float64): setting an
    # address is cheaper than building a typed ctypes pointer on every call
    _fields_ = [("n", ctypes.c_int32), ("colptr", ctypes.c_void_p), ("rowidx", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class PermOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("chunk_log2", ctypes.c_int32), ("unroll_log2", ctypes.c_int32),
                ("block", ctypes.c_int32), ("vgpr_budget", ctypes.c_int32), ("force_k", ctypes.c_int32),
                ("force_c", ctypes.c_int32), ("max_levels", ctypes.c_int32), ("zero_skip", ctypes.c_int32),
                ("batch_mode", ctypes.c_int32), ("batch_kappa_shift", ctypes.c_int32),
                ("cold_tier", ctypes.c_int32), ("gr_ratio", ctypes.c_double),
                ("hip_stream", ctypes.c_void_p), ("block_partials", ctypes.POINTER(ctypes.c_double)),
                ("block_partials_cap", ctypes.c_int64), ("progress", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("block_queue", ctypes.c_int32), ("exact", ctypes.c_int32), ("exact_passes", ctypes.c_int32),
                ("copy_cols", ctypes.c_int32)]


class PermBatchStats(ctypes.Structure):
    _fields_ = [("wall_ms", ctypes.c_double), ("prep_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("steps", ctypes.c_double), ("count", ctypes.c_int32), ("singular", ctypes.c_int32),
                ("launches", ctypes.c_int32), ("pad", ctypes.c_int32), ("fp64_ops", ctypes.c_double),
                ("flops", ctypes.c_double), ("exact_ops", ctypes.c_double), ("exact_certified", ctypes.c_int32),
                ("exact_uncertified", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("graph_captures", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name not in ("pad", "pad2")}


class PermStats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("reduce_ms", ctypes.c_double), ("compile_ms", ctypes.c_double),
                ("host_ms", ctypes.c_double), ("total_ms", ctypes.c_double), ("steps", ctypes.c_double),
                ("ops_per_step", ctypes.c_double), ("flops_per_step", ctypes.c_double),
                ("sum_hi", ctypes.c_double), ("sum_lo", ctypes.c_double), ("evaluated_steps", ctypes.c_double),
                ("nblocks", ctypes.c_int64), ("nchunks", ctypes.c_int64),
                ("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("k", ctypes.c_int32), ("c", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("chunk_log2", ctypes.c_int32), ("unroll_log2", ctypes.c_int32), ("block", ctypes.c_int32),
                ("vgprs", ctypes.c_int32), ("sgprs", ctypes.c_int32), ("scratch_bytes", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32), ("cache_hit", ctypes.c_int32),
                ("singular", ctypes.c_int32), ("waves_hint", ctypes.c_int32), ("vgpr_spills", ctypes.c_int32),
                ("exact", ctypes.c_int32), ("exact_passes", ctypes.c_int32), ("estimate", ctypes.c_double),
                ("err_bound", ctypes.c_double), ("exact_ops_per_step", ctypes.c_double),
                ("exact_bound_log2", ctypes.c_int32), ("copy_cols", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = ctypes.POINTER
_lib.perm_sparse.restype = ctypes.c_double
_lib.perm_sparse.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.perm_sparse_ex.restype = ctypes.c_int
_lib.perm_sparse_ex.argtypes = [_P(PermCsc), _P(PermOpts), _P(ctypes.c_double), _P(PermStats)]
_lib.perm_batch.restype = ctypes.c_int
_lib.perm_batch.argtypes = [ctypes.c_int32, _P(PermCsc), _P(PermOpts), _P(ctypes.c_double)]
_lib.perm_batch_ex.restype = ctypes.c_int
_lib.perm_batch_ex.argtypes = [ctypes.c_int32, _P(PermCsc), _P(PermOpts), _P(ctypes.c_double), _P(PermBatchStats)]
_lib.perm_batch_noalloc.restype = ctypes.c_int
_lib.perm_batch_noalloc.argtypes = [ctypes.c_int32, _P(PermCsc), _P(PermOpts), _P(ctypes.c_double),
                                    _P(PermBatchStats)]
_lib.perm_plan.restype = ctypes.c_int
_lib.perm_plan.argtypes = [_P(PermCsc), _P(PermOpts), _P(ctypes.c_int32), _P(ctypes.c_int32),
                           _P(ctypes.c_double), _P(ctypes.c_int32), _P(ctypes.c_int32), _P(ctypes.c_int32),
                           _P(ctypes.c_int32)]
_lib.perm_partition.restype = ctypes.c_int
_lib.perm_partition.argtypes = [_P(PermCsc), _P(ctypes.c_double), ctypes.c_double, _P(ctypes.c_int32),
                                _P(ctypes.c_int32)]
_lib.perm_codegen.restype = ctypes.c_int
_lib.perm_codegen.argtypes = [_P(PermCsc), _P(PermOpts), ctypes.c_char_p, ctypes.c_size_t,
                              _P(ctypes.c_size_t)]
_lib.perm_compile_info.restype = ctypes.c_int
_lib.perm_compile_info.argtypes = [_P(PermCsc), _P(PermOpts), _P(PermStats)]
_lib.perm_batch_describe.restype = ctypes.c_int
_lib.perm_batch_describe.argtypes = [_P(PermCsc), _P(PermOpts), _P(ctypes.c_int32), _P(ctypes.c_double),
                                     ctypes.c_size_t, _P(ctypes.c_size_t), _P(ctypes.c_int32), ctypes.c_size_t,
                                     _P(ctypes.c_size_t)]
class PermTuneStats(ctypes.Structure):
    _fields_ = [("default_ms", ctypes.c_double), ("best_ms", ctypes.c_double), ("sample_fraction", ctypes.c_double),
                ("tune_ms", ctypes.c_double), ("candidates", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad"}


_lib.perm_autotune.restype = ctypes.c_int
_lib.perm_autotune.argtypes = [_P(PermCsc), _P(PermOpts), _P(PermOpts), _P(PermTuneStats)]
_lib.perm_batch_autotune.restype = ctypes.c_int
_lib.perm_batch_autotune.argtypes = [ctypes.c_int32, _P(PermCsc), _P(PermOpts), _P(PermOpts), _P(PermTuneStats)]
_lib.perm_last_error.restype = ctypes.c_char_p
_lib.perm_last_error.argtypes = []
_lib.perm_version.restype = ctypes.c_char_p
_lib.perm_version.argtypes = []

class PermServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("pending", ctypes.c_uint64), ("active", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("arena_used", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64), ("busy_ms", ctypes.c_double),
                ("exact_certified", ctypes.c_uint64), ("exact_uncertified", ctypes.c_uint64),
                ("extra_passes", ctypes.c_uint64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib.perm_server_create.restype = ctypes.c_void_p
_lib.perm_server_create.argtypes = [_P(PermOpts), ctypes.c_size_t, ctypes.c_int32, ctypes.c_double]
_lib.perm_submit.restype = ctypes.c_int
_lib.perm_submit.argtypes = [ctypes.c_void_p, _P(PermCsc), _P(ctypes.c_uint64)]
_lib.perm_poll.restype = ctypes.c_int
_lib.perm_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, _P(ctypes.c_double)]
_lib.perm_wait.restype = ctypes.c_int
_lib.perm_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, _P(ctypes.c_double)]
_lib.perm_server_get_stats.restype = ctypes.c_int
_lib.perm_server_get_stats.argtypes = [ctypes.c_void_p, _P(PermServerStats)]
_lib.perm_server_destroy.restype = None
_lib.perm_server_destroy.argtypes = [ctypes.c_void_p]

# every symbol include/perm.h declares
EXPORTED = ["perm_sparse", "perm_sparse_ex", "perm_batch", "perm_batch_ex", "perm_batch_noalloc",
            "perm_server_create", "perm_submit",
            "perm_poll", "perm_wait", "perm_server_get_stats", "perm_server_destroy", "perm_batch_describe",
            "perm_plan", "perm_partition", "perm_codegen",
            "perm_compile_info", "perm_autotune", "perm_batch_autotune", "perm_exact_recover", "perm_exact_primes",
            "perm_last_error", "perm_version"]


_lib.perm_exact_recover.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_double), _P(ctypes.c_double),
                                    _P(ctypes.c_int32), _P(ctypes.c_int32)]
_lib.perm_exact_primes.restype = None
_lib.perm_exact_primes.argtypes = [_P(ctypes.c_double)]


def exact_primes():
    out = (ctypes.c_double * 3)()
    _lib.perm_exact_primes(out)
    return [int(v) for v in out]


def exact_recover(n, hi, lo, abs_sum, chunk_log2, resid):
    """perm_exact_recover: returns (value, estimate, err_bound, certified, more)."""
    r = (ctypes.c_double * 3)(*[float(v) for v in resid])
    out = (ctypes.c_double * 3)()
    cert, more = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.perm_exact_recover(int(n), float(hi), float(lo), float(abs_sum), int(chunk_log2), len(resid), r,
                                   out, ctypes.byref(cert), ctypes.byref(more)))
    return out[0], out[1], out[2], bool(cert.value), bool(more.value)


def library():
    return _lib


def last_error() -> str:
    return _lib.perm_last_error().decode()


def version() -> str:
    return _lib.perm_version().decode()


class _Csc:
    """Holds the arrays alive while the C struct points at them."""

    def __init__(self, ccs):
        n, colptr, rowidx, val = ccs
        self.colptr = np.ascontiguousarray(colptr, dtype=np.int32)
        self.rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        if self.rowidx.size == 0:  # keep valid pointers for empty matrices
            self.rowidx = np.zeros(1, np.int32)
            self.val = np.zeros(1, np.float64)
        self.c = PermCsc(int(n), self.colptr.ctypes.data, self.rowidx.ctypes.data, self.val.ctypes.data)


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):  # torch.cuda.Stream
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def make_opts(mode="auto", chunk_log2=0, unroll_log2=0, block=0, vgpr_budget=0, force_k=0, force_c=0,
              max_levels=0, gr_ratio=0.0, stream=None, zero_skip="auto", batch_mode="streams",
              batch_kappa_shift=0, cold_tier="global", progress=False, waves_per_simd=0,
              block_queue=True, exact="auto", exact_passes=0, copy_cols=0):
    o = PermOpts()
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.chunk_log2, o.unroll_log2, o.block = chunk_log2, unroll_log2, block
    o.vgpr_budget, o.force_k, o.force_c, o.max_levels = vgpr_budget, force_k, force_c, max_levels
    o.gr_ratio = gr_ratio
    o.zero_skip = {"auto": 0, True: 1, False: -1}[zero_skip]
    o.batch_mode = {"streams": 0, "graph": 1, "persistent": 1, "sequential": 2, "one_stream": 3}[batch_mode]
    o.batch_kappa_shift = batch_kappa_shift
    o.cold_tier = {"global": 0, "lds": 1}[cold_tier]
    o.progress = 1 if progress else 0
    o.waves_per_simd = waves_per_simd
    o.block_queue = (0 if block_queue is True else -1 if block_queue is False else int(block_queue))
    o.exact = {"auto": 0, True: 1, False: -1}[exact]
    o.exact_passes = exact_passes
    o.copy_cols = copy_cols
    o.hip_stream = _stream_handle(stream)
    return o


def _check(status):
    if status != PERM_OK:
        raise PermError(status, last_error())


def perm_sparse(n, colptr, rowidx, val) -> float:
    """Permanent (NaN on error, as the C call)."""
    m = _Csc((n, colptr, rowidx, val))
    return _lib.perm_sparse(m.c.n, m.c.colptr, m.c.rowidx, m.c.val)


def perm_sparse_ex(ccs, block_partials=False, **opts):
    """Returns (value, stats dict[, partials array (nblocks, 2)])."""
    m = _Csc(ccs)
    o = make_opts(**opts)
    parts = None
    if block_partials:
        plan_stats = compile_plan_stats(ccs, **opts)
        nb = max(1, int(plan_stats["nblocks"]))
        parts = np.zeros((nb, 2), np.float64)
        o.block_partials = parts.ctypes.data_as(_P(ctypes.c_double))
        o.block_partials_cap = nb
    out = ctypes.c_double()
    st = PermStats()
    _check(_lib.perm_sparse_ex(ctypes.byref(m.c), ctypes.byref(o), ctypes.byref(out), ctypes.byref(st)))
    if block_partials:
        return out.value, st.as_dict(), parts
    return out.value, st.as_dict()


def perm_batch(mats, **opts):
    return perm_batch_ex(mats, **opts)[0]


def perm_batch_ex(mats, **opts):
    """Returns (results array, batch stats dict)."""
    held = [_Csc(c) for c in mats]
    arr = (PermCsc * max(1, len(held)))(*[h.c for h in held])
    out = np.zeros(max(1, len(held)), np.float64)
    o = make_opts(**opts)
    st = PermBatchStats()
    _check(_lib.perm_batch_ex(len(held), arr, ctypes.byref(o), out.ctypes.data_as(_P(ctypes.c_double)),
                              ctypes.byref(st)))
    return out[:len(held)], st.as_dict()


def perm_batch_noalloc(mats, **opts):
    """perm_batch_ex without device allocation (the library's fixed scratch
    region); returns (results array, batch stats dict)."""
    held = [_Csc(c) for c in mats]
    arr = (PermCsc * max(1, len(held)))(*[h.c for h in held])
    out = np.zeros(max(1, len(held)), np.float64)
    o = make_opts(**opts)
    st = PermBatchStats()
    _check(_lib.perm_batch_noalloc(len(held), arr, ctypes.byref(o), out.ctypes.data_as(_P(ctypes.c_double)),
                                   ctypes.byref(st)))
    return out[:len(held)], st.as_dict()


def _opts_kwargs(o):
    """make_opts keyword arguments that rebuild the tuning fields of o."""
    inv = {v: k for k, v in MODES.items()}
    return {"mode": inv.get(o.mode, o.mode), "chunk_log2": o.chunk_log2, "unroll_log2": o.unroll_log2,
            "block": o.block, "vgpr_budget": o.vgpr_budget, "force_k": o.force_k, "force_c": o.force_c,
            "max_levels": o.max_levels, "gr_ratio": o.gr_ratio,
            "zero_skip": {0: "auto", 1: True, -1: False}[o.zero_skip],
            "batch_mode": {0: "streams", 1: "graph", 2: "sequential", 3: "one_stream"}[o.batch_mode],
            "batch_kappa_shift": o.batch_kappa_shift, "cold_tier": {0: "global", 1: "lds"}[o.cold_tier],
            "waves_per_simd": o.waves_per_simd,
            "block_queue": {0: True, -1: False}.get(o.block_queue, o.block_queue),
            "exact": {0: "auto", 1: True, -1: False}[o.exact], "exact_passes": o.exact_passes,
            "copy_cols": o.copy_cols}


def perm_autotune(ccs, **opts):
    """Times candidate launch options for one matrix (perm_autotune); returns
    (keyword options for perm_sparse_ex, tuning stats dict)."""
    m = _Csc(ccs)
    o = make_opts(**opts)
    best = PermOpts()
    st = PermTuneStats()
    _check(_lib.perm_autotune(ctypes.byref(m.c), ctypes.byref(o), ctypes.byref(best), ctypes.byref(st)))
    return _opts_kwargs(best), st.as_dict()


def perm_batch_autotune(mats, **opts):
    """Times candidate perm_batch options on the batch (perm_batch_autotune);
    returns (keyword options for perm_batch_ex, tuning stats dict)."""
    held = [_Csc(c) for c in mats]
    arr = (PermCsc * max(1, len(held)))(*[h.c for h in held])
    o = make_opts(**opts)
    best = PermOpts()
    st = PermTuneStats()
    _check(_lib.perm_batch_autotune(len(held), arr, ctypes.byref(o), ctypes.byref(best), ctypes.byref(st)))
    return _opts_kwargs(best), st.as_dict()


def perm_plan(ccs, **opts):
    m = _Csc(ccs)
    n = int(ccs[0])
    rp = np.zeros(n, np.int32)
    cp = np.zeros(n, np.int32)
    tau = np.zeros(2 * n + 1, np.float64)
    k, c, lev, rank = (ctypes.c_int32() for _ in range(4))
    o = make_opts(**opts)
    _check(_lib.perm_plan(ctypes.byref(m.c), ctypes.byref(o), rp.ctypes.data_as(_P(ctypes.c_int32)),
                          cp.ctypes.data_as(_P(ctypes.c_int32)), tau.ctypes.data_as(_P(ctypes.c_double)),
                          ctypes.byref(k), ctypes.byref(c), ctypes.byref(lev), ctypes.byref(rank)))
    return {"row_perm": rp.tolist(), "col_perm": cp.tolist(), "tau": tau, "k": k.value, "c": c.value,
            "levels": lev.value, "structural_rank": rank.value}


def perm_partition(ordered_ccs, tau, gr_ratio=16.0):
    m = _Csc(ordered_ccs)
    tau = np.ascontiguousarray(tau, np.float64)
    k, c = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.perm_partition(ctypes.byref(m.c), tau.ctypes.data_as(_P(ctypes.c_double)), gr_ratio,
                               ctypes.byref(k), ctypes.byref(c)))
    return k.value, c.value


def perm_codegen(ccs, **opts) -> str:
    m = _Csc(ccs)
    o = make_opts(**opts)
    ln = ctypes.c_size_t()
    _check(_lib.perm_codegen(ctypes.byref(m.c), ctypes.byref(o), None, 0, ctypes.byref(ln)))
    buf = ctypes.create_string_buffer(ln.value + 1)
    _check(_lib.perm_codegen(ctypes.byref(m.c), ctypes.byref(o), buf, ln.value + 1, ctypes.byref(ln)))
    return buf.value.decode()


def compile_info(ccs, **opts):
    """hipRTC-compile the generated kernel (no GPU needed); plan + resources."""
    m = _Csc(ccs)
    o = make_opts(**opts)
    st = PermStats()
    _check(_lib.perm_compile_info(ctypes.byref(m.c), ctypes.byref(o), ctypes.byref(st)))
    return st.as_dict()


def batch_describe(ccs, **opts):
    """The batch kernels' data for one matrix (see perm_batch_describe)."""
    m = _Csc(ccs)
    o = make_opts(**opts)
    desc = (ctypes.c_int32 * 8)()
    nv, nt = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.perm_batch_describe(ctypes.byref(m.c), ctypes.byref(o), desc, None, 0, ctypes.byref(nv), None, 0,
                                    ctypes.byref(nt)))
    vals = np.zeros(max(1, nv.value), np.float64)
    tops = np.zeros(max(1, nt.value), np.int32)
    _check(_lib.perm_batch_describe(ctypes.byref(m.c), ctypes.byref(o), desc,
                                    vals.ctypes.data_as(_P(ctypes.c_double)), vals.size, ctypes.byref(nv),
                                    tops.ctypes.data_as(_P(ctypes.c_int32)), tops.size, ctypes.byref(nt)))
    keys = ["n", "ng", "kappa", "zero_skip", "chunk_top", "singular", "exact"]
    return dict(zip(keys, list(desc))), vals[:nv.value], tops[:nt.value]


def compile_plan_stats(ccs, **opts):
    return compile_info(ccs, **opts)


class Server:
    """Submit/poll permanent server (perm_server_*)."""

    def __init__(self, device_mem_budget=0, max_inflight=0, round_steps=0.0, **opts):
        self._opts = make_opts(**opts)
        h = _lib.perm_server_create(ctypes.byref(self._opts), device_mem_budget, max_inflight, float(round_steps))
        if not h:
            raise PermError(PERM_EDEVICE, last_error())
        self._h = ctypes.c_void_p(h)

    def submit(self, ccs) -> int:
        m = _Csc(ccs)
        t = ctypes.c_uint64()
        _check(_lib.perm_submit(self._h, ctypes.byref(m.c), ctypes.byref(t)))
        return t.value

    def try_submit(self, ccs):
        """Ticket, or None when the server is full (PERM_EAGAIN)."""
        m = _Csc(ccs)
        t = ctypes.c_uint64()
        st = _lib.perm_submit(self._h, ctypes.byref(m.c), ctypes.byref(t))
        if st == PERM_EAGAIN:
            return None
        _check(st)
        return t.value

    def poll(self, ticket):
        """The result, or None while the request is not done."""
        out = ctypes.c_double()
        st = _lib.perm_poll(self._h, ticket, ctypes.byref(out))
        if st == PERM_ENOTREADY:
            return None
        _check(st)
        return out.value

    def wait(self, ticket) -> float:
        out = ctypes.c_double()
        _check(_lib.perm_wait(self._h, ticket, ctypes.byref(out)))
        return out.value

    def stats(self):
        st = PermServerStats()
        _check(_lib.perm_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self._h:
            _lib.perm_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
