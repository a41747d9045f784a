"""ctypes binding of include/hlu.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loaded first so that libhlu.so shares torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
build_lib_path = os.path.join(HERE, "libhlu.so")

if not os.path.exists(build_lib_path):
    raise ImportError(
        f"{build_lib_path} is missing: build it with `python -c 'import __graft_entry__ as g; "
        "g.build()'` (no CPU fallback exists)")

lib = C.CDLL(build_lib_path)

KERNEL_WEIGHTED, KERNEL_POINT, KERNEL_LOG1D, KERNEL_LOG2D = 0, 1, 2, 3
OP_LU, OP_PRODUCT, OP_INVERSE = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1

HLU_OK, HLU_ERR_ARG, HLU_ERR_NOMEM, HLU_ERR_DEVICE = 0, 1, 2, 3
HLU_ERR_SINGULAR, HLU_ERR_NOT_CONVERGED, HLU_ERR_STATE = 4, 5, 6
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_NOMEM", 3: "ERR_DEVICE", 4: "ERR_SINGULAR",
                5: "ERR_NOT_CONVERGED", 6: "ERR_STATE"}


class Params(C.Structure):
    _fields_ = [("kernel", C.c_int), ("eta", C.c_double), ("leaf_size", C.c_int),
                ("fixed_rank", C.c_int), ("eps_factor", C.c_double),
                ("rank_cap_factor", C.c_int), ("eps_matvec", C.c_double),
                ("rank_cap_matvec", C.c_int), ("precision", C.c_int),
                ("refine_tol", C.c_double), ("refine_max_iter", C.c_int),
                ("max_nrhs", C.c_int), ("seed", C.c_uint64),
                ("scratch_cap_bytes", C.c_int64), ("operation", C.c_int),
                ("kernel_b", C.c_int), ("device_assembly", C.c_int)]


class Info(C.Structure):
    _fields_ = [("info", C.c_int64), ("iters", C.c_int), ("eta_hist", C.c_double * 16),
                ("eta_final", C.c_double), ("cap_hits", C.c_int64), ("max_rank", C.c_int64)]


class PlanStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("leaves", C.c_int64), ("dense_blocks", C.c_int64),
                ("lowrank_blocks", C.c_int64), ("ops_factor", C.c_int64),
                ("waves_factor", C.c_int64), ("ops_solve", C.c_int64),
                ("waves_solve", C.c_int64), ("flops_factor_model", C.c_double),
                ("bytes_factor_region", C.c_int64), ("bytes_matvec_region", C.c_int64),
                ("bytes_scratch", C.c_int64), ("bytes_total", C.c_int64),
                ("offset_scratch", C.c_int64)]


OP_TYPES = 12   # HLU_OP_TYPES of the C header

# Host views of the schedule descriptors (struct PRef / Op / Term of the
# kernels' header), as returned by HLU.schedule_ops.
PREF_DTYPE = np.dtype([("ptr", "<u8"), ("rankp", "<u8"), ("ld", "<i4"), ("rows", "<i4"),
                       ("cols", "<i4"), ("dt", "u1"), ("trans", "u1"), ("kind", "u1"),
                       ("pad", "u1")])
OP_DTYPE = np.dtype([("type", "<i4"), ("i0", "<i4"), ("i1", "<i4"), ("i2", "<i4"),
                     ("d0", "<f8"), ("cost", "<u8"), ("p", PREF_DTYPE, (4,))])
TERM_DTYPE = np.dtype([("X", PREF_DTYPE), ("Y", PREF_DTYPE), ("xo", "<i4"), ("yo", "<i4"),
                       ("pad", "<i4", (2,))])
assert PREF_DTYPE.itemsize == 32 and OP_DTYPE.itemsize == 160 and TERM_DTYPE.itemsize == 80

_P = C.c_void_p
_sig = {
    "hlu_plan": (C.c_int, [_P, _P, C.c_int64, C.POINTER(Params), C.POINTER(_P)]),
    "hlu_required_bytes": (C.c_size_t, [_P]),
    "hlu_validate": (C.c_int, [_P]),
    "hlu_bind": (C.c_int, [_P, _P, C.c_size_t]),
    "hlu_assemble": (C.c_int, [_P, _P]),
    "hlu_reset": (C.c_int, [_P, _P]),
    "hlu_clone": (C.c_int, [_P, C.POINTER(_P)]),
    "hlu_assemble_from": (C.c_int, [_P, _P, _P]),
    "hlu_set_workers": (C.c_int, [_P, C.c_int]),
    "hlu_set_priorities": (C.c_int, [_P, C.c_double, C.c_int, C.POINTER(C.c_int32)]),
    "hlu_factor": (C.c_int, [_P, _P]),
    "hlu_batch_create": (C.c_int, [C.POINTER(_P), C.c_int, C.POINTER(_P)]),
    "hlu_batch_required_bytes": (C.c_size_t, [_P]),
    "hlu_batch_bind": (C.c_int, [_P, _P, C.c_size_t]),
    "hlu_batch_factor": (C.c_int, [_P, _P]),
    "hlu_batch_sync": (C.c_int, [_P, _P]),
    "hlu_batch_destroy": (None, [_P]),
    "hlu_factor_profile": (C.c_int, [_P, _P, _P, _P]),
    "hlu_set_graph": (C.c_int, [_P, C.c_int]),
    "hlu_set_refinement": (C.c_int, [_P, C.c_double, C.c_int]),
    "hlu_set_executor": (C.c_int, [_P, C.c_int]),
    "hlu_factor_records": (C.c_int, [_P, _P, _P]),
    "hlu_factor_graph": (C.c_int, [_P, _P, _P, _P]),
    "hlu_schedule_records": (C.c_int, [_P, C.c_int, _P, _P]),
    "hlu_schedule_graph": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "hlu_schedule_ops": (C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P]),
    "hlu_solve": (C.c_int, [_P, _P, _P, C.c_int, C.c_int64, _P]),
    "hlu_matvec": (C.c_int, [_P, _P, _P, C.c_int, C.c_int64, _P]),
    "hlu_sync": (C.c_int, [_P, _P, C.POINTER(Info)]),
    "hlu_get_stats": (C.c_int, [_P, C.POINTER(PlanStats)]),
    "hlu_factor_cost": (C.c_int, [_P, _P, _P, _P]),
    "hlu_factor_batches": (C.c_int, [_P, _P]),
    "hlu_get_perm": (C.c_int, [_P, _P]),
    "hlu_export_factors": (C.c_int, [_P, _P, _P, _P]),
    "hlu_export_pivots": (C.c_int, [_P, _P, _P]),
    "hlu_import_blocks": (C.c_int, [_P, C.c_char_p]),
    "hlu_export_blocks": (C.c_int, [_P, C.c_char_p]),
    "hlu_export_result": (C.c_int, [_P, _P, C.c_int64]),
    "hlu_set_tuning": (C.c_int, [_P, C.c_int]),
    "hlu_batch_set_tuning": (C.c_int, [_P, C.c_int, C.c_int]),
    "hlu_destroy": (None, [_P]),
    "hlu_last_error": (C.c_char_p, []),
    "hlu_getrf_batched": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, _P]),
    "hlu_truncate_add": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_double, C.c_int, _P]),
    "hlu_truncate_add_noalloc": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, C.c_int, C.c_int,
                                           C.c_int, C.c_int, C.c_double, C.c_int, _P]),
    "hlu_static_scratch_bytes": (C.c_size_t, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class HLUError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st):
    if st != HLU_OK:
        raise HLUError(st, lib.hlu_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def make_params(kernel=KERNEL_WEIGHTED, eta=2.0, leaf=32, fixed_rank=0, eps=1e-6, cap=32,
                eps_mv=1e-12, cap_mv=64, precision=PREC_FP64, refine_tol=0.0,
                refine_max_iter=10, max_nrhs=32, seed=0, scratch_cap=0, operation=0,
                kernel_b=0, device_assembly=0):
    return Params(kernel, eta, leaf, fixed_rank, eps, cap, eps_mv, cap_mv, precision,
                  refine_tol, refine_max_iter, max_nrhs, seed, scratch_cap, operation, kernel_b,
                  device_assembly)


class HLU:
    """One H-matrix on one device: plan on construction; `bind_and_assemble`
    allocates the device buffer through torch and uploads the blocks."""

    def __init__(self, xyz, area, device="cuda", assemble=True, **kw):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        area = np.ascontiguousarray(area, dtype=np.float64)
        self.n = xyz.shape[0]
        self.params = make_params(**kw)
        h = C.c_void_p()
        _check(lib.hlu_plan(xyz.ctypes.data_as(_P), area.ctypes.data_as(_P), self.n,
                            C.byref(self.params), C.byref(h)))
        self.h = h
        self.device = device
        self.buf = None
        if assemble:
            self.bind_and_assemble()

    def clone(self, bind=True, stream=None):
        """A handle over the same plan with a buffer of its own, filled from
        this (assembled) handle device to device when `bind` is true."""
        c = HLU.__new__(HLU)
        h = C.c_void_p()
        _check(lib.hlu_clone(self.h, C.byref(h)))
        c.h, c.n, c.params, c.device, c.buf = h, self.n, self.params, self.device, None
        if bind:
            c.bind()
            _check(lib.hlu_assemble_from(c.h, self.h, _stream(stream)))
        return c

    def assemble_from(self, src, stream=None):
        _check(lib.hlu_assemble_from(self.h, src.h, _stream(stream)))

    def import_blocks(self, path):
        """Replace the factored copy's blocks by those of a block file
        (format in include/hlu.h), e.g. the oracle's A_H."""
        _check(lib.hlu_import_blocks(self.h, str(path).encode()))

    def export_result(self):
        """A B (product plan) or A^-1 (inverse plan) after factor(), dense,
        original point order (numpy, n <= 16384)."""
        out = np.zeros((self.n, self.n), order="F")
        _check(lib.hlu_export_result(self.h, out.ctypes.data_as(_P), self.n))
        return out

    def export_blocks(self, path):
        """Write the factored copy's current blocks to a block file."""
        _check(lib.hlu_export_blocks(self.h, str(path).encode()))

    def set_tuning(self, trunc_width):
        """Widest stack of a truncation pass in later dataflow factorisations
        (0: 64)."""
        _check(lib.hlu_set_tuning(self.h, int(trunc_width)))

    def set_workers(self, workers):
        """Dataflow workgroups per launch (0: one per compute unit)."""
        _check(lib.hlu_set_workers(self.h, int(workers)))

    def set_priorities(self, slack_frac, high_workers):
        """Flag the factor ops within slack_frac of the longest path (from
        the last factorisation's records) for the high ring served by
        high_workers workgroups (0 clears); returns the flagged count."""
        nf = C.c_int32(0)
        _check(lib.hlu_set_priorities(self.h, float(slack_frac), int(high_workers),
                                      C.byref(nf)))
        return int(nf.value)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib.hlu_destroy(h)
            self.h = None

    # -- host-side queries ------------------------------------------------
    @property
    def required_bytes(self):
        return int(lib.hlu_required_bytes(self.h))

    def stats(self):
        s = PlanStats()
        _check(lib.hlu_get_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in PlanStats._fields_}

    def perm(self):
        p = np.empty(self.n, dtype=np.int64)
        _check(lib.hlu_get_perm(self.h, p.ctypes.data_as(_P)))
        return p

    def validate(self):
        _check(lib.hlu_validate(self.h))

    def batches(self):
        b = np.zeros(OP_TYPES, dtype=np.int64)
        _check(lib.hlu_factor_batches(self.h, b.ctypes.data_as(_P)))
        return b

    # -- device ------------------------------------------------------------
    def bind(self, buf=None):
        nbytes = self.required_bytes
        if buf is None:
            buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        self.buf = buf
        _check(lib.hlu_bind(self.h, C.c_void_p(buf.data_ptr() + off), nbytes))

    def bind_and_assemble(self, stream=None):
        self.bind()
        _check(lib.hlu_assemble(self.h, _stream(stream)))

    def set_refinement(self, tol, max_iter=10):
        """Refinement target of later solves (0: the plain solve)."""
        _check(lib.hlu_set_refinement(self.h, float(tol), int(max_iter)))

    def set_graph(self, enable):
        _check(lib.hlu_set_graph(self.h, int(bool(enable))))

    def set_executor(self, mode):
        """0: one launch per wave; 1: persistent dataflow executor."""
        _check(lib.hlu_set_executor(self.h, int(mode)))

    def reset(self, stream=None):
        _check(lib.hlu_reset(self.h, _stream(stream)))

    def factor(self, stream=None):
        _check(lib.hlu_factor(self.h, _stream(stream)))

    def factor_profile(self, stream=None):
        """Factor with per-launch events; returns (ms per op type, launches)."""
        ms = np.zeros(OP_TYPES)
        ln = np.zeros(OP_TYPES, dtype=np.int64)
        _check(lib.hlu_factor_profile(self.h, _stream(stream), ms.ctypes.data_as(_P),
                                      ln.ctypes.data_as(_P)))
        return ms, ln

    def sync(self, stream=None, check=True):
        inf = Info()
        st = lib.hlu_sync(self.h, _stream(stream), C.byref(inf))
        if check:
            _check(st)
        return st, inf

    @staticmethod
    def _cm(b):
        """(n,) or (n, k) tensor -> column-major (k, n) contiguous FP64."""
        if b.dim() == 1:
            b = b[:, None]
        return b.t().contiguous().to(torch.float64)

    def solve(self, b, stream=None):
        """x = A^{-1} b; b: CUDA tensor (n,) or (n, nrhs), original order."""
        one = b.dim() == 1
        bc = self._cm(b)
        xc = torch.empty_like(bc)
        nrhs = bc.shape[0]
        _check(lib.hlu_solve(self.h, _ptr(bc), _ptr(xc), nrhs, self.n, _stream(stream)))
        x = xc.t()
        return x[:, 0] if one else x

    def solve_cm(self, bc, xc, stream=None):
        """Column-major solve on preallocated (nrhs, n) tensors."""
        _check(lib.hlu_solve(self.h, _ptr(bc), _ptr(xc), bc.shape[0], self.n, _stream(stream)))

    def matvec(self, x, stream=None):
        one = x.dim() == 1
        xc = self._cm(x)
        yc = torch.empty_like(xc)
        _check(lib.hlu_matvec(self.h, _ptr(xc), _ptr(yc), xc.shape[0], self.n, _stream(stream)))
        y = yc.t()
        return y[:, 0] if one else y

    def factor_cost(self):
        f = np.zeros(OP_TYPES)
        b = np.zeros(OP_TYPES)
        c = np.zeros(OP_TYPES, dtype=np.int64)
        _check(lib.hlu_factor_cost(self.h, f.ctypes.data_as(_P), b.ctypes.data_as(_P),
                                   c.ctypes.data_as(_P)))
        return f, b, c

    def factor_records(self):
        """(records (ops, 8) float64, info (ops, 4) int32) of the last factor."""
        return self.schedule_records(0)

    def schedule_records(self, which):
        """Per-op records of schedule `which` (0: factor, 1: last solve sweep)."""
        no = self.stats()["ops_solve" if which else "ops_factor"]
        r = np.zeros((no, 8))
        i = np.zeros((no, 4), dtype=np.int32)
        _check(lib.hlu_schedule_records(self.h, which, r.ctypes.data_as(_P),
                                        i.ctypes.data_as(_P)))
        return r, i

    def schedule_ops(self, which):
        """(ops, waves, terms) of schedule `which` (0: factor, 1: solve) in
        schedule order: OP_DTYPE / int32 / TERM_DTYPE arrays, device
        addresses given relative to the handle's buffer."""
        no, nt = C.c_int64(), C.c_int64()
        _check(lib.hlu_schedule_ops(self.h, which, None, None, C.byref(no), None, C.byref(nt)))
        ops = np.zeros(no.value, OP_DTYPE)
        waves = np.zeros(no.value, np.int32)
        terms = np.zeros(max(1, nt.value), TERM_DTYPE)
        _check(lib.hlu_schedule_ops(self.h, which, ops.ctypes.data_as(_P),
                                    waves.ctypes.data_as(_P), C.byref(no),
                                    terms.ctypes.data_as(_P), C.byref(nt)))
        return ops, waves, terms[:nt.value]

    def schedule_graph(self, which):
        """(succ_off, succ) of schedule `which` (0: factor, 1: solve)."""
        ne = C.c_int64()
        _check(lib.hlu_schedule_graph(self.h, which, None, None, C.byref(ne)))
        off = np.zeros(self.stats()["ops_solve" if which else "ops_factor"] + 1, dtype=np.int32)
        su = np.zeros(max(1, ne.value), dtype=np.int32)
        _check(lib.hlu_schedule_graph(self.h, which, off.ctypes.data_as(_P),
                                      su.ctypes.data_as(_P), C.byref(ne)))
        return off, su[:ne.value]

    def factor_graph(self):
        """(succ_off, succ) of the factor schedule's dependency graph."""
        ne = C.c_int64()
        _check(lib.hlu_factor_graph(self.h, None, None, C.byref(ne)))
        off = np.zeros(self.stats()["ops_factor"] + 1, dtype=np.int32)
        su = np.zeros(max(1, ne.value), dtype=np.int32)
        _check(lib.hlu_factor_graph(self.h, off.ctypes.data_as(_P), su.ctypes.data_as(_P),
                                    C.byref(ne)))
        return off, su[:ne.value]

    def export_factors(self, stream=None):
        """(Lhat, U) dense in cluster order (numpy, n <= 8192)."""
        L = np.zeros((self.n, self.n), order="F")
        U = np.zeros((self.n, self.n), order="F")
        _check(lib.hlu_export_factors(self.h, L.ctypes.data_as(_P), U.ctypes.data_as(_P),
                                      _stream(stream)))
        return L, U

    def export_pivots(self, stream=None):
        p = np.zeros(self.n, dtype=np.int32)
        _check(lib.hlu_export_pivots(self.h, p.ctypes.data_as(_P), _stream(stream)))
        return p


class Batch:
    """Batched factorisation of several HLU handles by one persistent launch
    (hlu_batch_*); the workspace is a torch uint8 tensor."""

    def __init__(self, handles, device="cuda"):
        self.handles = list(handles)   # keep them alive as long as the batch
        arr = (_P * len(self.handles))(*[h.h for h in self.handles])
        b = C.c_void_p()
        _check(lib.hlu_batch_create(arr, len(self.handles), C.byref(b)))
        self.b = b
        nb = int(lib.hlu_batch_required_bytes(self.b))
        self.buf = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        ptr = (self.buf.data_ptr() + 255) & ~255
        _check(lib.hlu_batch_bind(self.b, C.c_void_p(ptr), nb))

    def __del__(self):
        b = getattr(self, "b", None)
        if b is not None and b.value:
            lib.hlu_batch_destroy(b)
            self.b = None

    def factor(self, stream=None):
        _check(lib.hlu_batch_factor(self.b, _stream(stream)))

    def sync(self, stream=None):
        _check(lib.hlu_batch_sync(self.b, _stream(stream)))

    def set_tuning(self, trunc_width, workers=0):
        """Truncation stack width (0: 64) and persistent workgroups (0: one
        per compute unit) of later launches."""
        _check(lib.hlu_batch_set_tuning(self.b, int(trunc_width), int(workers)))


def getrf_batched(a, stream=None):
    """a: CUDA FP64 tensor (count, b, b) holding column-major blocks (i.e.
    a[q] is the transpose of block q).  In place; returns (piv, info)."""
    count, b, _ = a.shape
    if not a.is_contiguous() or a.dtype != torch.float64:
        raise ValueError("a must be a contiguous float64 tensor")
    piv = torch.empty((count, b), dtype=torch.int32, device=a.device)
    info = torch.empty((count,), dtype=torch.int32, device=a.device)
    _check(lib.hlu_getrf_batched(_ptr(a), _ptr(piv), _ptr(info), b, count, _stream(stream)))
    return piv, info


def truncate_add(U, V, kc, X, Y, cap, eps, fixed_rank=0, stream=None, noalloc=False):
    """U: (cap, m) and V: (cap, n) column-major FP64 tensors (rows = columns
    of the factor); X: (kx, m), Y: (kx, n).  In place; returns the rank.
    noalloc: through hlu_truncate_add_noalloc (static device scratch)."""
    m, n = U.shape[1], V.shape[1]
    kx = X.shape[0] if X is not None else 0
    for t in (U, V) + ((X, Y) if kx else ()):
        if not t.is_contiguous() or t.dtype != torch.float64:
            raise ValueError("factors must be contiguous float64 tensors")
    rank = torch.empty((1,), dtype=torch.int32, device=U.device)
    fn = lib.hlu_truncate_add_noalloc if noalloc else lib.hlu_truncate_add
    _check(fn(_ptr(U), _ptr(V), _ptr(rank),
                                _ptr(X) if kx else None, _ptr(Y) if kx else None,
                                m, n, kc, kx, cap, eps, fixed_rank, _stream(stream)))
    return int(rank.item())
