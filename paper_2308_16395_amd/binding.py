"""ctypes binding of libstucker.so (argument marshalling only).

The functions below carry the names of the C ABI in include/stucker.h and pass
plain pointers and sizes through. ``StreamingTucker`` is a convenience wrapper
that hands torch device tensors (float32, column-major slices) to those calls;
every arithmetic step runs in the library's kernels. If the library is not
built this module raises on import: there is no fallback path.

torch here carries its own copy of the HIP runtime with the same soname as the
system one the library links. Importing torch first makes the dynamic loader
bind the library to that already-loaded copy, so one runtime serves both; the
module refuses to load if two copies end up mapped (they would each claim the
GPU). The library runs on the runtime's null stream (or on a raw stream handle
passed as an int), which is also torch's default stream, so torch work queued
there is ordered before each call; ``_ready`` waits only for work on another
torch stream. Library calls that hand results to the caller return after their
device work has finished; ``st_update`` may return while the tail of its device
work still runs on the library's stream (later calls and torch's default stream
order after it).
"""

from __future__ import annotations

import ctypes as C
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstucker.so")

ST_MAX_MODES = 8
ST_OK, ST_EINVAL, ST_ENOMEM, ST_EHIP, ST_ESTATE = 0, -1, -2, -3, -4
ST_ENONFINITE, ST_EDEGENERATE, ST_ESMALL, ST_ECAPACITY, ST_ESOLVER = -5, -6, -7, -8, -9
ST_FP32, ST_BF16X3, ST_FP64 = 0, 1, 2
PRECISIONS = {"fp32": ST_FP32, "bf16x3": ST_BF16X3, "fp64": ST_FP64}
ST_HOST, ST_DEVICE = 0, 1
CORE_UPDATES = {"literal": 0, "factored": 1}

STATUS_NAMES = {
    ST_OK: "ST_OK", ST_EINVAL: "ST_EINVAL", ST_ENOMEM: "ST_ENOMEM", ST_EHIP: "ST_EHIP",
    ST_ESTATE: "ST_ESTATE", ST_ENONFINITE: "ST_ENONFINITE",
    ST_EDEGENERATE: "ST_EDEGENERATE", ST_ESMALL: "ST_ESMALL",
    ST_ECAPACITY: "ST_ECAPACITY", ST_ESOLVER: "ST_ESOLVER",
}

EXPORTED = ["st_create", "st_init", "st_update", "st_update_block", "st_ranks", "st_core",
            "st_factor", "st_sv", "st_recon_error", "st_stats", "st_reconstruct_slice",
            "st_destroy", "st_last_error", "st_ttm", "st_gram", "st_profile", "st_aux_v",
            "st_tucker_workspace", "st_tucker_fwd", "st_tucker_bwd", "st_ttm_noalloc",
            "st_symeig"]
ST_RECONSTRUCT, ST_PROJECT = 0, 1

KERNEL_GROUPS = ["ttm1", "ttm", "gram", "eig", "ttm_ext", "isvd", "svd", "rot_v", "rot_c",
                 "ud", "refine", "orth"]


class st_config(C.Structure):
    _fields_ = [
        ("nmodes", C.c_int32),
        ("dims", C.c_int64 * ST_MAX_MODES),
        ("tau", C.c_double),
        ("precision", C.c_int32),
        ("orth_tol", C.c_double),
        ("guard_rel", C.c_double),
        ("max_rank_d", C.c_int64),
        ("stream", C.c_void_p),
        ("profile", C.c_int32),
        ("core_update", C.c_int32),
    ]


class st_kernel_profile(C.Structure):
    _fields_ = [
        ("launches", C.c_int64),
        ("ms", C.c_double),
        ("flops", C.c_double),
        ("bytes", C.c_double),
    ]


class st_slice_stats(C.Structure):
    _fields_ = [
        ("ynorm", C.c_double),
        ("eps", C.c_double),
        ("e_norm", C.c_double * ST_MAX_MODES),
        ("grew", C.c_int32 * ST_MAX_MODES),
        ("q", C.c_double),
        ("isvd_ignored", C.c_int32),
        ("qr_fired", C.c_int32),
        ("guard_hits", C.c_int32),
        ("orth_check", C.c_double),
        ("delta2", C.c_double),
        ("ms_total", C.c_double),
        ("ms_modes", C.c_double),
        ("ms_isvd", C.c_double),
        ("refined_modes", C.c_int32),
        ("refined_isvd", C.c_int32),
        ("refined_gram", C.c_int32),
        ("e_norm_fast", C.c_double * ST_MAX_MODES),
        ("q_fast", C.c_double),
        ("qr_total", C.c_int64),
    ]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                      "python paper_2308_16395_amd/build.py")

try:
    import torch  # noqa: F401  (load torch's HIP runtime before the library)
except ImportError:  # pragma: no cover - the binding's tensors are torch tensors
    torch = None


def _hip_runtimes():
    with open("/proc/self/maps") as f:
        return {line.split()[-1] for line in f if "libamdhip64" in line.split()[-1]}


lib = C.CDLL(LIB_PATH)
if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are mapped in this process "
                      f"({sorted(_hip_runtimes())}); import paper_2308_16395_amd (or torch) "
                      "before anything that loads the system libamdhip64")
_h = C.c_void_p
_sig = {
    "st_create": (C.c_int, [C.POINTER(st_config), C.POINTER(_h)]),
    "st_init": (C.c_int, [_h, C.c_void_p, C.c_int64]),
    "st_update": (C.c_int, [_h, C.c_void_p]),
    "st_update_block": (C.c_int, [_h, C.c_void_p, C.c_int64]),
    "st_ranks": (C.c_int, [_h, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "st_core": (C.c_int, [_h, C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.c_int]),
    "st_aux_v": (C.c_int, [_h, C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.c_int]),
    "st_factor": (C.c_int, [_h, C.c_int, C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                            C.POINTER(C.c_int64), C.c_int]),
    "st_sv": (C.c_int, [_h, C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_int64)]),
    "st_recon_error": (C.c_int, [_h, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "st_stats": (C.c_int, [_h, C.POINTER(st_slice_stats)]),
    "st_reconstruct_slice": (C.c_int, [_h, C.c_int64, C.c_void_p]),
    "st_ttm": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.c_void_p,
                         C.c_int64, C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_void_p]),
    "st_ttm_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.c_int32,
                                 C.c_void_p, C.c_int64, C.c_void_p, C.POINTER(C.c_double),
                                 C.c_int32, C.c_void_p]),
    "st_gram": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.c_void_p,
                          C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]),
    "st_symeig": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                            C.c_void_p]),
    "st_profile": (C.c_int, [_h, C.POINTER(st_kernel_profile), C.c_int32, C.c_int32]),
    "st_tucker_workspace": (C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.c_int32, C.POINTER(C.c_int64)]),
    "st_tucker_fwd": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64), C.c_void_p, C.POINTER(C.c_void_p),
                                C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p]),
    "st_tucker_bwd": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64), C.c_void_p, C.POINTER(C.c_void_p),
                                C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.c_int32,
                                C.c_void_p, C.c_int64, C.c_void_p]),
    "st_destroy": (None, [_h]),
    "st_last_error": (C.c_char_p, [_h]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

st_create = lib.st_create
st_init = lib.st_init
st_update = lib.st_update
st_update_block = lib.st_update_block
st_ranks = lib.st_ranks
st_core = lib.st_core
st_factor = lib.st_factor
st_aux_v = lib.st_aux_v
st_sv = lib.st_sv
st_recon_error = lib.st_recon_error
st_stats = lib.st_stats
st_reconstruct_slice = lib.st_reconstruct_slice
st_ttm = lib.st_ttm
st_ttm_noalloc = lib.st_ttm_noalloc
st_gram = lib.st_gram
st_symeig = lib.st_symeig
st_profile = lib.st_profile
st_tucker_workspace = lib.st_tucker_workspace
st_tucker_fwd = lib.st_tucker_fwd
st_tucker_bwd = lib.st_tucker_bwd
st_destroy = lib.st_destroy
st_last_error = lib.st_last_error


def _ready():
    """Order torch's queued device work before a library call that reads or
    writes torch-allocated memory. The library runs on the runtime's null
    stream: work torch queued on its default stream (the same null stream) is
    already ordered before it, so only work on another torch stream is waited
    for here."""
    import torch

    cur = torch.cuda.current_stream()
    if cur.cuda_stream != 0:
        cur.synchronize()


def _stream_arg(stream):
    """NULL (the library runtime's null stream) or a raw hipStream_t of that runtime."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    raise TypeError("stream must be None or a raw hipStream_t (int) of the library's runtime")


class StError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def ttm(x, dims, mode, a, precision="fp32", norms=False, stream=None):
    """X x_mode A through st_ttm; x and a are float32 CUDA tensors (a: rows x n_mode
    row-major). Returns the output tensor (flat, column-major) and optionally
    (||X - (X x A) x A^T||^2, ||X||^2)."""
    import torch

    dims = tuple(int(n) for n in dims)
    rows = int(a.shape[0])
    out_elems = math.prod(dims) // dims[mode] * rows
    out = torch.empty(out_elems, dtype=torch.float32, device=x.device)
    cdims = (C.c_int64 * len(dims))(*dims)
    nrm = (C.c_double * 2)() if norms else None
    _ready()
    rc = st_ttm(C.c_void_p(x.data_ptr()), len(dims), cdims, int(mode), C.c_void_p(a.data_ptr()),
                rows, C.c_void_p(out.data_ptr()), nrm,
                PRECISIONS[precision], _stream_arg(stream))
    if rc != ST_OK:
        raise StError(rc, "st_ttm failed")
    if norms:
        return out, (nrm[0], nrm[1])
    return out


def gram(x, dims, mode, a=None, precision="fp64", stream=None):
    """Gram of the mode-`mode` unfolding of X (a None) or of the residual
    X - (X x A) x A^T, through st_gram. Returns a float64 numpy array."""
    import numpy as np
    import torch

    dims = tuple(int(n) for n in dims)
    n = dims[mode]
    g = np.zeros(n * n)
    cdims = (C.c_int64 * len(dims))(*dims)
    rows = 0 if a is None else int(a.shape[0])
    _ready()
    rc = st_gram(C.c_void_p(x.data_ptr()), len(dims), cdims, int(mode),
                 C.c_void_p(a.data_ptr() if a is not None else 0), rows,
                 g.ctypes.data_as(C.c_void_p), {"fp32": 0, "bf16x3": 1, "fp64": 2}[precision],
                 _stream_arg(stream))
    if rc != ST_OK:
        raise StError(rc, "st_gram failed")
    return g.reshape(n, n, order="F")


def symeig(a, k=0, stream=None):
    """Eigenvalues (ascending) of the symmetric float64 CUDA matrix a (n x n,
    lower triangle read, n <= 128) and orthonormal eigenvectors of the k
    largest (column c for the c-th largest), through st_symeig."""
    import torch

    n = int(a.shape[0])
    a = a.to(torch.float64).t().contiguous()  # column-major as the library reads it
    w = torch.empty(n, dtype=torch.float64, device=a.device)
    q = torch.empty((int(k), n), dtype=torch.float64, device=a.device)  # rows = columns of Q
    _ready()
    rc = st_symeig(C.c_void_p(a.data_ptr()), n, C.c_void_p(w.data_ptr()),
                   C.c_void_p(q.data_ptr() if k > 0 else 0), int(k), _stream_arg(stream))
    if rc != ST_OK:
        raise StError(rc, "st_symeig failed")
    return w, q.t()


class StreamingTucker:
    """Streaming Tucker decomposition on the current GPU (torch tensors in/out).

    Slices are float32 device tensors whose memory is the column-major slice
    n_1 x ... x n_{d-1} (for example a contiguous tensor of shape
    (n_{d-1}, ..., n_1), or any contiguous tensor with that many elements).
    """

    def __init__(self, dims, tau, precision="fp32", orth_tol=0.0, guard_rel=0.0,
                 max_rank_d=0, stream=None, profile=False, core_update="literal"):
        import torch

        self._torch = torch
        self.dims = tuple(int(n) for n in dims)
        if not 1 <= len(self.dims) <= ST_MAX_MODES:
            raise ValueError("1..8 slice modes")
        cfg = st_config()
        cfg.nmodes = len(self.dims)
        for k, n in enumerate(self.dims):
            cfg.dims[k] = n
        cfg.tau = float(tau)
        cfg.precision = PRECISIONS[precision]
        cfg.orth_tol = float(orth_tol)
        cfg.guard_rel = float(guard_rel)
        cfg.max_rank_d = int(max_rank_d)
        cfg.profile = 1 if profile else 0
        cfg.core_update = CORE_UPDATES[core_update]
        self.core_update = core_update
        cfg.stream = _stream_arg(stream)
        h = _h()
        rc = st_create(C.byref(cfg), C.byref(h))
        if rc != ST_OK:
            raise StError(rc, st_last_error(None).decode())
        self._h = h
        self.d = len(self.dims) + 1
        self.slice_elems = math.prod(self.dims)

    def _check(self, rc):
        if rc != ST_OK:
            raise StError(rc, st_last_error(self._h).decode())

    def _call(self, fn, *args):
        _ready()
        self._check(fn(self._h, *args))

    def _dev(self, x, count):
        t = self._torch
        if not (isinstance(x, t.Tensor) and x.is_cuda and x.dtype == t.float32
                and x.is_contiguous() and x.numel() == count):
            raise ValueError(f"expected a contiguous float32 CUDA tensor with {count} elements")
        return C.c_void_p(x.data_ptr())

    def close(self):
        if getattr(self, "_h", None):
            st_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, x0, n_init):
        self._call(st_init, self._dev(x0, self.slice_elems * n_init), int(n_init))

    def update(self, y):
        self._call(st_update, self._dev(y, self.slice_elems))

    def update_block(self, y, b):
        """b slices at once (y: b slices back to back, the block mode last)."""
        self._call(st_update_block, self._dev(y, self.slice_elems * int(b)), int(b))

    @property
    def ranks(self):
        buf = (C.c_int64 * (ST_MAX_MODES + 1))()
        nd = C.c_int64()
        self._check(st_ranks(self._h, buf, C.byref(nd)))
        return tuple(buf[k] for k in range(self.d))

    @property
    def n_slices(self):
        buf = (C.c_int64 * (ST_MAX_MODES + 1))()
        nd = C.c_int64()
        self._check(st_ranks(self._h, buf, C.byref(nd)))
        return nd.value

    def core(self):
        """Core as a float32 device tensor, column-major r_1 x ... x r_d (flat)."""
        t = self._torch
        need = C.c_int64()
        self._check(st_core(self._h, None, 0, C.byref(need), ST_DEVICE))
        out = t.empty(need.value, dtype=t.float32, device="cuda")
        self._call(st_core, C.c_void_p(out.data_ptr()), need.value, None, ST_DEVICE)
        return out

    def aux_v(self):
        """V of C = V x_d S as a float64 device tensor of shape (r_1...r_{d-1}, r_d)."""
        t = self._torch
        need = C.c_int64()
        self._check(st_aux_v(self._h, None, 0, C.byref(need), ST_DEVICE))
        out = t.empty(need.value, dtype=t.float64, device="cuda")
        self._call(st_aux_v, C.c_void_p(out.data_ptr()), need.value, None, ST_DEVICE)
        rd = self.ranks[-1]
        return out.reshape(rd, -1).T

    def factor(self, mode):
        """Factor U_mode as a float64 device tensor (column-major rows x cols)."""
        t = self._torch
        rows, cols = C.c_int64(), C.c_int64()
        self._check(st_factor(self._h, mode, None, 0, C.byref(rows), C.byref(cols), ST_DEVICE))
        out = t.empty(rows.value * cols.value, dtype=t.float64, device="cuda")
        self._call(st_factor, mode, C.c_void_p(out.data_ptr()), out.numel(), None, None,
                   ST_DEVICE)
        return out.reshape(cols.value, rows.value).T  # (rows, cols) view

    def factors(self):
        return [self.factor(k) for k in range(self.d)]

    def sv(self):
        cnt = C.c_int64()
        self._check(st_sv(self._h, None, 0, C.byref(cnt)))
        buf = (C.c_double * max(cnt.value, 1))()
        self._check(st_sv(self._h, buf, cnt.value, C.byref(cnt)))
        return [buf[i] for i in range(cnt.value)]

    def recon_error(self):
        b, nx = C.c_double(), C.c_double()
        self._check(st_recon_error(self._h, C.byref(b), C.byref(nx)))
        return b.value, nx.value

    def stats(self):
        s = st_slice_stats()
        self._check(st_stats(self._h, C.byref(s)))
        m = self.d - 1
        return dict(ynorm=s.ynorm, eps=s.eps, e_norm=[s.e_norm[k] for k in range(m)],
                    grew=[s.grew[k] for k in range(m)], q=s.q,
                    isvd_ignored=bool(s.isvd_ignored), qr_fired=bool(s.qr_fired),
                    guard_hits=s.guard_hits, orth_check=s.orth_check, delta2=s.delta2,
                    ms_total=s.ms_total, ms_modes=s.ms_modes, ms_isvd=s.ms_isvd,
                    refined_modes=bool(s.refined_modes), refined_isvd=bool(s.refined_isvd),
                    refined_gram=s.refined_gram,
                    e_norm_fast=[s.e_norm_fast[k] for k in range(m)], q_fast=s.q_fast,
                    qr_total=s.qr_total)

    def profile(self, reset=False):
        """Per kernel group: launches, device ms, algorithmic flops and bytes."""
        buf = (st_kernel_profile * len(KERNEL_GROUPS))()
        self._check(st_profile(self._h, buf, len(KERNEL_GROUPS), 1 if reset else 0))
        return {name: dict(launches=buf[i].launches, ms=buf[i].ms, flops=buf[i].flops,
                           bytes=buf[i].bytes) for i, name in enumerate(KERNEL_GROUPS)}

    def reconstruct_slice(self, t_index, out=None):
        t = self._torch
        if out is None:
            out = t.empty(self.slice_elems, dtype=t.float32, device="cuda")
        self._call(st_reconstruct_slice, int(t_index), self._dev(out, self.slice_elems))
        return out
