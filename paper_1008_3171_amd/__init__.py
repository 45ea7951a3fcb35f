"""Python binding of the MI355X bit-extraction library for pi (libpibbp.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/pibbp.h``. PyTorch provides
device memory and streams. If the library is not built, or no GPU is present,
the calls raise; there is no CPU fallback.

Limb layout (as in the C ABI): a P-bit sum S comes back as
L = ceil(P/64) little-endian 64-bit limbs holding S * 2^(64L - P), stored in a
torch.int64 tensor on the device (bit pattern of uint64).
"""
from __future__ import annotations

import ctypes
import os

BBP = 0
BELLARD = 1
PI_OK = 0
PI_UNCERTAIN = 1
PI_EINVAL = -1
PI_ENOMEM = -2
PI_EDEVICE = -3
PI_EUNSUPPORTED = -4
PI_ESCRATCH = -5
MAX_P = 1088

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpibbp.so")
_lib = None


class PiError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = _lib.pi_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s failed: %s (code %d)" % (what, msg, code))
        self.code = code


class pi_query(ctypes.Structure):
    _fields_ = [("formula", ctypes.c_int32), ("nbits", ctypes.c_uint32),
                ("P", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("n", ctypes.c_uint64), ("out_offset", ctypes.c_uint64)]


def term_id(formula: int, j: int) -> int:
    """PI_TERM(formula, j)."""
    return formula * 16 + j


def load():
    """Load libpibbp.so (built by ``python -m paper_1008_3171_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpibbp.so is not built; run python -m paper_1008_3171_amd.build")
        # torch ships its own HIP runtime under the same soname. Loaded first,
        # it is the one the library binds to, so the process keeps a single
        # runtime that owns torch's memory and streams; loaded second, it
        # would come in as a second runtime beside the system one.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        lib.pi_extract.argtypes = [i32, u64, u32, vp, vp]
        lib.pi_extract_ex.argtypes = [i32, u64, u32, u32, vp, vp, vp]
        lib.pi_sum_slice.argtypes = [i32, u64, u64, u64, u32, vp, vp]
        lib.pi_extract_batch.argtypes = [vp, i32, vp, vp, vp, ctypes.c_size_t, vp]
        lib.pi_workspace_size.argtypes = [vp, i32]
        lib.pi_workspace_size.restype = ctypes.c_size_t
        lib.pi_head_terms.argtypes = [i32, u64]
        lib.pi_head_terms.restype = u64
        lib.pi_plan_head.argtypes = [i32, u32, u64, u64, u64, u32, vp, i32, vp]
        lib.pi_plan_head.restype = i32
        lib.pi_strerror.argtypes = [i32]
        lib.pi_strerror.restype = ctypes.c_char_p
        lib.pi_shutdown.argtypes = []
        for f in (lib.pi_extract, lib.pi_extract_ex, lib.pi_sum_slice, lib.pi_extract_batch):
            f.restype = i32
        lib.pi_set_tuning.argtypes = [i32, u32, u32]
        lib.pi_set_tuning.restype = i32
        lib.pi_get_tuning.argtypes = [i32, ctypes.POINTER(u32), ctypes.POINTER(u32)]
        lib.pi_get_tuning.restype = i32
        lib.pi_set_arith.argtypes = [i32]
        lib.pi_set_arith.restype = i32
        lib.pi_get_arith.argtypes = []
        lib.pi_get_arith.restype = i32
        _lib = lib
        _apply_tuning_cache()
    return _lib


def tuning_cache_path() -> str:
    """Where the autotuner keeps its choices: tuning.json in this package, as
    measured on an MI355X and kept with the sources (PIBBP_TUNING names
    another file; an empty PIBBP_TUNING keeps the library's defaults)."""
    env = os.environ.get("PIBBP_TUNING")
    return env if env is not None else os.path.join(_HERE, "tuning.json")


def _apply_tuning_cache():
    import json
    path = tuning_cache_path()
    if not path:
        return
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        return
    for limbs_s, t in cache.get("classes", {}).items():
        _lib.pi_set_tuning(int(limbs_s), int(t["wg_per_cu"]), int(t["run_cap"]))
    t = cache.get("fused")
    if t:
        _lib.pi_set_tuning(-1, int(t["wg_per_cu"]), int(t["run_cap"]))


TUNE_FUSED = -1   # pi_set_tuning's key for the fused launch of 1 to 6 limbs


def set_tuning(limbs: int, wg_per_cu: int, run_cap: int):
    rc = load().pi_set_tuning(limbs, wg_per_cu, run_cap)
    if rc != 0:
        raise PiError(rc, "pi_set_tuning")


def get_tuning(limbs: int):
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    rc = load().pi_get_tuning(limbs, ctypes.byref(a), ctypes.byref(b))
    if rc != 0:
        raise PiError(rc, "pi_get_tuning")
    return a.value, b.value


ARITH_FAST = 0
ARITH_INTEGER = 1


def set_arith(mode: int):
    """pi_set_arith: ARITH_FAST (exact binary64 where cheaper) or ARITH_INTEGER
    (integer Montgomery arithmetic everywhere); results are bit-identical."""
    rc = load().pi_set_arith(mode)
    if rc != 0:
        raise PiError(rc, "pi_set_arith")


def get_arith() -> int:
    return int(load().pi_get_arith())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the HIP library needs a ROCm device")
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def limbs(P: int) -> int:
    return (P + 63) // 64


def _check(t, name: str, dtype, need: int):
    """A caller's buffer must be a contiguous device tensor of `dtype` with at
    least `need` elements: the kernels write through its raw pointer, so a
    host tensor or a short buffer would be written out of bounds."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU (got device %s)" % (name, t.device))
    if t.dtype != dtype:
        raise ValueError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < need:
        raise ValueError("%s holds %d elements; the call writes %d" % (name, t.numel(), need))


def _check_limbs(out, P: int, name: str = "out"):
    _check(out, name, _torch().int64, limbs(P))


def _check_status(status, count: int = 1):
    _check(status, "status", _torch().int32, 4 * count)


def head_terms(formula: int, n: int) -> int:
    return int(load().pi_head_terms(formula, n))


class Segment(ctypes.Structure):
    """pi_segment."""
    _fields_ = [("j", ctypes.c_uint32), ("cls", ctypes.c_uint32), ("run", ctypes.c_uint32),
                ("pre", ctypes.c_uint32), ("kb", ctypes.c_uint64), ("ke", ctypes.c_uint64),
                ("nchunks", ctypes.c_uint64)]


def plan_head(formula: int, n: int, P: int, k0: int = 0, k1: int = 2 ** 64 - 1,
              series_mask: int = 0x7F) -> list:
    """pi_plan_head: the head segments a query or slice would launch, as
    dicts (host only)."""
    lib = load()
    count = ctypes.c_int(0)
    rc = lib.pi_plan_head(formula, series_mask, n, k0, k1, P, None, 0, ctypes.byref(count))
    if rc != PI_OK and count.value == 0:
        raise PiError(rc, "pi_plan_head")
    segs = (Segment * max(1, count.value))()
    rc = lib.pi_plan_head(formula, series_mask, n, k0, k1, P, segs, count.value,
                          ctypes.byref(count))
    if rc != PI_OK:
        raise PiError(rc, "pi_plan_head")
    return [{f: getattr(segs[i], f) for f, _ in Segment._fields_} for i in range(count.value)]


def extract(formula: int, n: int, nbits: int, P: int | None = None, out=None, status=None,
            stream=None):
    """pi_extract_ex: returns (out limbs tensor, status tensor [4] int32).

    P defaults to nbits + 64. Asynchronous on `stream` (default: current)."""
    torch = _torch()
    lib = load()
    P = nbits + 64 if P is None else P
    if out is None:
        out = torch.zeros(limbs(P), dtype=torch.int64, device="cuda")
    if status is None:
        status = torch.zeros(4, dtype=torch.int32, device="cuda")
    _check_limbs(out, P)
    _check_status(status)
    rc = lib.pi_extract_ex(formula, n, nbits, P, ctypes.c_void_p(out.data_ptr()),
                           ctypes.c_void_p(status.data_ptr()), _stream(stream))
    if rc != 0:
        raise PiError(rc, "pi_extract_ex")
    return out, status


def extract_noalloc(formula: int, n: int, nbits: int, P: int, out, status, stream=None):
    """pi_extract_noalloc: pi_extract_ex on the library's static device
    scratch (nothing allocated, nothing waited for). out and status are the
    caller's; calls that overlap on one device race (see include/pibbp.h)."""
    lib = load()
    lib.pi_extract_noalloc.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]
    lib.pi_extract_noalloc.restype = ctypes.c_int
    _check_limbs(out, P)
    _check_status(status)
    rc = lib.pi_extract_noalloc(formula, n, nbits, P, ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(status.data_ptr()), _stream(stream))
    if rc != 0:
        raise PiError(rc, "pi_extract_noalloc")
    return out, status


def extract_default(formula: int, n: int, nbits: int, out=None, stream=None):
    """pi_extract (P = nbits + 64, no status)."""
    torch = _torch()
    lib = load()
    if out is None:
        out = torch.zeros(limbs(nbits + 64), dtype=torch.int64, device="cuda")
    _check_limbs(out, nbits + 64)
    rc = lib.pi_extract(formula, n, nbits, ctypes.c_void_p(out.data_ptr()), _stream(stream))
    if rc != 0:
        raise PiError(rc, "pi_extract")
    return out


def sum_slice(term: int, n: int, k0: int, k1: int, P: int, out=None, stream=None):
    """pi_sum_slice: the signed sum of one series over k in [k0, k1) mod 2^P."""
    torch = _torch()
    lib = load()
    if out is None:
        out = torch.zeros(limbs(P), dtype=torch.int64, device="cuda")
    _check_limbs(out, P)
    rc = lib.pi_sum_slice(term, n, k0, k1, P, ctypes.c_void_p(out.data_ptr()), _stream(stream))
    if rc != 0:
        raise PiError(rc, "pi_sum_slice")
    return out


def make_queries(specs):
    """specs: iterable of (formula, n, nbits, P). Returns (ctypes array, total limbs)."""
    specs = list(specs)
    arr = (pi_query * max(1, len(specs)))()
    off = 0
    for i, (formula, n, nbits, P) in enumerate(specs):
        arr[i].formula, arr[i].n, arr[i].nbits, arr[i].P = formula, n, nbits, P
        arr[i].reserved = 0
        arr[i].out_offset = off
        off += limbs(P)
    return arr, off


def workspace_size(qarr, count: int) -> int:
    return int(load().pi_workspace_size(ctypes.cast(qarr, ctypes.c_void_p), count))


def extract_batch(qarr, count: int, out, status=None, workspace=None, stream=None):
    """pi_extract_batch over a ctypes pi_query array (see make_queries).

    status: an int32 tensor of 4*count, None to allocate one, or False to pass
    NULL (no certification written)."""
    torch = _torch()
    lib = load()
    if status is None:
        status = torch.zeros(4 * max(1, count), dtype=torch.int32, device="cuda")
    if count < 0 or count > len(qarr):
        raise ValueError("count %d outside the query array's %d entries" % (count, len(qarr)))
    need = max([qarr[i].out_offset + limbs(qarr[i].P) for i in range(count)], default=0)
    _check(out, "out", torch.int64, need)
    if status is not False:
        _check_status(status, count)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        _check(workspace, "workspace", workspace.dtype, 0)
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    st_ptr = None if status is False else status.data_ptr()
    rc = lib.pi_extract_batch(ctypes.cast(qarr, ctypes.c_void_p), count,
                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st_ptr),
                              ctypes.c_void_p(ws_ptr), ws_bytes, _stream(stream))
    if rc != 0:
        raise PiError(rc, "pi_extract_batch")
    return out, status


def to_int(limb_tensor, P: int | None = None) -> int:
    """Limbs (int64 tensor, any device) -> the P-bit integer S (not left-aligned)."""
    vals = [int(v) & 0xFFFFFFFFFFFFFFFF for v in limb_tensor.cpu().tolist()]
    x = 0
    for i, v in enumerate(vals):
        x |= v << (64 * i)
    if P is not None:
        x >>= 64 * len(vals) - P
    return x


def status_of(status_tensor, i: int = 0):
    """(code, nterms) of the i-th pi_status in an int32 tensor."""
    s = [int(v) & 0xFFFFFFFF for v in status_tensor[4 * i:4 * i + 4].cpu().tolist()]
    return s[0] if s[0] < 2 ** 31 else s[0] - 2 ** 32, s[2] | (s[3] << 32)


class pi_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("code", ctypes.c_int32), ("P", ctypes.c_uint32),
                ("nterms", ctypes.c_uint64), ("limbs", ctypes.c_uint64 * 17)]


PI_BUSY = 2


class Server:
    """pi_server_*: continuous batching on one device and stream."""

    def __init__(self, max_active: int = 1024, step_terms: int = 1 << 30, stream=None):
        torch = _torch()
        lib = load()
        vp = ctypes.c_void_p
        lib.pi_server_create.argtypes = [ctypes.c_uint32, ctypes.c_uint64, vp, ctypes.POINTER(vp)]
        lib.pi_server_submit.argtypes = [vp, vp, ctypes.c_uint64]
        lib.pi_server_step.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
        lib.pi_server_poll.argtypes = [vp, vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        lib.pi_server_active.argtypes = [vp]
        lib.pi_server_active.restype = ctypes.c_uint32
        lib.pi_server_capacity.argtypes = [vp]
        lib.pi_server_capacity.restype = ctypes.c_uint32
        lib.pi_server_destroy.argtypes = [vp]
        lib.pi_server_set_memory_limit.argtypes = [vp, ctypes.c_size_t]
        lib.pi_server_set_memory_limit.restype = ctypes.c_int
        lib.pi_server_set_pipeline.argtypes = [vp, ctypes.c_int]
        lib.pi_server_set_pipeline.restype = ctypes.c_int
        for f in (lib.pi_server_create, lib.pi_server_submit, lib.pi_server_step,
                  lib.pi_server_poll):
            f.restype = ctypes.c_int
        self._lib = lib
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = lib.pi_server_create(max_active, step_terms, ctypes.c_void_p(self._stream.cuda_stream),
                                  ctypes.byref(h))
        if rc != 0:
            raise PiError(rc, "pi_server_create")
        self._h = h
        self._q = pi_query()
        self._buf = (pi_result * 4096)()

    def set_memory_limit(self, nbytes: int):
        """pi_server_set_memory_limit: the device bytes its slots may take."""
        rc = self._lib.pi_server_set_memory_limit(self._h, nbytes)
        if rc != 0:
            raise PiError(rc, "pi_server_set_memory_limit")

    def set_pipeline(self, depth: int):
        """pi_server_set_pipeline: 1 (default) leaves a step running when step()
        returns; 0 waits for it."""
        rc = self._lib.pi_server_set_pipeline(self._h, depth)
        if rc != 0:
            raise PiError(rc, "pi_server_set_pipeline")

    def submit(self, formula: int, n: int, nbits: int, P: int, tag: int) -> bool:
        """Admit a query; False when every slot is busy."""
        q = self._q
        q.formula, q.n, q.nbits, q.P, q.reserved, q.out_offset = formula, n, nbits, P, 0, 0
        rc = self._lib.pi_server_submit(self._h, ctypes.byref(q), tag)
        if rc == PI_BUSY:
            return False
        if rc != 0:
            raise PiError(rc, "pi_server_submit")
        return True

    def cancel(self, tag: int) -> bool:
        """pi_server_cancel: withdraw an active query; False when none is
        active under the tag (finishing, delivered or unknown)."""
        f = self._lib.pi_server_cancel
        f.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        f.restype = ctypes.c_int
        rc = f(self._h, tag)
        if rc == PI_EINVAL:
            return False
        if rc != 0:
            raise PiError(rc, "pi_server_cancel")
        return True

    def step(self) -> int:
        """Enqueue one step and wait for the previous one (or for this one,
        unpipelined); the number of results delivered (poll returns them)."""
        fin = ctypes.c_uint32()
        rc = self._lib.pi_server_step(self._h, ctypes.byref(fin))
        if rc != 0:
            raise PiError(rc, "pi_server_step")
        return fin.value

    def poll(self):
        """[(tag, S, code, nterms)] of the queries finished since the last poll."""
        out = []
        while True:
            cnt = ctypes.c_uint32()
            rc = self._lib.pi_server_poll(self._h, self._buf, len(self._buf), ctypes.byref(cnt))
            if rc != 0:
                raise PiError(rc, "pi_server_poll")
            for r in self._buf[:cnt.value]:
                L = limbs(r.P)
                S = 0
                for i in range(L):
                    S |= int(r.limbs[i]) << (64 * i)
                out.append((int(r.tag), S >> (64 * L - r.P), int(r.code), int(r.nterms)))
            if cnt.value < len(self._buf):
                return out

    def active(self) -> int:
        return int(self._lib.pi_server_active(self._h))

    def capacity(self) -> int:
        return int(self._lib.pi_server_capacity(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pi_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sum_slice_ex(term: int, n: int, k0: int, k1: int, P: int, out=None, status=None, stream=None):
    """pi_sum_slice_ex: (limbs, status); status holds N, the indices summed."""
    torch = _torch()
    lib = load()
    lib.pi_sum_slice_ex.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]
    lib.pi_sum_slice_ex.restype = ctypes.c_int
    if out is None:
        out = torch.zeros(limbs(P), dtype=torch.int64, device="cuda")
    if status is None:
        status = torch.zeros(4, dtype=torch.int32, device="cuda")
    _check_limbs(out, P)
    _check_status(status)
    rc = lib.pi_sum_slice_ex(term, n, k0, k1, P, ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(status.data_ptr()), _stream(stream))
    if rc != 0:
        raise PiError(rc, "pi_sum_slice_ex")
    return out, status


def combine(parts, count: int, P: int, nbits: int, nseries: int, nterms: int, out=None,
            status=None, stream=None):
    """pi_combine over a device int64 tensor of count x limbs(P) partial sums."""
    torch = _torch()
    lib = load()
    lib.pi_combine.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p]
    lib.pi_combine.restype = ctypes.c_int
    if out is None:
        out = torch.zeros(limbs(P), dtype=torch.int64, device="cuda")
    if status is None:
        status = torch.zeros(4, dtype=torch.int32, device="cuda")
    if count < 0:
        raise ValueError("count must be >= 0")
    _check(parts, "parts", torch.int64, count * limbs(P))
    _check_limbs(out, P)
    _check_status(status)
    rc = lib.pi_combine(ctypes.c_void_p(parts.data_ptr()), count, P, nbits, nseries, nterms,
                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(status.data_ptr()),
                        _stream(stream))
    if rc != 0:
        raise PiError(rc, "pi_combine")
    return out, status


class BatchPlan:
    """pi_batch_*: a batch planned once and launched many times (capturable)."""

    def __init__(self, qarr, count: int, out, status=None):
        lib = load()
        vp = ctypes.c_void_p
        lib.pi_batch_create.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.POINTER(vp)]
        lib.pi_batch_create.restype = ctypes.c_int
        lib.pi_batch_launch.argtypes = [vp, vp]
        lib.pi_batch_launch.restype = ctypes.c_int
        lib.pi_batch_destroy.argtypes = [vp]
        self._lib = lib
        if count <= 0 or count > len(qarr):
            raise ValueError("count %d outside the query array's %d entries" % (count, len(qarr)))
        torch = _torch()
        need = max(qarr[i].out_offset + limbs(qarr[i].P) for i in range(count))
        _check(out, "out", torch.int64, need)
        if status is not None:
            _check_status(status, count)
        self.out, self.status = out, status
        h = vp()
        rc = lib.pi_batch_create(ctypes.cast(qarr, vp), count, vp(out.data_ptr()),
                                 vp(status.data_ptr() if status is not None else None),
                                 ctypes.byref(h))
        if rc != 0:
            raise PiError(rc, "pi_batch_create")
        self._h = h

    def launch(self, stream=None):
        rc = self._lib.pi_batch_launch(self._h, _stream(stream))
        if rc != 0:
            raise PiError(rc, "pi_batch_launch")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pi_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
