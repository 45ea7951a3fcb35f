"""The oracle: a plain, slow CPU evaluation of BBP-type bit extraction of pi.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. The GPU library never calls it, and
it shares no code with the GPU library.

The arithmetic lives in ``pio.c`` (portable C with its own big integers);
this module builds it on demand with gcc and marshals arguments with ctypes.
Every value it returns is a plain Python int: a P-bit sum ``S`` in
``[0, 2**P)`` (not left-aligned), a term ``t``, or a bit string of pi.

What each call computes, with the passage of Sze (2010) it follows:

* ``term``     -- one truncated term ``floor(2^P * frac(2^E/M))``, the A_k of
  eq (3.3) for E >= 0 and the B_k for E < 0.
* ``sum_slice`` -- the signed sum of the terms of one series over a k range,
  mod 2^P (one summand of eq (3.1)/(3.2)).
* ``extract``  -- every series of Bellard's formula (1.2) or the BBP formula
  (1.1, in the form of (3.1)) at 1-based bit position n, plus the
  certification of section 3.1 adapted to truncated terms.
* ``certify``  -- that certification on its own: the guard-window test of
  section 3.1 for a given sum S and error bound B.
* ``machin_bits`` -- pi's fraction bits from Machin's formula, a textbook
  method independent of every BBP-type formula.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

BBP = 0
BELLARD = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pio.c")
_LIB = os.path.join(_HERE, "libpio.so")
_lock = threading.Lock()
_lib = None


def compile_source(src: str, lib: str) -> str:
    """gcc -O2 of one copy of the oracle's C into a shared library."""
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-pthread",
                           "-o", tmp, src])
    os.replace(tmp, lib)
    return lib


def build(force: bool = False) -> str:
    """Compile pio.c into libpio.so next to it (gcc, -O2, pthreads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


def _bind(lib):
    """Argument and return types of the oracle's C functions on a loaded library."""
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64 = ctypes.c_uint64
    lib.pio_pow2mod.restype = u64
    lib.pio_pow2mod.argtypes = [u64, u64]
    lib.pio_term.argtypes = [ctypes.c_int, ctypes.c_int, u64, u64, ctypes.c_uint32, u32p]
    lib.pio_sum_slice.argtypes = [ctypes.c_int, ctypes.c_int, u64, u64, u64,
                                  ctypes.c_uint32, u32p, ctypes.POINTER(u64), ctypes.c_int]
    lib.pio_extract.argtypes = [ctypes.c_int, u64, ctypes.c_uint32, ctypes.c_uint32, u32p,
                                ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_int32),
                                ctypes.c_int]
    lib.pio_machin.argtypes = [ctypes.c_uint32, u32p]
    lib.pio_certify.argtypes = [u32p, ctypes.c_uint32, ctypes.c_uint32, u64]
    lib.pio_series_table.argtypes = [ctypes.c_int, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            _lib = _bind(ctypes.CDLL(build()))
    return _lib


def _words(bits: int):
    return (ctypes.c_uint32 * max(1, (bits + 31) // 32))()


def _to_int(words) -> int:
    v = 0
    for i, w in enumerate(words):
        v |= int(w) << (32 * i)
    return v


class _Series(ctypes.Structure):
    _fields_ = [("sign", ctypes.c_int32), ("c", ctypes.c_int32),
                ("a", ctypes.c_uint64), ("b", ctypes.c_uint64)]


class Oracle:
    """The oracle's calls on one compiled copy of its C. The module-level
    functions use the copy built from pio.c in this directory; a test can load
    another build, for instance one with a mistake planted on purpose to show
    that the pins catch it, as ``Oracle(path_to_shared_library)``."""

    def __init__(self, lib_path: str | None = None):
        self._path = lib_path
        self._own = None

    @property
    def lib(self):
        if self._path is None:
            return _load()
        if self._own is None:
            self._own = _bind(ctypes.CDLL(self._path))
        return self._own

    def series_table(self, formula: int):
        """[(sign, c, a, b), ...], step, alt for the formula."""
        buf = (_Series * 7)()
        step, alt = ctypes.c_int32(), ctypes.c_int32()
        J = self.lib.pio_series_table(formula, ctypes.byref(buf), ctypes.byref(step),
                                      ctypes.byref(alt))
        if J < 0:
            raise ValueError("unknown formula %r" % formula)
        return [(s.sign, s.c, s.a, s.b) for s in buf[:J]], step.value, alt.value

    def pow2mod(self, e: int, m: int) -> int:
        return int(self.lib.pio_pow2mod(e, m))

    def term(self, formula: int, j: int, d: int, k: int, P: int) -> int:
        """floor(2^P * frac(2^E/M)) for series j at shift d and index k."""
        out = _words(P)
        if self.lib.pio_term(formula, j, d, k, P, out) != 0:
            raise ValueError("bad term arguments")
        return _to_int(out)

    def sum_slice(self, formula: int, j: int, d: int, k0: int, k1: int, P: int,
                  nthreads: int = 1):
        """(S, nterms): signed sum of series j over k in [k0, k1) mod 2^P."""
        out = _words(P)
        cnt = ctypes.c_uint64()
        if self.lib.pio_sum_slice(formula, j, d, k0, k1, P, out, ctypes.byref(cnt),
                                  nthreads) != 0:
            raise ValueError("bad slice arguments")
        return _to_int(out), int(cnt.value)

    def extract(self, formula: int, n: int, w: int, P: int, nthreads: int = 1):
        """(S, N, certified) at 1-based position n; the result bits are S >> (P - w)."""
        out = _words(P)
        N = ctypes.c_uint64()
        cert = ctypes.c_int32()
        if self.lib.pio_extract(formula, n, w, P, out, ctypes.byref(N), ctypes.byref(cert),
                                nthreads) != 0:
            raise ValueError("bad extract arguments")
        return _to_int(out), int(N.value), bool(cert.value)

    def certify(self, S: int, P: int, w: int, B: int) -> bool:
        """The guard-window test of ``extract`` on its own: True when every
        number within B units of 2^-P of S/2^P (exclusive, modulo 1) has the
        same top w bits as S (section 3.1's caveat about runs of 0s and 1s)."""
        if not (1 <= w <= P) or not (0 <= S < 2 ** P) or not (0 <= B < 2 ** 64):
            raise ValueError("bad certify arguments")
        nw = (P + 31) // 32
        buf = (ctypes.c_uint32 * nw)(*[(S >> (32 * i)) & 0xFFFFFFFF for i in range(nw)])
        return bool(self.lib.pio_certify(buf, P, w, B))

    def machin_bits(self, nbits: int) -> int:
        """floor(frac(pi) * 2^nbits): bits 1..nbits of pi after the radix point."""
        out = _words(nbits)
        if self.lib.pio_machin(nbits, out) != 0:
            raise RuntimeError("Machin guard bits could not certify the result")
        return _to_int(out)


_default = Oracle()
series_table = _default.series_table
pow2mod = _default.pow2mod
term = _default.term
sum_slice = _default.sum_slice
extract = _default.extract
certify = _default.certify
machin_bits = _default.machin_bits
