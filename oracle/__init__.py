"""CPU oracle for RSA modular exponentiation -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  The GPU library never imports, links or runs it, and it
shares no code with the GPU library (its own limb packing included).

Two layers:

* ``bn_oracle.c`` (loaded through ctypes): plain positional bignums --
  schoolbook multiplication, Knuth's Algorithm D remainder, left-to-right
  binary square-and-multiply -- computing b^e mod N, the RSA operations of
  the paper's Sec. 3.3 and a Garner CRT decryption for CPU timing.
* ``rns_ref``: plain Python-integer definitions of the intermediate RNS
  quantities of the RNS Montgomery product (Sec. 3.1), for step-level tests.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bn_oracle.c")
# RNSRSA_SANITIZED=1 loads the AddressSanitizer + UndefinedBehaviorSanitizer
# builds (build(sanitize=True), clang with the shared sanitizer runtime)
_SANITIZED = os.environ.get("RNSRSA_SANITIZED") == "1"
_SUFFIX = "_san" if _SANITIZED else ""
_LIBS = {32: os.path.join(_HERE, "liboracle%s.so" % _SUFFIX), 8: os.path.join(_HERE, "liboracle8%s.so" % _SUFFIX)}
_loaded = {}


def build(force: bool = False, sanitize: bool = None) -> None:
    """Compile the oracle with gcc (32-bit limbs, plus the 8-bit test build);
    sanitize: with clang, -fsanitize=address,undefined (the *_san.so files)."""
    sanitize = _SANITIZED if sanitize is None else sanitize
    for bits in (32, 8):
        path = os.path.join(_HERE, "liboracle%s%s.so" % ("" if bits == 32 else "8", "_san" if sanitize else ""))
        if not force and os.path.exists(path) and os.path.getmtime(path) >= os.path.getmtime(_SRC):
            continue
        tmp = path + ".tmp"
        if sanitize:
            cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-Wall",
                   "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                   "-shared-libsan", "-DORACLE_LIMB_BITS=%d" % bits, "-o", tmp, _SRC]
        else:
            cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                   "-DORACLE_LIMB_BITS=%d" % bits, "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)


def _lib(bits: int = 32):
    if bits in _loaded:
        return _loaded[bits]
    path = _LIBS[bits]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(path)
    pre = "oracle_" if bits == 32 else "oracle8_"
    P = ctypes.c_void_p
    S = ctypes.c_size_t
    for name, args in {
        "divmod": [P, S, P, S, P, P],
        "mul": [P, S, P, S, P],
        "modexp_batch": [P, S, P, S, S, P, S, P, S, ctypes.c_int],
        "rsa_crt_batch": [P, S, P, P, P, P, P, S, P, S, ctypes.c_int],
    }.items():
        f = getattr(lib, pre + name)
        f.argtypes = args
        f.restype = ctypes.c_int
    for name in ("addback_count", "qhat_fix_count"):
        f = getattr(lib, pre + name)
        f.argtypes = []
        f.restype = ctypes.c_longlong
    getattr(lib, pre + "reset_counters").argtypes = []
    getattr(lib, pre + "reset_counters").restype = None
    _loaded[bits] = (lib, pre)
    return _loaded[bits]


def _dtype(bits):
    return np.uint32 if bits == 32 else np.uint8


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def int_to_limbs(x: int, nlimbs: int, bits: int = 32) -> np.ndarray:
    """Little-endian limbs of x (the oracle's own packing)."""
    if x < 0 or x.bit_length() > bits * nlimbs:
        raise ValueError("value does not fit")
    mask = (1 << bits) - 1
    return np.array([(x >> (bits * i)) & mask for i in range(nlimbs)], dtype=_dtype(bits))


def limbs_to_int(a, bits: int = 32) -> int:
    """Integer value of a little-endian limb vector."""
    v = 0
    for i, limb in enumerate(np.asarray(a).reshape(-1).tolist()):
        v |= int(limb) << (bits * i)
    return v


def rows_to_ints(a: np.ndarray, bits: int = 32) -> list:
    return [limbs_to_int(row, bits) for row in np.asarray(a)]


def divmod_limbs(u: np.ndarray, v: np.ndarray, bits: int = 32):
    """(q, r) = divmod(u, v) by Algorithm D on limb vectors."""
    lib, pre = _lib(bits)
    u = np.ascontiguousarray(u, dtype=_dtype(bits))
    v = np.ascontiguousarray(v, dtype=_dtype(bits))
    q = np.zeros(len(u), dtype=_dtype(bits))
    r = np.zeros(len(v), dtype=_dtype(bits))
    rc = getattr(lib, pre + "divmod")(_ptr(u), len(u), _ptr(v), len(v), _ptr(q), _ptr(r))
    if rc:
        raise ValueError("oracle divmod failed (zero divisor?)")
    return q, r


def mul_limbs(a: np.ndarray, b: np.ndarray, bits: int = 32) -> np.ndarray:
    lib, pre = _lib(bits)
    a = np.ascontiguousarray(a, dtype=_dtype(bits))
    b = np.ascontiguousarray(b, dtype=_dtype(bits))
    w = np.zeros(len(a) + len(b), dtype=_dtype(bits))
    rc = getattr(lib, pre + "mul")(_ptr(a), len(a), _ptr(b), len(b), _ptr(w))
    if rc:
        raise ValueError("oracle mul failed")
    return w


def addback_count(bits: int = 32) -> int:
    lib, pre = _lib(bits)
    return int(getattr(lib, pre + "addback_count")())


def qhat_fix_count(bits: int = 32) -> int:
    lib, pre = _lib(bits)
    return int(getattr(lib, pre + "qhat_fix_count")())


def reset_counters(bits: int = 32) -> None:
    lib, pre = _lib(bits)
    getattr(lib, pre + "reset_counters")()


def modexp_batch(base: np.ndarray, exp: np.ndarray, mod: np.ndarray,
                 nthreads: int = 0, bits: int = 32) -> np.ndarray:
    """out[i] = base[i] ^ exp(i) mod N.

    base: [B, lb] limbs; exp: [le] (shared) or [B, le] (per element);
    mod: [lm] limbs.  Returns [B, lm] limbs, canonical in [0, N).
    """
    lib, pre = _lib(bits)
    dt = _dtype(bits)
    base = np.ascontiguousarray(np.atleast_2d(base), dtype=dt)
    exp = np.ascontiguousarray(exp, dtype=dt)
    mod = np.ascontiguousarray(mod, dtype=dt).reshape(-1)
    B, lb = base.shape
    if exp.ndim == 1:
        le, stride = exp.shape[0], 0
    else:
        if exp.shape[0] != B:
            raise ValueError("per-element exponents need one row per base")
        le, stride = exp.shape[1], exp.shape[1]
    out = np.zeros((B, len(mod)), dtype=dt)
    if B == 0:
        return out
    rc = getattr(lib, pre + "modexp_batch")(_ptr(base), lb, _ptr(exp), le, stride,
                                             _ptr(mod), len(mod), _ptr(out), B, int(nthreads))
    if rc:
        raise ValueError("oracle modexp failed (zero modulus?)")
    return out


def modexp_int(b: int, e: int, n: int) -> int:
    """b^e mod n for Python ints through the C oracle."""
    ln = max(1, (n.bit_length() + 31) // 32)
    lb = max(1, (b.bit_length() + 31) // 32)
    le = max(1, (e.bit_length() + 31) // 32)
    out = modexp_batch(int_to_limbs(b, lb)[None, :], int_to_limbs(e, le), int_to_limbs(n, ln))
    return limbs_to_int(out[0])


def rsa_crt_batch(c: np.ndarray, p: int, q: int, dp: int, dq: int, qinv: int,
                  nthreads: int = 0) -> np.ndarray:
    """Garner CRT decryption of c [B, ln] limbs; returns [B, ln] limbs."""
    lib, pre = _lib(32)
    c = np.ascontiguousarray(np.atleast_2d(c), dtype=np.uint32)
    B, ln = c.shape
    lh = max(limbs_needed(p), limbs_needed(q))
    if ln < 2 * lh:
        raise ValueError("ciphertext rows need at least 2x the prime limb count")
    arrs = [int_to_limbs(v, lh) for v in (p, q, dp, dq, qinv)]
    out = np.zeros((B, ln), dtype=np.uint32)
    if B == 0:
        return out
    rc = getattr(lib, pre + "rsa_crt_batch")(_ptr(c), ln, *[_ptr(a) for a in arrs], lh,
                                              _ptr(out), B, int(nthreads))
    if rc:
        raise ValueError("oracle CRT decryption failed")
    return out


def limbs_needed(x: int) -> int:
    return max(1, (x.bit_length() + 31) // 32)
