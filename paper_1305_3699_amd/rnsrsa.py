"""Python binding of librnsrsa (ctypes), argument marshalling only.

Every computation runs in the HIP library: the binding converts Python
integers to limb arrays for set-up calls, checks tensor shapes, and passes
device pointers and the current HIP stream.  Batch buffers are torch int32
tensors on the GPU used as raw 32-bit limb storage (little-endian limbs,
one row per element).  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RNSRSA_SANITIZED=1 selects the host-sanitizer build (build.py --sanitize)
LIB_PATH = os.path.join(_HERE, "_lib", "librnsrsa_san.so" if os.environ.get("RNSRSA_SANITIZED") == "1"
                        else "librnsrsa.so")

RNS_OK = 0
STATUS_NAMES = {0: "RNS_OK", -1: "RNS_EINVAL", -2: "RNS_ERANGE", -3: "RNS_EFACTOR", -4: "RNS_ENOMEM",
                -5: "RNS_EDEVICE", -6: "RNS_EVERIFY", -7: "RNS_EBUSY", -8: "RNS_EUNSUPPORTED"}
PRIMES_HIGH = 0
PRIMES_FULL = 1
ENGINE_AUTO = 0
ENGINE_CHANNEL = 1
ENGINE_MATRIX = 2


class RnsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, message))
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("window", ctypes.c_int), ("waves", ctypes.c_int),
                ("prime_range", ctypes.c_int), ("prime_seed", ctypes.c_uint64),
                ("primes", ctypes.POINTER(ctypes.c_uint32)), ("n_primes", ctypes.c_size_t),
                ("engine", ctypes.c_int), ("group", ctypes.c_int), ("unscaled", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("waves", ctypes.c_int), ("window", ctypes.c_int),
                ("mod_limbs", ctypes.c_int), ("mod_bits", ctypes.c_int), ("engine", ctypes.c_int),
                ("group", ctypes.c_int), ("scaled", ctypes.c_int)]


class RsaOp(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("kind", ctypes.c_int), ("inp", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("count", ctypes.c_size_t)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_int), ("use_graph", ctypes.c_int), ("window", ctypes.c_int)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int), ("jobs", ctypes.c_int), ("garner_launches", ctypes.c_int),
                ("workspace_bytes", ctypes.c_size_t), ("modmuls", ctypes.c_size_t),
                ("tuning_launches", ctypes.c_int)]


class BatchClass(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("waves", ctypes.c_int), ("group", ctypes.c_int), ("exp_bits", ctypes.c_int),
                ("window", ctypes.c_int), ("window_offset", ctypes.c_int), ("jobs", ctypes.c_int),
                ("tuned", ctypes.c_int), ("launch_ms", ctypes.c_double)]


OP_ENCRYPT = 0
OP_DECRYPT = 1


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_int),
                ("max_dispatch_ops", ctypes.c_size_t), ("max_pending", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_size_t), ("rejected", ctypes.c_size_t), ("dispatches", ctypes.c_size_t),
                ("elapsed", ctypes.c_double),
                ("p50_latency", ctypes.c_double), ("p99_latency", ctypes.c_double),
                ("max_latency", ctypes.c_double), ("mean_dispatch_ops", ctypes.c_double),
                ("peak_inflight_bytes", ctypes.c_size_t), ("peak_inflight", ctypes.c_int)]


# layout of struct rsa_request
REQUEST_DTYPE = np.dtype([("key", "<i4"), ("kind", "<i4"), ("inp", "<u8"), ("out", "<u8"), ("arrival", "<f8")],
                         align=True)

_P = ctypes.c_void_p
_S = ctypes.c_size_t
_I = ctypes.c_int
_SIGNATURES = {
    "rns_last_error": ([], ctypes.c_char_p),
    "rns_abi_version": ([], _I),
    "rns_setup": ([_P, _S, _P, _P], _I),
    "rns_free": ([_P], None),
    "rns_get_info": ([_P, _P], _I),
    "rns_get_primes": ([_P, _P, _S], _I),
    "rns_modexp_batch": ([_P, _P, _P, _S, _S, _P, _S, _P], _I),
    "rns_modexp_jobs": ([_P, _S, _P], _I),
    "rsa_crt_verify": ([_P, _P, _P, _S, _P, _P], _I),
    "rns_probe_alu": ([_I, _P, _P], _I),
    "rns_mont_mul_batch": ([_P, _P, _P, _P, _S, _P], _I),
    "rsa_key_load": ([_P, _S, _P, _S, _P, _P, _P, _P, _P, _P, _S, _P, _P], _I),
    "rsa_key_free": ([_P], None),
    "rsa_key_info": ([_P, _I, _P], _I),
    "rsa_encrypt": ([_P, _P, _P, _S, _P], _I),
    "rsa_decrypt": ([_P, _P, _P, _S, _I, _P], _I),
    "rsa_decrypt_noalloc": ([_P, _P, _P, _S, _I, _P], _I),
    "rsa_crt_halves": ([_P, _P, _P, _S, _P], _I),
    "rsa_key_status": ([_P, _P, _P], _I),
    "rsa_crt_combine": ([_P, _P, _P, _S, _P], _I),
    "rsa_batch_create": ([_P, _S, _P, _P, _P], _I),
    "rsa_batch_run": ([_P, _P], _I),
    "rsa_batch_info_get": ([_P, _P], _I),
    "rsa_batch_classes": ([_P, _P, _S, _P], _I),
    "rsa_batch_free": ([_P], None),
    "rsa_server_create": ([_P, _S, _P, _P], _I),
    "rsa_server_replay": ([_P, _P, _S, _P, _P], _I),
    "rsa_server_free": ([_P], None),
    "rsa_trial_division": ([_P, _S, _I, _I, _P, _P], _I),
    "rsa_miller_rabin": ([_P, _S, _I, _P, _I, _P, _P], _I),
    "rsa_keygen": ([_P, _P, _P, _P, _S, _I, _I, ctypes.c_uint32, _P, _P, _P, _P], _I),
    "rns_plan_create": ([_P, _S, _P, _P], _I),
    "rns_plan_free": ([_P], None),
    "rns_plan_info": ([_P, _P], _I),
    "rns_plan_primes": ([_P, _P, _S], _I),
    "rns_emul_modexp": ([_P, _P, _P, _S, _S, _P, _S], _I),
    "rns_emul_mont_mul": ([_P, _P, _P, _P, _S], _I),
    "rns_emul_mfma_extension": ([_P, _I, _P, _S, _P, _P, _P], _I),
    "rns_emul_mfma_matrix": ([_P, _I, _P, _P, _P], _I),
}

_lib_handle = None


ABI_VERSION = 6           # rns_opts / rns_info layout of include/rnsrsa.h


def lib():
    """The loaded library (raises ImportError if it has not been built)."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB_PATH):
        raise ImportError("librnsrsa.so not found at %s; build it with "
                          "`python -m paper_1305_3699_amd.build`" % LIB_PATH)
    try:
        # torch ships its own HIP runtime; load it first so the library binds
        # to the same one (two runtimes in a process do not share devices)
        import torch  # noqa: F401
    except ImportError:
        pass
    h = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGNATURES.items():
        f = getattr(h, name)
        f.argtypes = args
        f.restype = res
    if h.rns_abi_version() != ABI_VERSION:
        raise ImportError("librnsrsa.so has ABI %d, this binding needs %d; rebuild it"
                          % (h.rns_abi_version(), ABI_VERSION))
    _lib_handle = h
    return h


def exported_symbols() -> list:
    return sorted(_SIGNATURES)


def _check(rc: int) -> None:
    if rc != RNS_OK:
        msg = lib().rns_last_error()
        raise RnsError(rc, msg.decode() if msg else "")


def int_to_limbs(x: int, nlimbs: int) -> np.ndarray:
    if x < 0 or x.bit_length() > 32 * nlimbs:
        raise ValueError("integer does not fit in %d limbs" % nlimbs)
    return np.frombuffer(x.to_bytes(4 * nlimbs, "little"), dtype="<u4").copy()


def nlimbs(x: int) -> int:
    return max(1, (x.bit_length() + 31) // 32)


def _host_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _make_opts(k=0, window=0, waves=0, prime_range=PRIMES_HIGH, prime_seed=0, primes=None, engine=ENGINE_AUTO,
               group=0, unscaled=False):
    o = Opts()
    o.k, o.window, o.waves, o.prime_range, o.prime_seed = k, window, waves, prime_range, prime_seed
    o.engine = engine
    o.group = group
    o.unscaled = 1 if unscaled else 0
    keep = None
    if primes is not None:
        keep = np.ascontiguousarray(primes, dtype=np.uint32)
        o.primes = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        o.n_primes = keep.size
    return o, keep


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_ptr(t, rows: int, cols: int, what: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA (HIP) tensor" % what)
    if t.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
        raise TypeError("%s must hold 32-bit limbs (torch.int32)" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.numel() != rows * cols:
        raise ValueError("%s must have %d x %d limbs, got shape %s" % (what, rows, cols, tuple(t.shape)))
    return t.data_ptr()


def _info(getter, handle, *extra) -> dict:
    inf = Info()
    _check(getter(handle, *extra, ctypes.byref(inf)))
    return {"k": inf.k, "waves": inf.waves, "window": inf.window, "mod_limbs": inf.mod_limbs,
            "mod_bits": inf.mod_bits, "engine": inf.engine, "group": inf.group, "scaled": inf.scaled}


class RnsContext:
    """A modulus N with its RNS bases and constants resident on the GPU."""

    def __init__(self, modulus: int, mod_limbs: Optional[int] = None, **opts):
        self.modulus = int(modulus)
        self.L = mod_limbs or nlimbs(self.modulus)
        mod = int_to_limbs(self.modulus, self.L)
        o, keep = _make_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().rns_setup(_host_ptr(mod), self.L, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        del keep

    def close(self):
        if getattr(self, "_h", None):
            lib().rns_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self) -> dict:
        return _info(lib().rns_get_info, self._h)

    @property
    def primes(self) -> list:
        k = self.info["k"]
        out = np.zeros(2 * k, dtype=np.uint32)
        _check(lib().rns_get_primes(self._h, _host_ptr(out), out.size))
        return [int(p) for p in out]

    def modexp(self, base, exp, out=None, stream=None):
        """out[i] = base[i]^e mod N.  base: [B, L] int32 CUDA tensor; exp: [E]
        (shared) or [B, E] (per element).  Returns out ([B, L])."""
        import torch
        B = base.shape[0] if base.dim() == 2 else 0
        if base.dim() != 2 or base.shape[1] != self.L:
            raise ValueError("base must be [B, %d]" % self.L)
        xp, E, stride = _exp_args(exp, B)
        if out is None:
            out = torch.empty_like(base)
        _check(lib().rns_modexp_batch(self._h, _dev_ptr(base, B, self.L, "base"), xp, E, stride,
                                      _dev_ptr(out, B, self.L, "out"), B, _stream_handle(stream)))
        return out

    def mont_mul(self, x, y, out=None, stream=None):
        """One RNS Montgomery product per element on [2k+1, B] residue tensors."""
        import torch
        k = self.info["k"]
        if x.dim() != 2 or x.shape[0] != 2 * k + 1 or y.shape != x.shape:
            raise ValueError("x, y must be [2k+1, B]")
        B = x.shape[1]
        if out is None:
            out = torch.empty_like(x)
        _check(lib().rns_mont_mul_batch(self._h, _dev_ptr(x, 2 * k + 1, B, "x"), _dev_ptr(y, 2 * k + 1, B, "y"),
                                        _dev_ptr(out, 2 * k + 1, B, "out"), B, _stream_handle(stream)))
        return out


def _exp_args(exp, B):
    """(device pointer, limbs, stride) of a shared [E] or per-element [B, E] exponent tensor."""
    if exp.dim() == 1:
        return _dev_ptr(exp, 1, exp.shape[0], "exp"), exp.shape[0], 0
    if exp.dim() == 2 and exp.shape[0] == B:
        return _dev_ptr(exp, B, exp.shape[1], "exp"), exp.shape[1], exp.shape[1]
    raise ValueError("exp must be [E] or [B, E]")


class RnsJob(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("base", ctypes.c_void_p), ("exp", ctypes.c_void_p),
                ("exp_limbs", ctypes.c_size_t), ("exp_stride", ctypes.c_size_t), ("out", ctypes.c_void_p),
                ("count", ctypes.c_size_t)]


def modexp_jobs(jobs, stream=None):
    """rns_modexp_jobs: jobs is a sequence of (ctx, base, exp) or (ctx, base,
    exp, out) with the tensors of RnsContext.modexp on each job's context;
    jobs of one matrix-core kernel shape share a launch.  Returns the outputs."""
    import torch
    arr = (RnsJob * len(jobs))()
    outs = []
    for i, job in enumerate(jobs):
        ctx, base, exp = job[:3]
        out = job[3] if len(job) > 3 and job[3] is not None else None
        if base.dim() != 2 or base.shape[1] != ctx.L:
            raise ValueError("job %d: base must be [B, %d]" % (i, ctx.L))
        B = base.shape[0]
        xp, E, stride = _exp_args(exp, B)
        if out is None:
            out = torch.empty_like(base)
        arr[i] = RnsJob(ctx._h, _dev_ptr(base, B, ctx.L, "base"), xp, E, stride, _dev_ptr(out, B, ctx.L, "out"), B)
        outs.append(out)
    _check(lib().rns_modexp_jobs(arr, len(jobs), _stream_handle(stream)))
    return outs


class RsaKey:
    """An RSA key (Sec. 3.3) with its RNS contexts resident on the GPU."""

    def __init__(self, n: int, e: int, d: Optional[int] = None, p: Optional[int] = None,
                 q: Optional[int] = None, dp: Optional[int] = None, dq: Optional[int] = None,
                 qinv: Optional[int] = None, n_limbs: Optional[int] = None, **opts):
        self.n, self.e = int(n), int(e)
        self.L = n_limbs or nlimbs(self.n)
        nl = int_to_limbs(self.n, self.L)
        el = int_to_limbs(self.e, nlimbs(self.e))
        dl = int_to_limbs(int(d), self.L) if d is not None else None
        crt = [p, q, dp, dq, qinv]
        if any(v is not None for v in crt) and not all(v is not None for v in crt):
            raise ValueError("p, q, dp, dq, qinv must be given together")
        half = max(nlimbs(int(p)), nlimbs(int(q))) if p is not None else 0
        arrs = [int_to_limbs(int(v), half) if v is not None else None for v in crt]
        ptr = lambda a: _host_ptr(a) if a is not None else None
        o, keep = _make_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().rsa_key_load(_host_ptr(nl), self.L, _host_ptr(el), el.size, ptr(dl), *[ptr(a) for a in arrs],
                                  half, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.has_crt = p is not None
        self._half = half
        del keep

    @classmethod
    def _adopt(cls, handle, n: int, e: int, n_limbs: int, half: int) -> "RsaKey":
        """Wrap a key the library built (rsa_keygen)."""
        k = cls.__new__(cls)
        k.n, k.e, k.L = n, e, n_limbs
        k._h = handle
        k.has_crt = True
        k._half = half
        return k

    def close(self):
        if getattr(self, "_h", None):
            lib().rsa_key_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, which: int = 0) -> dict:
        return _info(lib().rsa_key_info, self._h, which)

    def encrypt(self, m, out=None, stream=None):
        import torch
        B = m.shape[0]
        if out is None:
            out = torch.empty_like(m)
        _check(lib().rsa_encrypt(self._h, _dev_ptr(m, B, self.L, "m"), _dev_ptr(out, B, self.L, "out"), B,
                                 _stream_handle(stream)))
        return out

    def decrypt(self, c, use_crt: bool = True, out=None, stream=None):
        import torch
        B = c.shape[0]
        if out is None:
            out = torch.empty_like(c)
        _check(lib().rsa_decrypt(self._h, _dev_ptr(c, B, self.L, "c"), _dev_ptr(out, B, self.L, "out"), B,
                                 1 if use_crt else 0, _stream_handle(stream)))
        return out

    def decrypt_noalloc(self, c, out, use_crt: bool = True, stream=None):
        """rsa_decrypt_noalloc: decrypt into the caller's out ([B, n_limbs])
        with the library's fixed device scratch (no allocation anywhere)."""
        B = c.shape[0]
        _check(lib().rsa_decrypt_noalloc(self._h, _dev_ptr(c, B, self.L, "c"), _dev_ptr(out, B, self.L, "out"), B,
                                         1 if use_crt else 0, _stream_handle(stream)))
        return out


    def status(self, stream=None) -> int:
        """rsa_key_status: synchronises the stream, returns the number of
        inputs not below n seen since the last call (and clears it)."""
        nb = ctypes.c_size_t(0)
        rc = lib().rsa_key_status(self._h, ctypes.byref(nb), _stream_handle(stream))
        if rc not in (0, -2):
            _check(rc)
        return int(nb.value)

    def verify_crt(self, c, m, stream=None) -> int:
        """rsa_crt_verify: recomputes m^e mod n for every row and compares it
        with c; failing rows of m are zeroed.  Returns their number (0: all
        pass).  Synchronises the stream."""
        B = c.shape[0]
        nb = ctypes.c_size_t(0)
        rc = lib().rsa_crt_verify(self._h, _dev_ptr(c, B, self.L, "c"), _dev_ptr(m, B, self.L, "m"), B,
                                  ctypes.byref(nb), _stream_handle(stream))
        if rc not in (0, -6):
            _check(rc)
        return int(nb.value)

    @property
    def half_limbs(self) -> int:
        return self._half

    def crt_halves(self, c, out=None, stream=None):
        """[B, 2*half] tensor of (c^dp mod p | c^dq mod q) per row (one launch)."""
        import torch
        B = c.shape[0]
        if out is None:
            out = torch.empty((B, 2 * self._half), dtype=torch.int32, device=c.device)
        _check(lib().rsa_crt_halves(self._h, _dev_ptr(c, B, self.L, "c"), _dev_ptr(out, B, 2 * self._half, "mpq"),
                                    B, _stream_handle(stream)))
        return out

    def crt_combine(self, mpq, out=None, stream=None):
        """Garner recombination of crt_halves output into [B, n_limbs]."""
        import torch
        B = mpq.shape[0]
        if out is None:
            out = torch.empty((B, self.L), dtype=torch.int32, device=mpq.device)
        _check(lib().rsa_crt_combine(self._h, _dev_ptr(mpq, B, 2 * self._half, "mpq"), _dev_ptr(out, B, self.L, "m"),
                                     B, _stream_handle(stream)))
        return out


class Plan:
    """Host-side planning and the host model of the kernels (no GPU needed)."""

    def __init__(self, modulus: int, mod_limbs: Optional[int] = None, **opts):
        self.modulus = int(modulus)
        self.L = mod_limbs or nlimbs(self.modulus)
        mod = int_to_limbs(self.modulus, self.L)
        o, keep = _make_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().rns_plan_create(_host_ptr(mod), self.L, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        del keep

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().rns_plan_free(self._h)
                self._h = None
        except Exception:
            pass

    @property
    def info(self) -> dict:
        return _info(lib().rns_plan_info, self._h)

    @property
    def primes(self) -> list:
        k = self.info["k"]
        out = np.zeros(2 * k, dtype=np.uint32)
        _check(lib().rns_plan_primes(self._h, _host_ptr(out), out.size))
        return [int(p) for p in out]

    def emul_modexp(self, base: np.ndarray, exp: np.ndarray) -> np.ndarray:
        base = np.ascontiguousarray(base, dtype=np.uint32)
        exp = np.ascontiguousarray(exp, dtype=np.uint32)
        B = base.shape[0]
        if base.ndim != 2 or base.shape[1] != self.L:
            raise ValueError("base must be [B, %d]" % self.L)
        E, stride = (exp.shape[0], 0) if exp.ndim == 1 else (exp.shape[1], exp.shape[1])
        out = np.zeros((B, self.L), dtype=np.uint32)
        _check(lib().rns_emul_modexp(self._h, _host_ptr(base), _host_ptr(exp), E, stride, _host_ptr(out), B))
        return out

    def emul_mfma_extension(self, which: int, xi: np.ndarray):
        """rns_emul_mfma_extension on raw digits xi [B, k]: returns (status,
        partials [B, rows, 4] int64, value [B, rows] int64)."""
        xi = np.ascontiguousarray(xi, dtype=np.uint32)
        if xi.ndim != 2 or xi.shape[1] != self.info["k"]:
            raise ValueError("xi must be [B, %d]" % self.info["k"])
        B = xi.shape[0]
        rows = ctypes.c_size_t(0)
        _check(lib().rns_emul_mfma_extension(self._h, int(which), None, 0, ctypes.byref(rows), None, None))
        parts = np.zeros((B, rows.value, 4), dtype=np.int64)
        value = np.zeros((B, rows.value), dtype=np.int64)
        rc = lib().rns_emul_mfma_extension(self._h, int(which), _host_ptr(xi), B, ctypes.byref(rows),
                                           _host_ptr(parts), _host_ptr(value))
        if rc not in (0, -6):
            _check(rc)
        return rc, parts, value

    def emul_mfma_matrix(self, which: int) -> np.ndarray:
        """rns_emul_mfma_matrix: int8 [rows, 4, kdim] constant bytes."""
        rows, kd = ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(lib().rns_emul_mfma_matrix(self._h, int(which), ctypes.byref(rows), ctypes.byref(kd), None))
        A = np.zeros((rows.value, 4, kd.value), dtype=np.int8)
        _check(lib().rns_emul_mfma_matrix(self._h, int(which), ctypes.byref(rows), ctypes.byref(kd), _host_ptr(A)))
        return A

    def emul_mont_mul(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint32)
        y = np.ascontiguousarray(y, dtype=np.uint32)
        out = np.zeros_like(x)
        _check(lib().rns_emul_mont_mul(self._h, _host_ptr(x), _host_ptr(y), _host_ptr(out), x.shape[1]))
        return out


class RsaBatch:
    """A planned list of RSA operations over many keys (rsa_batch_*).

    ops: list of (key: RsaKey, kind: OP_ENCRYPT | OP_DECRYPT, inp, out) with
    inp/out int32 CUDA tensors of shape [count, n_limbs(key)].  The tensors and
    keys are bound at creation and must stay alive; run() enqueues all of the
    operations on the current stream."""

    def __init__(self, ops, autotune: bool = False, use_graph: bool = True, window: int = 0, stream=None):
        arr = (RsaOp * max(1, len(ops)))()
        self._keep = []
        for i, (key, kind, inp, out) in enumerate(ops):
            count = inp.shape[0]
            L = key.L
            arr[i].key = key._h
            arr[i].kind = kind
            arr[i].inp = _dev_ptr(inp, count, L, "inp") if count else None
            arr[i].out = _dev_ptr(out, count, L, "out") if count else None
            arr[i].count = count
            self._keep += [key, inp, out]
        o = BatchOpts(int(autotune), int(use_graph), int(window))
        h = ctypes.c_void_p()
        _check(lib().rsa_batch_create(arr, len(ops), ctypes.byref(o), _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(lib().rsa_batch_run(self._h, _stream_handle(stream)))

    @property
    def info(self) -> dict:
        inf = BatchInfo()
        _check(lib().rsa_batch_info_get(self._h, ctypes.byref(inf)))
        return {"launches": inf.launches, "jobs": inf.jobs, "garner_launches": inf.garner_launches,
                "workspace_bytes": inf.workspace_bytes, "modmuls": inf.modmuls,
                "tuning_launches": inf.tuning_launches}

    @property
    def classes(self) -> list:
        """rsa_batch_classes: per (kernel shape, exponent length) class, the
        base size, waves, tile, window and whether the autotuner chose them."""
        n = ctypes.c_size_t(0)
        _check(lib().rsa_batch_classes(self._h, None, 0, ctypes.byref(n)))
        arr = (BatchClass * max(1, n.value))()
        _check(lib().rsa_batch_classes(self._h, arr, n.value, ctypes.byref(n)))
        return [{"k": c.k, "waves": c.waves, "group": c.group, "exp_bits": c.exp_bits, "window": c.window,
                 "window_offset": c.window_offset, "jobs": c.jobs, "tuned": bool(c.tuned),
                 "launch_ms": round(c.launch_ms, 4)} for c in arr[:n.value]]

    def close(self):
        if getattr(self, "_h", None):
            lib().rsa_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RsaServer:
    """Request server over resident keys (rsa_server_*): continuous batching
    of RSA operations admitted by device-memory budget."""

    def __init__(self, keys, hbm_budget: int = 0, max_inflight: int = 0, max_dispatch_ops: int = 0,
                 max_pending: int = 0):
        self._keys = list(keys)
        arr = (ctypes.c_void_p * len(self._keys))(*[k._h.value for k in self._keys])
        o = ServerOpts(hbm_budget, max_inflight, max_dispatch_ops, max_pending)
        h = ctypes.c_void_p()
        _check(lib().rsa_server_create(arr, len(self._keys), ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def replay(self, key_index, kind, arrival, messages: np.ndarray, allow_refused: bool = False):
        """Open-loop replay.  key_index, kind, arrival (seconds, non-decreasing):
        length-n sequences; messages: uint32 [n, W] host array, row i holding
        request i's input in its first n_limbs(key) limbs.  Returns (outputs
        [n, W] uint32, latency [n] seconds (-1: refused by max_pending), stats
        dict).  With refused requests the call raises RnsError(RNS_EBUSY)
        unless allow_refused."""
        n = len(key_index)
        if len(kind) != n or len(arrival) != n:
            raise ValueError("key_index, kind and arrival must have the same length")
        msgs = np.ascontiguousarray(messages, dtype=np.uint32)
        if msgs.ndim != 2 or msgs.shape[0] < n:
            raise ValueError("messages must be a 2-D array with at least %d rows" % n)
        kidx = np.asarray(key_index, dtype=np.int64)
        if n and (kidx.min() < 0 or kidx.max() >= len(self._keys)):
            raise ValueError("key index out of range")
        if n:
            need = max(self._keys[int(j)].L for j in np.unique(kidx))
            if msgs.shape[1] < need:
                raise ValueError("message rows hold %d limbs; the keys used need %d" % (msgs.shape[1], need))
        outs = np.zeros_like(msgs)
        req = np.zeros(n, dtype=REQUEST_DTYPE)
        req["key"] = np.asarray(key_index, dtype=np.int32)
        req["kind"] = np.asarray(kind, dtype=np.int32)
        req["arrival"] = np.asarray(arrival, dtype=np.float64)
        stride = msgs.strides[0]
        req["inp"] = msgs.ctypes.data + stride * np.arange(n, dtype=np.uint64)
        req["out"] = outs.ctypes.data + stride * np.arange(n, dtype=np.uint64)
        lat = np.zeros(n, dtype=np.float64)
        st = ServerStats()
        rc = lib().rsa_server_replay(self._h, req.ctypes.data_as(ctypes.c_void_p), n,
                                     lat.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st))
        if not (rc == -7 and allow_refused and st.rejected):
            _check(rc)
        stats = {f: getattr(st, f) for f, _ in ServerStats._fields_}
        return outs, lat, stats

    def close(self):
        if getattr(self, "_h", None):
            lib().rsa_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trial_division(cand, n_primes: int = 10000, out=None, stream=None):
    """rsa_trial_division: one flag byte per row of ``cand`` (a [count, limbs]
    int32 device tensor of 32-bit limbs), 0 when one of the first n_primes
    primes divides the row and differs from it."""
    import torch
    count, limbs = cand.shape
    if out is None:
        out = torch.empty(count, dtype=torch.uint8, device=cand.device)
    if out.dtype != torch.uint8 or out.numel() != count or not out.is_contiguous():
        raise ValueError("out must be a contiguous uint8 tensor of %d flags" % count)
    _check(lib().rsa_trial_division(_dev_ptr(cand, count, limbs, "cand"), count, limbs, n_primes, out.data_ptr(),
                                    _stream_handle(stream)))
    return out


def miller_rabin(cand: np.ndarray, bases: np.ndarray, stream=None) -> np.ndarray:
    """rsa_miller_rabin: ``cand`` [count, limbs] and ``bases`` [count, rounds,
    limbs] host uint32 limbs; returns one verdict byte per candidate (1: every
    base passes the strong test)."""
    cand = np.ascontiguousarray(cand, dtype=np.uint32)
    bases = np.ascontiguousarray(bases, dtype=np.uint32)
    if cand.ndim != 2 or bases.ndim != 3 or bases.shape[0] != cand.shape[0] or bases.shape[2] != cand.shape[1]:
        raise ValueError("cand must be [count, limbs] and bases [count, rounds, limbs]")
    count, limbs = cand.shape
    verdict = np.zeros(count, dtype=np.uint8)
    _check(lib().rsa_miller_rabin(_host_ptr(cand), count, limbs, _host_ptr(bases), bases.shape[1],
                                  _host_ptr(verdict), _stream_handle(stream)))
    return verdict


def keygen(cand_p: np.ndarray, bases_p: np.ndarray, cand_q: np.ndarray, bases_q: np.ndarray, e: int = 65537,
           stream=None, **opts) -> "RsaKey":
    """rsa_keygen: candidate streams [count, half_limbs] and their bases
    [count, rounds, half_limbs] (host uint32 limbs); returns the loaded key,
    of which only n and e are known to the caller."""
    arrs = [np.ascontiguousarray(a, dtype=np.uint32) for a in (cand_p, bases_p, cand_q, bases_q)]
    cp, bp, cq, bq = arrs
    if cp.ndim != 2 or cp.shape != cq.shape or bp.shape != bq.shape or bp.shape[0] != cp.shape[0] \
            or bp.shape[2] != cp.shape[1]:
        raise ValueError("candidates must be [count, half_limbs] and bases [count, rounds, half_limbs]")
    count, half = cp.shape
    nl = np.zeros(2 * half, dtype=np.uint32)
    o, keep = _make_opts(**opts)
    h = ctypes.c_void_p()
    _check(lib().rsa_keygen(_host_ptr(cp), _host_ptr(bp), _host_ptr(cq), _host_ptr(bq), count, half, bp.shape[1],
                            int(e), ctypes.byref(o), _host_ptr(nl), ctypes.byref(h), _stream_handle(stream)))
    del keep
    return RsaKey._adopt(h, int.from_bytes(nl.astype("<u4").tobytes(), "little"), int(e), 2 * half, half)
