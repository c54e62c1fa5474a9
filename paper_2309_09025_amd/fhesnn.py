"""ctypes binding of libfhesnn (include/fhesnn.h): argument marshalling only.

Every entry point keeps the C name without the ``fs_`` prefix.  Device
buffers are torch tensors on a HIP device (int32 storage holding the uint32
torus words); streams are torch streams.  Nothing here computes on
ciphertexts: each call goes straight to the library, which must be built
(``python -m paper_2309_09025_amd.build``); importing without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfhesnn.so")

FS_OK, FS_EINVAL, FS_ENOMEM, FS_EDEVICE, FS_EPARAM, FS_EBUDGET, FS_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
FS_PARAMS_VERSION = 1
FS_KEY_EXACT, FS_KEY_ONE_LIMB = 0, 1


class FsError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


class CParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("N", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("l", ctypes.c_uint32), ("bg_bit", ctypes.c_uint32), ("ks_t", ctypes.c_uint32),
                ("ks_base_bit", ctypes.c_uint32), ("p", ctypes.c_uint32),
                ("sigma_lwe", ctypes.c_double), ("sigma_bsk", ctypes.c_double),
                ("sigma_ksk", ctypes.c_double), ("version", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class CLif(ctypes.Structure):
    _fields_ = [("v_th", ctypes.c_int32), ("tau", ctypes.c_uint32)]


class CLifRange(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("h", ctypes.c_void_p), ("spike2_out", ctypes.c_void_p),
                ("v_out", ctypes.c_void_p), ("count", ctypes.c_size_t)]


_vp = ctypes.c_void_p
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_sz = ctypes.c_size_t
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32
_int = ctypes.c_int
_PP = ctypes.POINTER(CParams)
_LP = ctypes.POINTER(CLif)

# name -> (restype, argtypes); every symbol declared in include/fhesnn.h
SIGNATURES = {
    "fs_last_error": (ctypes.c_char_p, []),
    "fs_params_default": (_int, [_int, _PP]),
    "fs_keygen": (_int, [_PP, _u64, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "fs_encrypt": (_int, [_vp, _i32p, _sz, _u64, _u64, _u32p]),
    "fs_encrypt_z": (_int, [_vp, _i32p, _sz, _u64, _u64, _u32p]),
    "fs_decrypt": (_int, [_vp, _u32p, _sz, _u32, _i32p]),
    "fs_secret_export": (_int, [_vp, _i32p, _i32p]),
    "fs_ctx_set_split": (_int, [_vp, _u32, _sz, ctypes.POINTER(_sz)]),
    "fs_ctx_set_rows": (_int, [_vp, _u32, _sz, ctypes.POINTER(_sz)]),
    "fs_ctx_set_paired": (_int, [_vp, _u32, _sz, ctypes.POINTER(_sz)]),
    "fs_ctx_scratch_bytes": (_int, [_vp, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "fs_evk_export": (_int, [_vp, _u32p, _u32p]),
    "fs_evk_params": (_int, [_vp, _PP]),
    "fs_secret_free": (None, [_vp]),
    "fs_evk_free": (None, [_vp]),
    "fs_test_poly": (_int, [_u32, _u32, _i32p, _u32p]),
    "fs_test_poly_mspace": (_int, [_u32, _u32, _u32, _i32p, _u32p]),
    "fs_test_poly_two": (_int, [_u32, _u32, _i32p, _i32p, _u32p]),
    "fs_lif_luts": (_int, [_LP, _u32, _i32p, _i32p]),
    "fs_lif_range_check": (_int, [_LP, _u32, _i32p, _sz, _sz, _i32, _i32, _i64p]),
    "fs_ctx_create": (_int, [_int, ctypes.POINTER(_vp)]),
    "fs_ctx_destroy": (_int, [_vp]),
    "fs_ctx_reserve": (_int, [_vp, _u32, _sz]),
    "fs_ctx_set_budget": (_int, [_vp, _sz]),
    "fs_ctx_admit": (_int, [_vp, _sz]),
    "fs_ctx_release": (_int, [_vp, _sz]),
    "fs_ctx_admission": (_int, [_vp, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "fs_br_variants": (_int, [_u32]),
    "fs_ctx_set_br_variant": (_int, [_vp, _u32, _int]),
    "fs_evk_upload": (_int, [_vp, _vp, ctypes.POINTER(_vp)]),
    "fs_evk_upload_form": (_int, [_vp, _vp, _int, ctypes.POINTER(_vp)]),
    "fs_devkey_form": (_int, [_vp]),
    "fs_devkey_params": (_int, [_vp, _PP]),
    "fs_devkey_bytes": (_sz, [_vp]),
    "fs_devkey_free": (None, [_vp]),
    "fs_lwe_linear": (_int, [_vp, _vp, _sz, _sz, _u32, _vp, _vp, _vp, _vp]),
    "fs_lwe_conv2d": (_int, [_vp, _vp, _u32, _u32, _u32, _u32, _u32, _u32, _u32, _u32,
                             _vp, _vp, _vp, _vp]),
    "fs_lwe_add": (_int, [_vp, _vp, _vp, _sz, _vp, _vp]),
    "fs_lwe_add_plain": (_int, [_vp, _u32, _vp, _vp, _sz, _u32, _vp, _vp]),
    "fs_pbs": (_int, [_vp, _vp, _i32p, _vp, _sz, _vp, _int, _vp]),
    "fs_pbs_lif": (_int, [_vp, _vp, _LP, _vp, _sz, _vp, _vp, _vp]),
    "fs_pbs_mspace": (_int, [_vp, _vp, _i32p, _u32, _u32, _vp, _sz, _vp, _int, _vp]),
    "fs_pbs_lif_noalloc": (_int, [_vp, _vp, _LP, _vp, _sz, _vp, _vp, _vp]),
    "fs_pbs_lif_many_lut": (_int, [_vp, _vp, _LP, _vp, _sz, _vp, _vp, _vp]),
    "fs_pbs_lif_ks_first": (_int, [_vp, _vp, _LP, _vp, _sz, _vp, _vp, _vp]),
    "fs_pbs_lif_ranges": (_int, [_vp, _LP, ctypes.POINTER(CLifRange), _sz, _vp]),
    "fs_pbs_lif_ranges_many_lut": (_int, [_vp, _LP, ctypes.POINTER(CLifRange), _sz, _vp]),
    "fs_keyswitch": (_int, [_vp, _vp, _vp, _sz, _vp, _vp]),
    "fs_ntt_polymul": (_int, [_vp, _u32, _u32, _i32, _vp, _vp, _vp, _vp]),
    "fs_probe_valu": (_int, [_int, _u32, _u32, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double)]),
    "fs_probe_hbm": (_int, [_int, _sz, ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def lib():
    """Load libfhesnn.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname as the one
        # the library links: loaded first, it is the one both share (loaded
        # after the library, torch would run on the library's copy and find
        # no device)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2309_09025_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(fn: str, rc: int):
    if rc != FS_OK:
        raise FsError(fn, rc, lib().fs_last_error().decode())
    return rc


def _np_u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(_u32p)


def _np_i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _dptr(t):
    """Device pointer of a contiguous int32 device tensor (None -> NULL).
    The library cannot see buffer sizes, so every caller checks shapes
    first; this checks placement and element type."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if t.dtype != torch.int32:
        raise ValueError(f"expected an int32 tensor, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _rows(fn: str, name: str, t, rows: int, width: int):
    """Raise unless t is a 2-D [rows][width] tensor."""
    if t is None or t.dim() != 2 or t.shape[0] != rows or t.shape[1] != width:
        got = None if t is None else tuple(t.shape)
        raise ValueError(f"{fn}: {name} must be [{rows}][{width}], got {got}")


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ params

def params_default(shape: int = 0) -> CParams:
    p = CParams()
    _check("fs_params_default", lib().fs_params_default(shape, ctypes.byref(p)))
    return p


# ------------------------------------------------------------------ client

class Secret:
    def __init__(self, handle, params: CParams):
        self.h = ctypes.c_void_p(handle)
        self.params = params

    def __del__(self):
        if _lib is not None and self.h:
            _lib.fs_secret_free(self.h)
            self.h = ctypes.c_void_p()

    def export(self):
        P = self.params
        s = np.zeros(P.n, np.int32)
        z = np.zeros(P.N, np.int32)
        _check("fs_secret_export", lib().fs_secret_export(self.h, s.ctypes.data_as(_i32p),
                                                          z.ctypes.data_as(_i32p)))
        return s, z


class EvalKey:
    def __init__(self, handle, params: CParams):
        self.h = ctypes.c_void_p(handle)
        self.params = params

    def __del__(self):
        if _lib is not None and self.h:
            _lib.fs_evk_free(self.h)
            self.h = ctypes.c_void_p()

    def export(self, bsk: bool = True, ksk: bool = True):
        P = self.params
        base = 1 << P.ks_base_bit
        b = np.zeros((P.n, 2 * P.l, 2, P.N), np.uint32) if bsk else None
        k = np.zeros((P.N, P.ks_t, base - 1, P.n + 1), np.uint32) if ksk else None
        _check("fs_evk_export", lib().fs_evk_export(
            self.h, b.ctypes.data_as(_u32p) if b is not None else None,
            k.ctypes.data_as(_u32p) if k is not None else None))
        return b, k


def keygen(params: CParams, seed: int):
    sk, evk = ctypes.c_void_p(), ctypes.c_void_p()
    _check("fs_keygen", lib().fs_keygen(ctypes.byref(params), seed, ctypes.byref(sk),
                                        ctypes.byref(evk)))
    return Secret(sk.value, params), EvalKey(evk.value, params)


def encrypt(sk: Secret, m, seed: int, first_index: int = 0) -> np.ndarray:
    m, mp = _np_i32(np.atleast_1d(m))
    ct = np.zeros((m.size, sk.params.n + 1), np.uint32)
    _check("fs_encrypt", lib().fs_encrypt(sk.h, mp, m.size, seed, first_index,
                                          ct.ctypes.data_as(_u32p)))
    return ct


def encrypt_z(sk: Secret, m, seed: int, first_index: int = 0) -> np.ndarray:
    """Encryption under the extracted key z: [count][N+1]."""
    m, mp = _np_i32(np.atleast_1d(m))
    ct = np.zeros((m.size, sk.params.N + 1), np.uint32)
    _check("fs_encrypt_z", lib().fs_encrypt_z(sk.h, mp, m.size, seed, first_index,
                                              ct.ctypes.data_as(_u32p)))
    return ct


def decrypt(sk: Secret, ct) -> np.ndarray:
    ct, cp = _np_u32(np.atleast_2d(ct))
    m = np.zeros(ct.shape[0], np.int32)
    _check("fs_decrypt", lib().fs_decrypt(sk.h, cp, ct.shape[0], ct.shape[1],
                                          m.ctypes.data_as(_i32p)))
    return m


def test_poly(N: int, p: int, f) -> np.ndarray:
    f, fp = _np_i32(f)
    v = np.zeros(N, np.uint32)
    _check("fs_test_poly", lib().fs_test_poly(N, p, fp, v.ctypes.data_as(_u32p)))
    return v


def test_poly_mspace(N: int, p_in: int, p_out: int, f) -> np.ndarray:
    f, fp = _np_i32(f)
    if f.size != p_in:
        raise ValueError(f"test_poly_mspace: f must have p_in = {p_in} entries")
    v = np.zeros(N, np.uint32)
    _check("fs_test_poly_mspace",
           lib().fs_test_poly_mspace(N, p_in, p_out, fp, v.ctypes.data_as(_u32p)))
    return v


def test_poly_two(N: int, p: int, f0, f1) -> np.ndarray:
    f0, p0 = _np_i32(f0)
    f1, p1 = _np_i32(f1)
    if f0.size != p or f1.size != p:
        raise ValueError(f"test_poly_two: both functions need p = {p} entries")
    v = np.zeros(N, np.uint32)
    _check("fs_test_poly_two", lib().fs_test_poly_two(N, p, p0, p1, v.ctypes.data_as(_u32p)))
    return v


def lif_luts(v_th: int, tau: int, p: int):
    fire = np.zeros(p, np.int32)
    reset = np.zeros(p, np.int32)
    lif = CLif(v_th, tau)
    _check("fs_lif_luts", lib().fs_lif_luts(ctypes.byref(lif), p, fire.ctypes.data_as(_i32p),
                                            reset.ctypes.data_as(_i32p)))
    return fire, reset


def lif_range_check(v_th: int, tau: int, p: int, W, x_lo: int, x_hi: int):
    """(M, holds) for the range condition of Theorem 4.1."""
    W, wp = _np_i32(np.atleast_2d(W))
    m = ctypes.c_int64()
    rc = lib().fs_lif_range_check(ctypes.byref(CLif(v_th, tau)), p, wp, W.shape[0], W.shape[1],
                                  x_lo, x_hi, ctypes.byref(m))
    if rc not in (0, 1):
        _check("fs_lif_range_check", rc)
    return m.value, rc == 0


# ------------------------------------------------------------------ server

class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check("fs_ctx_create", lib().fs_ctx_create(device, ctypes.byref(h)))
        self.h = h
        self.device = device

    def __del__(self):
        if _lib is not None and getattr(self, "h", None):
            _lib.fs_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def reserve(self, N: int, max_jobs: int):
        _check("fs_ctx_reserve", lib().fs_ctx_reserve(self.h, N, max_jobs))

    def _set_limit(self, fn: str, N: int, max_jobs: int) -> int:
        prev = ctypes.c_size_t()
        _check(fn, getattr(lib(), fn)(self.h, N, max_jobs, ctypes.byref(prev)))
        return prev.value

    def set_split(self, N: int, max_jobs: int) -> int:
        """Batches of at most max_jobs jobs at ring degree N use two thread
        groups per job; returns the previous threshold."""
        return self._set_limit("fs_ctx_set_split", N, max_jobs)

    def set_rows(self, N: int, max_jobs: int) -> int:
        """Batches of at most max_jobs jobs at ring degree N use one thread
        group per digit row (lowest latency); returns the previous threshold."""
        return self._set_limit("fs_ctx_set_rows", N, max_jobs)

    def set_paired(self, N: int, max_jobs: int) -> int:
        """Batches of at most max_jobs jobs at ring degree N (after the row
        threshold) use two thread groups per job and two jobs per workgroup
        (N = 1024 only); returns the previous threshold."""
        return self._set_limit("fs_ctx_set_paired", N, max_jobs)

    def set_budget(self, nbytes: int):
        """Device bytes admissible for requests (0: no budget)."""
        _check("fs_ctx_set_budget", lib().fs_ctx_set_budget(self.h, int(nbytes)))

    def admit(self, nbytes: int) -> bool:
        """Admit a request of nbytes: True, or False when it does not fit the
        budget or the device's free memory (FS_EBUDGET)."""
        rc = lib().fs_ctx_admit(self.h, int(nbytes))
        if rc == FS_EBUDGET:
            return False
        _check("fs_ctx_admit", rc)
        return True

    def release(self, nbytes: int):
        _check("fs_ctx_release", lib().fs_ctx_release(self.h, int(nbytes)))

    def admission(self):
        """(budget, admitted) device bytes."""
        b, a = ctypes.c_size_t(), ctypes.c_size_t()
        _check("fs_ctx_admission", lib().fs_ctx_admission(self.h, ctypes.byref(b), ctypes.byref(a)))
        return b.value, a.value

    def scratch_bytes(self):
        """(live, retired) device bytes of the context's scratch."""
        live, retired = ctypes.c_size_t(), ctypes.c_size_t()
        _check("fs_ctx_scratch_bytes", lib().fs_ctx_scratch_bytes(self.h, ctypes.byref(live),
                                                                  ctypes.byref(retired)))
        return live.value, retired.value

    def groups(self, mode: str, N=None):
        """Context manager forcing the thread groups per job at ring degree N
        (None: both 1024 and 2048): "one", "two", "paired" (two groups, two
        jobs per workgroup; N = 1024) or "rows" (restores the thresholds on
        exit)."""
        import contextlib

        @contextlib.contextmanager
        def cm():
            big = 1 << 40
            rows, paired, split = {"one": (0, 0, 0), "two": (0, 0, big), "paired": (0, big, 0),
                                   "rows": (big, 0, 0)}[mode]
            saved = []
            for n in ((1024, 2048) if N is None else (N,)):
                saved.append((n, self.set_rows(n, rows), self.set_paired(n, paired),
                              self.set_split(n, split)))
            try:
                yield self
            finally:
                for n, pr, pp, ps in saved:
                    self.set_rows(n, pr)
                    self.set_paired(n, pp)
                    self.set_split(n, ps)
        return cm()

    def set_br_variant(self, N: int, variant: int):
        _check("fs_ctx_set_br_variant", lib().fs_ctx_set_br_variant(self.h, N, variant))


def br_variants(N: int) -> int:
    return int(lib().fs_br_variants(N))


class DevKey:
    def __init__(self, ctx: Context, evk: EvalKey, form: int = 0):
        h = ctypes.c_void_p()
        _check("fs_evk_upload_form", lib().fs_evk_upload_form(ctx.h, evk.h, form, ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self.params = CParams()
        _check("fs_devkey_params", lib().fs_devkey_params(h, ctypes.byref(self.params)))
        self.form = _check_form(lib().fs_devkey_form(h))

    @property
    def nbytes(self) -> int:
        return int(lib().fs_devkey_bytes(self.h))

    def __del__(self):
        if _lib is not None and getattr(self, "h", None):
            _lib.fs_devkey_free(self.h)
            self.h = ctypes.c_void_p()


def _check_form(rc: int) -> int:
    if rc < 0:
        _check("fs_devkey_form", rc)
    return rc


def evk_upload(ctx: Context, evk: EvalKey, form: int = 0) -> DevKey:
    """form: FS_KEY_EXACT (0, exact for every key) or FS_KEY_ONE_LIMB (1,
    whole 32-bit key coefficients at N = 2048; see include/fhesnn.h)."""
    return DevKey(ctx, evk, form)


def lwe_linear(ctx: Context, W, x, y, add=None, stream=None):
    """y = add + W x on ciphertext rows: W [O][I], x [I][dim], y and add
    [O][dim]."""
    if W.dim() != 2 or x.dim() != 2:
        raise ValueError("lwe_linear: W must be [O][I] and x [I][dim]")
    O, I = W.shape
    dim = x.shape[1]
    _rows("lwe_linear", "x", x, I, dim)
    _rows("lwe_linear", "y", y, O, dim)
    if add is not None:
        _rows("lwe_linear", "add", add, O, dim)
    _check("fs_lwe_linear", lib().fs_lwe_linear(ctx.h, _dptr(W), O, I, dim, _dptr(x),
                                                _dptr(add), _dptr(y), _stream(stream)))
    return y


def conv_out_size(H: int, Wd: int, K: int, stride: int, pad: int):
    """(Ho, Wo) of a K x K convolution with this stride and zero padding."""
    return (H + 2 * pad - K) // stride + 1, (Wd + 2 * pad - K) // stride + 1


def lwe_conv2d(ctx: Context, W, x, y, Ci, H, Wd, stride, pad, add=None, stream=None):
    """Convolution WeightSum: W [Co][Ci][K][K], x [Ci*H*Wd][dim], y and add
    [Co*Ho*Wo][dim]."""
    if W.dim() != 4 or W.shape[1] != Ci or W.shape[2] != W.shape[3]:
        raise ValueError(f"lwe_conv2d: W must be [Co][{Ci}][K][K]")
    Co, _, K, _ = W.shape
    if x.dim() != 2:
        raise ValueError("lwe_conv2d: x must be [Ci*H*Wd][dim]")
    dim = x.shape[1]
    _rows("lwe_conv2d", "x", x, Ci * H * Wd, dim)
    if stride > 0 and H + 2 * pad >= K and Wd + 2 * pad >= K:  # else the library rejects it
        Ho, Wo = conv_out_size(H, Wd, K, stride, pad)
        _rows("lwe_conv2d", "y", y, Co * Ho * Wo, dim)
        if add is not None:
            _rows("lwe_conv2d", "add", add, Co * Ho * Wo, dim)
    _check("fs_lwe_conv2d", lib().fs_lwe_conv2d(ctx.h, _dptr(W), Ci, H, Wd, Co, K, stride, pad,
                                                dim, _dptr(x), _dptr(add), _dptr(y),
                                                _stream(stream)))
    return y


def lwe_add(ctx: Context, a, b, y, stream=None):
    """y = a + b word by word; a, b, y of one shape."""
    if tuple(b.shape) != tuple(a.shape) or tuple(y.shape) != tuple(a.shape):
        raise ValueError(f"lwe_add: a, b and y must have one shape, got {tuple(a.shape)}, "
                         f"{tuple(b.shape)}, {tuple(y.shape)}")
    _check("fs_lwe_add", lib().fs_lwe_add(ctx.h, _dptr(a), _dptr(b), a.numel(), _dptr(y),
                                          _stream(stream)))
    return y


def lwe_add_plain(ctx: Context, p: int, x, c, y, stream=None):
    """y = x + Delta c on the body word of each row; x, y [rows][dim],
    c: device int32 [rows]."""
    if x.dim() != 2:
        raise ValueError("lwe_add_plain: x must be [rows][dim]")
    _rows("lwe_add_plain", "y", y, x.shape[0], x.shape[1])
    if c.dim() != 1 or c.numel() != x.shape[0]:
        raise ValueError(f"lwe_add_plain: c must be [{x.shape[0]}]")
    _check("fs_lwe_add_plain", lib().fs_lwe_add_plain(ctx.h, p, _dptr(x), _dptr(c), x.shape[0],
                                                      x.shape[1], _dptr(y), _stream(stream)))
    return y


def _pbs_shapes(fn, dk, x, out, keyswitch):
    P = dk.params
    wo = P.n + 1 if keyswitch else P.N + 1
    if x.dim() != 2 or x.shape[1] != P.n + 1:
        raise ValueError(f"{fn}: inputs must be [B][{P.n + 1}]")
    if out.dim() != 2 or out.shape[0] != x.shape[0] or out.shape[1] != wo:
        raise ValueError(f"{fn}: outputs must be [{x.shape[0]}][{wo}]")


def pbs(ctx: Context, dk: DevKey, lut, x, out, keyswitch: bool = True, stream=None):
    lut, lp = _np_i32(lut)
    if lut.size != dk.params.p:
        raise ValueError(f"pbs: the program function needs p = {dk.params.p} entries")
    _pbs_shapes("pbs", dk, x, out, keyswitch)
    _check("fs_pbs", lib().fs_pbs(ctx.h, dk.h, lp, _dptr(x), x.shape[0], _dptr(out),
                                  1 if keyswitch else 0, _stream(stream)))
    return out


def pbs_mspace(ctx: Context, dk: DevKey, lut, p_in: int, p_out: int, x, out,
               keyswitch: bool = True, stream=None):
    """Bootstrapping f: Z_p_in -> Z_p_out (outputs encoded with 2^32 / p_out)."""
    lut, lp = _np_i32(lut)
    if lut.size != p_in:
        raise ValueError(f"pbs_mspace: the program function needs p_in = {p_in} entries")
    _pbs_shapes("pbs_mspace", dk, x, out, keyswitch)
    _check("fs_pbs_mspace", lib().fs_pbs_mspace(ctx.h, dk.h, lp, p_in, p_out, _dptr(x),
                                                x.shape[0], _dptr(out), 1 if keyswitch else 0,
                                                _stream(stream)))
    return out


def pbs_lif(ctx: Context, dk: DevKey, v_th: int, tau: int, h, spike2_out, v_out, stream=None):
    """One LIF activation: h, spike2_out, v_out are [B][n+1]."""
    w = dk.params.n + 1
    if h.dim() != 2:
        raise ValueError(f"pbs_lif: h must be [B][{w}]")
    for name, t in (("h", h), ("spike2_out", spike2_out), ("v_out", v_out)):
        _rows("pbs_lif", name, t, h.shape[0], w)
    lif = CLif(v_th, tau)
    _check("fs_pbs_lif", lib().fs_pbs_lif(ctx.h, dk.h, ctypes.byref(lif), _dptr(h), h.shape[0],
                                          _dptr(spike2_out), _dptr(v_out), _stream(stream)))


def pbs_lif_noalloc(ctx: Context, dk: DevKey, v_th: int, tau: int, h, spike2_out, v_out,
                    stream=None):
    """pbs_lif through the entry point that allocates nothing (static
    device scratch; calls overlapping on one GPU race): h, spike2_out,
    v_out are [B][n+1]."""
    w = dk.params.n + 1
    if h.dim() != 2:
        raise ValueError(f"pbs_lif_noalloc: h must be [B][{w}]")
    for name, t in (("h", h), ("spike2_out", spike2_out), ("v_out", v_out)):
        _rows("pbs_lif_noalloc", name, t, h.shape[0], w)
    lif = CLif(v_th, tau)
    _check("fs_pbs_lif_noalloc",
           lib().fs_pbs_lif_noalloc(ctx.h, dk.h, ctypes.byref(lif), _dptr(h), h.shape[0],
                                    _dptr(spike2_out), _dptr(v_out), _stream(stream)))


def pbs_lif_many_lut(ctx: Context, dk: DevKey, v_th: int, tau: int, h, spike2_out, v_out,
                     stream=None):
    """Fire and Reset from one blind rotation per neuron: h, spike2_out,
    v_out are [B][n+1]."""
    w = dk.params.n + 1
    for name, t in (("h", h), ("spike2_out", spike2_out), ("v_out", v_out)):
        if t.dim() != 2 or t.shape[1] != w or t.shape[0] != h.shape[0]:
            raise ValueError(f"pbs_lif_many_lut: {name} must be [{h.shape[0]}][{w}]")
    lif = CLif(v_th, tau)
    _check("fs_pbs_lif_many_lut",
           lib().fs_pbs_lif_many_lut(ctx.h, dk.h, ctypes.byref(lif), _dptr(h), h.shape[0],
                                     _dptr(spike2_out), _dptr(v_out), _stream(stream)))


def pbs_lif_ks_first(ctx: Context, dk: DevKey, v_th: int, tau: int, h, spike2_out, v_out,
                     stream=None):
    """Key switch first, then Fire and Reset: h, spike2_out, v_out are
    [B][N+1] under z."""
    w = dk.params.N + 1
    for name, t in (("h", h), ("spike2_out", spike2_out), ("v_out", v_out)):
        if t.dim() != 2 or t.shape[1] != w or t.shape[0] != h.shape[0]:
            raise ValueError(f"pbs_lif_ks_first: {name} must be [{h.shape[0]}][{w}]")
    lif = CLif(v_th, tau)
    _check("fs_pbs_lif_ks_first",
           lib().fs_pbs_lif_ks_first(ctx.h, dk.h, ctypes.byref(lif), _dptr(h), h.shape[0],
                                     _dptr(spike2_out), _dptr(v_out), _stream(stream)))


def pbs_lif_ranges(ctx: Context, v_th: int, tau: int, ranges, stream=None,
                   many_lut: bool = False):
    """ranges: iterable of (DevKey, h, spike2_out, v_out) device tensors, each
    [count][n+1]; many_lut: the one-rotation activation."""
    rs = []
    for dk, h, s2, v in ranges:
        w = dk.params.n + 1
        for t in (h, s2, v):
            if t.dim() != 2 or t.shape[1] != w or t.shape[0] != h.shape[0]:
                raise ValueError(f"pbs_lif_ranges: buffers of a range must be [{h.shape[0]}][{w}]")
        rs.append(CLifRange(dk.h, _dptr(h).value, _dptr(s2).value, _dptr(v).value, h.shape[0]))
    arr = (CLifRange * max(1, len(rs)))(*rs)
    fn = "fs_pbs_lif_ranges_many_lut" if many_lut else "fs_pbs_lif_ranges"
    _check(fn, getattr(lib(), fn)(ctx.h, ctypes.byref(CLif(v_th, tau)), arr, len(rs),
                                  _stream(stream)))


def keyswitch(ctx: Context, dk: DevKey, x, out, stream=None):
    """x [B][N+1] under z -> out [B][n+1] under s."""
    P = dk.params
    if x.dim() != 2:
        raise ValueError(f"keyswitch: x must be [B][{P.N + 1}]")
    _rows("keyswitch", "x", x, x.shape[0], P.N + 1)
    _rows("keyswitch", "out", out, x.shape[0], P.n + 1)
    _check("fs_keyswitch", lib().fs_keyswitch(ctx.h, dk.h, _dptr(x), x.shape[0], _dptr(out),
                                              _stream(stream)))
    return out


def ntt_polymul(ctx: Context, N: int, dmax: int, d, b, out, stream=None):
    """out = sum_r d_r b_r mod X^N + 1: d, b [R][N], out [N]."""
    if d.dim() != 2:
        raise ValueError(f"ntt_polymul: d must be [R][{N}]")
    R = d.shape[0]
    _rows("ntt_polymul", "d", d, R, N)
    _rows("ntt_polymul", "b", b, R, N)
    if out.dim() != 1 or out.shape[0] != N:
        raise ValueError(f"ntt_polymul: out must be [{N}]")
    _check("fs_ntt_polymul", lib().fs_ntt_polymul(ctx.h, N, R, dmax, _dptr(d), _dptr(b),
                                                  _dptr(out), _stream(stream)))
    return out


# ------------------------------------------------------------------ torch helpers

def probe_valu(device: int, waves_per_simd: int, kind: int):
    """(lane-instructions/s, ms) of the binary64 VALU probe: kind 0 modular
    butterflies, 1 modular multiply-accumulates, 2 bare FMAs, at exactly
    waves_per_simd waves on every SIMD."""
    rate, ms = ctypes.c_double(), ctypes.c_double()
    _check("fs_probe_valu", lib().fs_probe_valu(device, waves_per_simd, kind,
                                                ctypes.byref(rate), ctypes.byref(ms)))
    return rate.value, ms.value


def probe_hbm(device: int, nbytes: int):
    """(bytes/s, ms per copy) of a device copy moving nbytes (half read,
    half written)."""
    rate, ms = ctypes.c_double(), ctypes.c_double()
    _check("fs_probe_hbm", lib().fs_probe_hbm(device, nbytes, ctypes.byref(rate),
                                              ctypes.byref(ms)))
    return rate.value, ms.value


def to_device(a: np.ndarray, device="cuda"):
    """Host uint32/int32 array -> device int32 tensor holding the same bits."""
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(device)


def to_host(t) -> np.ndarray:
    """Device int32 tensor -> host uint32 array with the same bits."""
    return t.detach().cpu().numpy().view(np.uint32)


def empty_ct(count: int, width: int, device="cuda"):
    import torch
    return torch.empty((count, width), dtype=torch.int32, device=device)
