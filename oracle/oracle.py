"""Python face of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this module.  It wraps the plain C oracle in ``oracle.c`` (built with gcc by
``build()``) and adds the network-level runs written out in Python:

* ``lif_step`` / ``network`` -- the encrypted LIF network, composed of the
  oracle's WeightSum (Sec. 4.1, Eq. "noise grows") and bootstrapping
  (Sec. 2.1, Theorem 2.1) with the FHE-Fire / FHE-Reset program functions
  (Sec. 4.2, Eq. FHE-Fire and Eq. FHE-Reset) in the discretised LIF
  recurrence of Theorem 3.1 (Eq. DiscretEquation);
* ``plain_*`` -- the same network on plaintext integers mod p, the
  spike-for-spike reference.

Batches of bootstrappings run on a thread pool (ctypes drops the GIL while a
C call runs); each bootstrapping itself is single-threaded.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# no contraction and no fast-math, so the Box-Muller sampler rounds exactly
# as its source reads
GCC_FLAGS = ["-O3", "-mavx2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (test infrastructure, not the product)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _CParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("N", ctypes.c_uint32), ("l", ctypes.c_uint32),
                ("bg_bit", ctypes.c_uint32), ("ks_t", ctypes.c_uint32),
                ("ks_base_bit", ctypes.c_uint32), ("p", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("sigma_lwe", ctypes.c_double), ("sigma_bsk", ctypes.c_double),
                ("sigma_ksk", ctypes.c_double)]


_L = None


def lib():
    global _L
    if _L is None:
        build()
        L = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        P = ctypes.POINTER(_CParams)
        sz = ctypes.c_size_t
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        sig = {
            "or_chacha_quarter": (None, [u32p, u32p, u32p, u32p]),
            "or_chacha20_block": (None, [u32p, u32, u32p, u32p]),
            "or_stream_word": (u32, [u64, u32, u64, u64]),
            "or_gauss_from_words": (u32, [u32, u32, ctypes.c_double]),
            "or_negacyclic_mul": (None, [u32, u32p, u32p, u32p]),
            "or_mul_xpow": (None, [u32, u32, u32p, u32p]),
            "or_secret_keys": (None, [P, u64, i32p, i32p]),
            "or_keygen_bsk_range": (None, [P, u64, i32p, i32p, u32, u32, u32p]),
            "or_keygen_ksk_range": (None, [P, u64, i32p, i32p, u32, u32, u32p]),
            "or_encrypt": (None, [P, i32p, i32p, sz, u64, u64, u32p]),
            "or_decrypt": (None, [u32, i32p, u32, u32p, sz, i32p]),
            "or_phase": (None, [i32p, u32, u32p, sz, u32p]),
            "or_test_poly": (ctypes.c_int, [u32, u32, i32p, u32p]),
            "or_test_poly_ms": (ctypes.c_int, [u32, u32, u32, i32p, u32p]),
            "or_mod_switch": (u32, [u32, u32]),
            "or_mod_switch_even": (u32, [u32, u32]),
            "or_blind_rotate_ms": (None, [P, u32p, u32p, u32p, ctypes.c_int, u32p]),
            "or_sample_extract_at": (None, [u32, u32p, u32, u32p]),
            "or_test_poly_two": (ctypes.c_int, [u32, u32, i32p, i32p, u32p]),
            "or_pbs_two": (None, [P, u32p, u32p, u32p, u32p, ctypes.c_int, u32p, u32p]),
            "or_gadget_digits": (None, [u32, u32, u32, i32p]),
            "or_blind_rotate": (None, [P, u32p, u32p, u32p, u32p]),
            "or_sample_extract": (None, [u32, u32p, u32p]),
            "or_keyswitch": (None, [P, u32p, u32p, u32p]),
            "or_pbs": (None, [P, u32p, u32p, u32p, u32p, ctypes.c_int, u32p]),
            "or_lwe_linear": (None, [u32, i32p, sz, sz, u32p, u32p, u32p]),
            "or_lwe_conv2d": (None, [u32, i32p, u32, u32, u32, u32, u32, u32, u32,
                                     u32p, u32p, u32p]),
            "or_add_plain": (None, [u32, u32, u32p, sz, i32]),
            "or_lut_fire": (None, [u32, i32, i32p]),
            "or_leak": (i32, [i32, u32]),
            "or_lut_reset": (None, [u32, i32, u32, i32p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _L = L
    return _L


def _u32(a):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _i32(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


@dataclass(frozen=True)
class Params:
    """TFHE parameters (k = 1, q = 2^32)."""
    n: int = 630
    N: int = 1024
    l: int = 3
    bg_bit: int = 7
    ks_t: int = 8
    ks_base_bit: int = 2
    p: int = 32
    sigma_lwe: float = 2.0 ** -15
    sigma_bsk: float = 2.0 ** -25
    sigma_ksk: float = 2.0 ** -15

    def c(self):
        return _CParams(self.n, self.N, self.l, self.bg_bit, self.ks_t, self.ks_base_bit,
                        self.p, 0, self.sigma_lwe, self.sigma_bsk, self.sigma_ksk)

    @property
    def delta(self):
        return (1 << 32) // self.p


# the two shapes the workloads use
SHAPE_A = Params()
SHAPE_B = Params(N=2048, l=2, bg_bit=10, p=64, sigma_bsk=2.0 ** -31)


def threads() -> int:
    """Worker threads for batches (bounded: the GPU host gives one GPU 16 cores)."""
    return max(1, min(16, os.cpu_count() or 1))


def _pmap(fn, items, nthreads=None):
    items = list(items)
    nt = nthreads or threads()
    if nt <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(nt) as ex:
        return list(ex.map(fn, items))


# ---------------------------------------------------------------- keys

@dataclass
class Keys:
    params: Params
    s: np.ndarray     # int32[n], binary LWE secret
    z: np.ndarray     # int32[N], binary RLWE secret
    bsk: np.ndarray   # uint32[n][2l][2][N], TGSW_z(s_i), coefficient domain
    ksk: np.ndarray   # uint32[N][t][base-1][n+1], LWE_s encryptions


def secret_keys(P: Params, seed: int):
    s = np.zeros(P.n, np.int32)
    z = np.zeros(P.N, np.int32)
    lib().or_secret_keys(ctypes.byref(P.c()), seed, _i32(s), _i32(z))
    return s, z


def keygen(P: Params, seed: int, with_ksk: bool = True, nthreads=None) -> Keys:
    """Secret keys, bootstrapping key and key-switching key from one seed."""
    L = lib()
    s, z = secret_keys(P, seed)
    bsk = np.zeros((P.n, 2 * P.l, 2, P.N), np.uint32)
    base = 1 << P.ks_base_bit
    ksk = np.zeros((P.N, P.ks_t, base - 1, P.n + 1), np.uint32)
    pc = P.c()
    nt = nthreads or threads()
    bsplit = [(int(c[0]), int(c[-1]) + 1) for c in np.array_split(np.arange(P.n), nt) if len(c)]
    _pmap(lambda r: L.or_keygen_bsk_range(ctypes.byref(pc), seed, _i32(s), _i32(z),
                                          r[0], r[1], _u32(bsk)), bsplit, nt)
    if with_ksk:
        ksplit = [(int(c[0]), int(c[-1]) + 1) for c in np.array_split(np.arange(P.N), nt) if len(c)]
        _pmap(lambda r: L.or_keygen_ksk_range(ctypes.byref(pc), seed, _i32(s), _i32(z),
                                              r[0], r[1], _u32(ksk)), ksplit, nt)
    return Keys(P, s, z, bsk, ksk)


# ---------------------------------------------------------------- LWE

def encrypt(P: Params, s, m, seed: int, first_index: int = 0):
    m = _c(np.atleast_1d(m), np.int32)
    ct = np.zeros((m.size, P.n + 1), np.uint32)
    lib().or_encrypt(ctypes.byref(P.c()), _i32(_c(s, np.int32)), _i32(m), m.size, seed,
                     first_index, _u32(ct))
    return ct


def encrypt_z(P: Params, z, m, seed: int, first_index: int = 0):
    """The same LWE encryption with the RLWE secret z as the key (dimension
    N): the form of the samples that sample extraction produces."""
    return encrypt(replace(P, n=P.N), z, m, seed, first_index)


def decrypt(p: int, key, ct):
    ct = _c(np.atleast_2d(ct), np.uint32)
    key = _c(key, np.int32)
    m = np.zeros(ct.shape[0], np.int32)
    lib().or_decrypt(p, _i32(key), key.size, _u32(ct), ct.shape[0], _i32(m))
    return m


def phase(key, ct):
    ct = _c(np.atleast_2d(ct), np.uint32)
    key = _c(key, np.int32)
    out = np.zeros(ct.shape[0], np.uint32)
    lib().or_phase(_i32(key), key.size, _u32(ct), ct.shape[0], _u32(out))
    return out


def add_plain(p: int, ct, c: int):
    ct = _c(ct, np.uint32).copy()
    lib().or_add_plain(p, ct.shape[-1] - 1, _u32(ct), ct.shape[0], int(c))
    return ct


# ---------------------------------------------------------------- ring / PBS pieces

def negacyclic_mul(a, b):
    a = _c(a, np.uint32)
    b = _c(b, np.uint32)
    out = np.zeros_like(a)
    lib().or_negacyclic_mul(a.size, _u32(a), _u32(b), _u32(out))
    return out


def mul_xpow(e: int, a):
    a = _c(a, np.uint32)
    out = np.zeros_like(a)
    lib().or_mul_xpow(a.size, e, _u32(a), _u32(out))
    return out


def mod_switch(x: int, N: int) -> int:
    return int(lib().or_mod_switch(int(x) & 0xFFFFFFFF, N))


def gadget_digits(x: int, l: int, bg_bit: int):
    d = np.zeros(l, np.int32)
    lib().or_gadget_digits(int(x) & 0xFFFFFFFF, l, bg_bit, _i32(d))
    return d


def test_poly(N: int, p: int, f, p_out: int | None = None):
    """Test polynomial of f: Z_p -> Z_p, or f: Z_p -> Z_p_out when p_out is
    given (outputs encoded with 2^32 / p_out)."""
    f = _c(f, np.int32)
    v = np.zeros(N, np.uint32)
    if p_out is None:
        rc = lib().or_test_poly(N, p, _i32(f), _u32(v))
    else:
        rc = lib().or_test_poly_ms(N, p, p_out, _i32(f), _u32(v))
    if rc != 0:
        raise ValueError("program function is not negacyclic: f(r+p/2) != -f(r)")
    return v


def lut_fire(p: int, vth: int):
    f = np.zeros(p, np.int32)
    lib().or_lut_fire(p, vth, _i32(f))
    return f


def lut_reset(p: int, vth: int, tau: int):
    f = np.zeros(p, np.int32)
    lib().or_lut_reset(p, vth, tau, _i32(f))
    return f


def leak(h: int, tau: int) -> int:
    return int(lib().or_leak(h, tau))


def blind_rotate(keys: Keys, v, ct):
    P = keys.params
    acc = np.zeros((2, P.N), np.uint32)
    lib().or_blind_rotate(ctypes.byref(P.c()), _u32(keys.bsk), _u32(_c(v, np.uint32)),
                          _u32(_c(ct, np.uint32)), _u32(acc))
    return acc


def mod_switch_even(x: int, N: int) -> int:
    return int(lib().or_mod_switch_even(int(x) & 0xFFFFFFFF, N))


def blind_rotate_even(keys: Keys, v, ct):
    """Blind rotation with every exponent rounded to an even one."""
    P = keys.params
    acc = np.zeros((2, P.N), np.uint32)
    lib().or_blind_rotate_ms(ctypes.byref(P.c()), _u32(keys.bsk), _u32(_c(v, np.uint32)),
                             _u32(_c(ct, np.uint32)), 1, _u32(acc))
    return acc


def sample_extract_at(acc, k: int):
    acc = _c(acc, np.uint32)
    N = acc.shape[-1]
    out = np.zeros(N + 1, np.uint32)
    lib().or_sample_extract_at(N, _u32(acc), k, _u32(out))
    return out


def test_poly_two(N: int, p: int, f0, f1):
    """Two program functions interleaved in one test polynomial."""
    v = np.zeros(N, np.uint32)
    rc = lib().or_test_poly_two(N, p, _i32(_c(f0, np.int32)), _i32(_c(f1, np.int32)), _u32(v))
    if rc != 0:
        raise ValueError("program function is not negacyclic: f(r+p/2) != -f(r)")
    return v


def pbs_two_from_one(keys: Keys, v, cts, keyswitch: bool = True, nthreads=None):
    """Both functions of a test_poly_two polynomial from one blind rotation
    per row: returns (out0, out1)."""
    P = keys.params
    cts = _c(np.atleast_2d(cts), np.uint32)
    v = _c(v, np.uint32)
    dim = (P.n + 1) if keyswitch else (P.N + 1)
    out = np.zeros((2, cts.shape[0], dim), np.uint32)
    L = lib()
    pc = P.c()

    def one(k):
        L.or_pbs_two(ctypes.byref(pc), _u32(keys.bsk), _u32(keys.ksk), _u32(v), _u32(cts[k]),
                     1 if keyswitch else 0, _u32(out[0, k]), _u32(out[1, k]))
    _pmap(one, range(cts.shape[0]), nthreads)
    return out[0], out[1]


def lif_step_one_rotation(keys: Keys, vth: int, tau: int, h, nthreads=None):
    """The LIF activation with Fire and Reset read from one blind rotation
    (their tables interleaved in one test polynomial): (LWE(2S), LWE(V'))."""
    P = keys.params
    v = test_poly_two(P.N, P.p, lut_fire(P.p, vth), lut_reset(P.p, vth, tau))
    s, r = pbs_two_from_one(keys, v, _c(np.atleast_2d(h), np.uint32), True, nthreads)
    return add_plain(P.p, s, 1), r


def sample_extract(acc):
    acc = _c(acc, np.uint32)
    N = acc.shape[-1]
    out = np.zeros(N + 1, np.uint32)
    lib().or_sample_extract(N, _u32(acc), _u32(out))
    return out


def keyswitch(keys: Keys, ext):
    P = keys.params
    ext = _c(np.atleast_2d(ext), np.uint32)
    out = np.zeros((ext.shape[0], P.n + 1), np.uint32)
    L = lib()
    pc = P.c()

    def one(k):
        L.or_keyswitch(ctypes.byref(pc), _u32(keys.ksk), _u32(ext[k]), _u32(out[k]))
    _pmap(one, range(ext.shape[0]))
    return out


def pbs(keys: Keys, v, cts, keyswitch: bool = True, nthreads=None):
    """Bootstrap every row of cts with test polynomial v (batched on threads)."""
    P = keys.params
    cts = _c(np.atleast_2d(cts), np.uint32)
    v = _c(v, np.uint32)
    dim = (P.n + 1) if keyswitch else (P.N + 1)
    out = np.zeros((cts.shape[0], dim), np.uint32)
    L = lib()
    pc = P.c()

    def one(k):
        L.or_pbs(ctypes.byref(pc), _u32(keys.bsk), _u32(keys.ksk), _u32(v), _u32(cts[k]),
                 1 if keyswitch else 0, _u32(out[k]))
    _pmap(one, range(cts.shape[0]), nthreads)
    return out


# ---------------------------------------------------------------- WeightSum

def lwe_linear(W, x, add=None):
    W = _c(W, np.int32)
    x = _c(x, np.uint32)
    O, I = W.shape
    dim1 = x.shape[1]
    y = np.zeros((O, dim1), np.uint32)
    a = _c(add, np.uint32) if add is not None else None
    lib().or_lwe_linear(dim1, _i32(W), O, I, _u32(x), _u32(a) if a is not None else None, _u32(y))
    return y


def lwe_conv2d(W, x, Ci, H, Wd, stride, pad, add=None):
    W = _c(W, np.int32)
    x = _c(x, np.uint32)
    Co, _, K, _ = W.shape
    Ho = (H + 2 * pad - K) // stride + 1
    Wo = (Wd + 2 * pad - K) // stride + 1
    dim1 = x.shape[1]
    y = np.zeros((Co * Ho * Wo, dim1), np.uint32)
    a = _c(add, np.uint32) if add is not None else None
    lib().or_lwe_conv2d(dim1, _i32(W), Ci, H, Wd, Co, K, stride, pad, _u32(x),
                        _u32(a) if a is not None else None, _u32(y))
    return y


# ---------------------------------------------------------------- LIF (Sec. 4.2)

def lif_test_polys(P: Params, vth: int, tau: int):
    """Test polynomials of FHE-Fire (threshold folded in) and FHE-Reset."""
    return test_poly(P.N, P.p, lut_fire(P.p, vth)), test_poly(P.N, P.p, lut_reset(P.p, vth, tau))


def lif_step(keys: Keys, vth: int, tau: int, h, nthreads=None):
    """One LIF activation on ciphertexts LWE(H): returns (LWE(2S), LWE(V')).

    2S = bootstrap_Fire(LWE(H)) + 1 and V' = bootstrap_Reset(LWE(H))
    (Eq. FHE-Fire, Eq. FHE-Reset); both bootstrap the same input."""
    P = keys.params
    vf, vr = lif_test_polys(P, vth, tau)
    h = _c(np.atleast_2d(h), np.uint32)
    both = pbs_two(keys, vf, vr, h, nthreads)
    spikes = add_plain(P.p, both[0], 1)
    return spikes, both[1]


def lif_step_ks_first(keys: Keys, vth: int, tau: int, h_z, nthreads=None):
    """The LIF activation with the bootstrapping's steps reordered (Sec. 2.1:
    Key Switching moved in front of the Blind Rotation): LWE_z(H) is
    key-switched to LWE_s(H), which both functions then bootstrap without a
    key switch; returns (LWE_z(2S), LWE_z(V'))."""
    P = keys.params
    vf, vr = lif_test_polys(P, vth, tau)
    hs = keyswitch(keys, _c(np.atleast_2d(h_z), np.uint32))
    spikes = add_plain(P.p, pbs(keys, vf, hs, keyswitch=False, nthreads=nthreads), 1)
    return spikes, pbs(keys, vr, hs, keyswitch=False, nthreads=nthreads)


def pbs_two(keys, v0, v1, h, nthreads=None):
    """Bootstrap every row of h with two test polynomials (one thread pool)."""
    P = keys.params
    B = h.shape[0]
    out = np.zeros((2, B, P.n + 1), np.uint32)
    L = lib()
    pc = P.c()
    vs = (_c(v0, np.uint32), _c(v1, np.uint32))

    def one(job):
        which, k = job
        L.or_pbs(ctypes.byref(pc), _u32(keys.bsk), _u32(keys.ksk), _u32(vs[which]),
                 _u32(h[k]), 1, _u32(out[which, k]))
    _pmap(one, [(w, k) for k in range(B) for w in (0, 1)], nthreads)
    return out


# ---------------------------------------------------------------- plaintext SNN

def plain_fire(p: int, vth: int, h):
    """2S from residues H: Fire LUT + 1, i.e. 2 when (H - V) mod p in [0, p/2)."""
    f = lut_fire(p, vth)
    return (f[np.asarray(h) % p] + 1) % p


def plain_reset(p: int, vth: int, tau: int, h):
    f = lut_reset(p, vth, tau)
    return f[np.asarray(h) % p] % p


def centred(p: int, r):
    r = np.asarray(r, np.int64) % p
    return np.where(r > p // 2, r - p, r)


# ---------------------------------------------------------------- networks (Theorem 3.1 recurrence)

def zero_ct(count: int, dim1: int):
    """V[0]: the all-zero ciphertext (a trivial encryption of 0)."""
    return np.zeros((count, dim1), np.uint32)


def lif_layer_run(keys: Keys, I_ct, vth: int, tau: int, T: int, nthreads=None,
                  ks_first: bool = False, one_rotation: bool = False):
    """One LIF layer driven by a static input current LWE(I) for T steps:
    H[t] = V[t-1] + I; (2S[t], V[t]) = (FHE-Fire(H) + 1, FHE-Reset(H)).
    Returns lists (per step) of H, 2S and V ciphertexts.  ks_first: the
    ciphertexts are under z and each step uses lif_step_ks_first;
    one_rotation: each step uses lif_step_one_rotation."""
    step = (lif_step_ks_first if ks_first else
            lif_step_one_rotation if one_rotation else lif_step)
    V = zero_ct(I_ct.shape[0], I_ct.shape[1])
    Hs, Ss, Vs = [], [], []
    for _ in range(T):
        H = (V + I_ct).astype(np.uint32)
        S2, V = step(keys, vth, tau, H, nthreads)
        Hs.append(H); Ss.append(S2); Vs.append(V)
    return Hs, Ss, Vs


def conv_snn_run(keys: Keys, px_ct, Wc, W1, W2, geom, vth: int, tau: int, T: int, nthreads=None,
                 one_rotation: bool = False):
    """Conv layer (LIF) -> FC (LIF) -> FC accumulators, T steps; the conv
    current is computed once since the encrypted image is static.
    geom = (Ci, H, Wd, stride, pad).  Returns per-step dicts of ciphertexts.
    one_rotation: each LIF step uses lif_step_one_rotation."""
    lif_step_ = lif_step_one_rotation if one_rotation else lif_step
    Ci, H, Wd, st, pd = geom
    I1 = lwe_conv2d(Wc, px_ct, Ci, H, Wd, st, pd)
    V1 = zero_ct(*I1.shape)
    V2 = zero_ct(W1.shape[0], I1.shape[1])
    score = zero_ct(W2.shape[0], I1.shape[1])
    steps = []
    for _ in range(T):
        H1 = (V1 + I1).astype(np.uint32)
        S1, V1 = lif_step_(keys, vth, tau, H1, nthreads)
        H2 = lwe_linear(W1, S1, add=V2)
        S2, V2 = lif_step_(keys, vth, tau, H2, nthreads)
        score = lwe_linear(W2, S2, add=score)
        steps.append(dict(H1=H1, S1=S1, V1=V1, H2=H2, S2=S2, V2=V2, score=score.copy()))
    return I1, steps


def lwe_sum_pool(ct, C: int, H: int, W: int, k: int):
    """Sum of each k x k window (stride k) of a [C*H*W] grid of ciphertexts:
    the numerator of the average pool, whose division by n = k^2 moves into
    the next layer's weights (Sec. 3.3, the average-pooling equation: the
    weights are discretised with scale theta / n and multiply the window
    sum of spikes)."""
    ct = np.asarray(ct, np.uint32).reshape(C, H, W, -1)
    Ho, Wo = H // k, W // k
    out = np.zeros((C, Ho, Wo, ct.shape[-1]), np.uint64)
    for dy in range(k):
        for dx in range(k):
            out += ct[:, dy:dy + k * Ho:k, dx:dx + k * Wo:k, :]
    return (out & 0xFFFFFFFF).astype(np.uint32).reshape(C * Ho * Wo, -1)


def paper_csnn_run(keys: Keys, px_ct, Wc, W1, W2, geom, pool: int, vth: int, tau: int, T: int,
                   nthreads=None, one_rotation: bool = False):
    """The paper's CSNN (Sec. 3.1) on ciphertexts: conv (LIF) -> average pool
    (window sum, Sec. 3.3) -> FC (LIF) -> FC (LIF), scores = the encrypted
    spike counts of the output layer, sum_t LWE(2S[t]).  Two bootstrappings
    per LIF neuron per step (Table 1).  geom = (Ci, H, Wd, stride, pad).
    one_rotation: each LIF step uses lif_step_one_rotation."""
    lif_step_ = lif_step_one_rotation if one_rotation else lif_step
    Ci, H, Wd, st, pd = geom
    Co, _, K, _ = np.asarray(Wc).shape
    Ho = (H + 2 * pd - K) // st + 1
    Wo = (Wd + 2 * pd - K) // st + 1
    I1 = lwe_conv2d(Wc, px_ct, Ci, H, Wd, st, pd)
    w = I1.shape[1]
    V1 = zero_ct(*I1.shape)
    V2 = zero_ct(W1.shape[0], w)
    V3 = zero_ct(W2.shape[0], w)
    score = zero_ct(W2.shape[0], w)
    steps = []
    for _ in range(T):
        H1 = (V1 + I1).astype(np.uint32)
        S1, V1 = lif_step_(keys, vth, tau, H1, nthreads)
        H2 = lwe_linear(W1, lwe_sum_pool(S1, Co, Ho, Wo, pool), add=V2)
        S2, V2 = lif_step_(keys, vth, tau, H2, nthreads)
        H3 = lwe_linear(W2, S2, add=V3)
        S3, V3 = lif_step_(keys, vth, tau, H3, nthreads)
        score = (score.astype(np.uint64) + S3).astype(np.uint32)
        steps.append(dict(H1=H1, S1=S1, V1=V1, H2=H2, S2=S2, V2=V2, H3=H3, S3=S3, V3=V3,
                          score=score.copy()))
    return I1, steps


def add_plain_rows(p: int, ct, c):
    """Row i plus the trivial encryption of c[i]: b += Delta c[i] (Sec. 4.1,
    adding a plaintext to a ciphertext)."""
    ct = np.array(ct, np.uint32, copy=True)
    delta = (1 << 32) // p
    c = np.asarray(c, np.int64)
    ct[:, -1] = ((ct[:, -1].astype(np.int64) + delta * c) & 0xFFFFFFFF).astype(np.uint32)
    return ct


def poisson_spikes(keys: Keys, px_ct, m_t):
    """Poisson coding on ciphertexts (Sec. 2.3: X = 1 iff X_o > M_t; Sec. 5.1:
    one comparison = one Sign bootstrapping): LWE(q - m_t) through the Fire
    function with threshold 1 (+1 if q - m_t >= 1, else -1), then +1 as in
    Eq. FHE-Fire, giving LWE(2X)."""
    P = keys.params
    h = add_plain_rows(P.p, px_ct, -np.asarray(m_t, np.int64))
    s = pbs(keys, test_poly(P.N, P.p, lut_fire(P.p, 1)), h, keyswitch=True)
    return add_plain(P.p, s, 1)


def poisson_snn_run(keys: Keys, px_ct, thresholds, W1, W2, vth: int, tau: int, T: int,
                    nthreads=None, one_rotation: bool = False):
    """The Poisson-encoded SNN (Sec. 5.1, Table 1): per step the pixel spikes
    of poisson_spikes, FC (LIF), FC (LIF), scores = the encrypted spike counts
    of the output layer.  one_rotation: the LIF steps use
    lif_step_one_rotation."""
    lif_step_ = lif_step_one_rotation if one_rotation else lif_step
    w = np.asarray(px_ct).shape[1]
    V1 = zero_ct(W1.shape[0], w)
    V2 = zero_ct(W2.shape[0], w)
    score = zero_ct(W2.shape[0], w)
    steps = []
    for t in range(T):
        S0 = poisson_spikes(keys, px_ct, thresholds[t])
        H1 = lwe_linear(W1, S0, add=V1)
        S1, V1 = lif_step_(keys, vth, tau, H1, nthreads)
        H2 = lwe_linear(W2, S1, add=V2)
        S2, V2 = lif_step_(keys, vth, tau, H2, nthreads)
        score = (score.astype(np.uint64) + S2).astype(np.uint32)
        steps.append(dict(S0=S0, H1=H1, S1=S1, V1=V1, H2=H2, S2=S2, V2=V2, score=score.copy()))
    return steps


# ---------------------------------------------------------------- plaintext SNN (mod p)

def plain_lif_layer_run(p: int, I, vth: int, tau: int, T: int):
    """The same recurrence on integers mod p (residues in [0, p))."""
    I = np.asarray(I, np.int64) % p
    V = np.zeros_like(I)
    Hs, Ss, Vs = [], [], []
    for _ in range(T):
        H = (V + I) % p
        S2 = plain_fire(p, vth, H)
        V = plain_reset(p, vth, tau, H)
        Hs.append(H); Ss.append(S2); Vs.append(V)
    return Hs, Ss, Vs


def plain_conv2d(W, x, Ci, H, Wd, stride, pad):
    """Integer 2-D cross-correlation with zero padding, x: [Ci*H*Wd]."""
    W = np.asarray(W, np.int64)
    Co, _, K, _ = W.shape
    xi = np.asarray(x, np.int64).reshape(Ci, H, Wd)
    xp = np.zeros((Ci, H + 2 * pad, Wd + 2 * pad), np.int64)
    xp[:, pad:pad + H, pad:pad + Wd] = xi
    Ho = (H + 2 * pad - K) // stride + 1
    Wo = (Wd + 2 * pad - K) // stride + 1
    y = np.zeros((Co, Ho, Wo), np.int64)
    for co in range(Co):
        for oy in range(Ho):
            for ox in range(Wo):
                win = xp[:, oy * stride:oy * stride + K, ox * stride:ox * stride + K]
                y[co, oy, ox] = int((win * W[co]).sum())
    return y.reshape(-1)


def plain_conv_snn_run(p: int, px, Wc, W1, W2, geom, vth: int, tau: int, T: int):
    Ci, H, Wd, st, pd = geom
    I1 = plain_conv2d(Wc, px, Ci, H, Wd, st, pd) % p
    V1 = np.zeros_like(I1)
    V2 = np.zeros(W1.shape[0], np.int64)
    score = np.zeros(W2.shape[0], np.int64)
    steps = []
    W1 = np.asarray(W1, np.int64)
    W2 = np.asarray(W2, np.int64)
    for _ in range(T):
        H1 = (V1 + I1) % p
        S1 = plain_fire(p, vth, H1)
        V1 = plain_reset(p, vth, tau, H1)
        H2 = (V2 + W1 @ S1) % p
        S2 = plain_fire(p, vth, H2)
        V2 = plain_reset(p, vth, tau, H2)
        score = (score + W2 @ S2) % p
        steps.append(dict(H1=H1, S1=S1, V1=V1, H2=H2, S2=S2, V2=V2, score=score.copy()))
    return I1, steps


def plain_paper_csnn_run(p: int, px, Wc, W1, W2, geom, pool: int, vth: int, tau: int, T: int):
    """paper_csnn_run on integers mod p."""
    Ci, H, Wd, st, pd = geom
    Wc = np.asarray(Wc, np.int64)
    Co, _, K, _ = Wc.shape
    Ho = (H + 2 * pd - K) // st + 1
    Wo = (Wd + 2 * pd - K) // st + 1
    I1 = plain_conv2d(Wc, px, Ci, H, Wd, st, pd) % p
    W1 = np.asarray(W1, np.int64)
    W2 = np.asarray(W2, np.int64)
    V1 = np.zeros_like(I1)
    V2 = np.zeros(W1.shape[0], np.int64)
    V3 = np.zeros(W2.shape[0], np.int64)
    score = np.zeros(W2.shape[0], np.int64)
    steps = []
    for _ in range(T):
        H1 = (V1 + I1) % p
        S1 = plain_fire(p, vth, H1)
        V1 = plain_reset(p, vth, tau, H1)
        g = S1.reshape(Co, Ho, Wo)
        pooled = sum(g[:, dy:dy + pool * (Ho // pool):pool, dx:dx + pool * (Wo // pool):pool]
                     for dy in range(pool) for dx in range(pool)).reshape(-1)
        H2 = (V2 + W1 @ pooled) % p
        S2 = plain_fire(p, vth, H2)
        V2 = plain_reset(p, vth, tau, H2)
        H3 = (V3 + W2 @ S2) % p
        S3 = plain_fire(p, vth, H3)
        V3 = plain_reset(p, vth, tau, H3)
        score = (score + S3) % p
        steps.append(dict(H1=H1, S1=S1, V1=V1, H2=H2, S2=S2, V2=V2, H3=H3, S3=S3, V3=V3,
                          score=score.copy()))
    return I1, steps


def plain_poisson_snn_run(p: int, px, thresholds, W1, W2, vth: int, tau: int, T: int):
    """poisson_snn_run on integers mod p: 2X = 2 [q > m_t]."""
    px = np.asarray(px, np.int64)
    W1 = np.asarray(W1, np.int64)
    W2 = np.asarray(W2, np.int64)
    V1 = np.zeros(W1.shape[0], np.int64)
    V2 = np.zeros(W2.shape[0], np.int64)
    score = np.zeros(W2.shape[0], np.int64)
    steps = []
    for t in range(T):
        S0 = 2 * (px > np.asarray(thresholds[t], np.int64)).astype(np.int64)
        H1 = (V1 + W1 @ S0) % p
        S1 = plain_fire(p, vth, H1)
        V1 = plain_reset(p, vth, tau, H1)
        H2 = (V2 + W2 @ S1) % p
        S2 = plain_fire(p, vth, H2)
        V2 = plain_reset(p, vth, tau, H2)
        score = (score + S2) % p
        steps.append(dict(S0=S0, H1=H1, S1=S1, V1=V1, H2=H2, S2=S2, V2=V2, score=score.copy()))
    return steps
