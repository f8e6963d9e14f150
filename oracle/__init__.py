"""CPU oracle for the recursive hypot-based norms -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  It shares no code with the GPU library.

Library contract applied on top of the paper's recursions (the paper's theorems
assume finite inputs; this is the build's reading): n <= 0 gives 0; any NaN input
gives NaN; otherwise any infinite input gives +inf; otherwise the recursion runs
(and may overflow to +inf).

Algorithms (paper: Novakovic, arXiv 2509.06220):
  'A'  R with cr_hypot (Sect. 2, Listing 1, Table 2)        -- the parity oracle
  'H'  R with v1_hypot (Listing 2)
  'Z'  Z with P lanes and the v1 node, then A (Sect. 3, Listing 4; the recommended xNRMF)
p-norms: R (or Z) with the Listing 5 node v1_lp using a correctly rounded pow;
p = 1 -> sumabs (Eq. vp1); p = inf or p >= cutoff (2^53 D, 2^24 S) -> maxabs (Eq. vpI).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import bounds, exact  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "vnp_oracle.c")
PLAIN_LIB = os.path.join(_HERE, "libvnp_oracle.so")
SANITIZED_LIB = os.path.join(_HERE, "libvnp_oracle_asan.so")
# VNP_ORACLE_SANITIZED=1 loads the AddressSanitizer + UndefinedBehaviorSanitizer build
# (the process must preload the ASan runtime; see tests/test_oracle_sanitized.py)
LIB = SANITIZED_LIB if os.environ.get("VNP_ORACLE_SANITIZED") == "1" else PLAIN_LIB

CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11"]
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
LIBS = ["-lquadmath", "-lm", "-ldl"]


def _compile(out, extra):
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, *extra, SRC, "-o", tmp, *LIBS])
    os.replace(tmp, out)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no SIMD options, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        _compile(LIB, SANITIZE if LIB == SANITIZED_LIB else [])
    return LIB


def build_sanitized(force: bool = False) -> str:
    """The same oracle built with AddressSanitizer and UndefinedBehaviorSanitizer."""
    if force or not os.path.exists(SANITIZED_LIB) or os.path.getmtime(SANITIZED_LIB) < os.path.getmtime(SRC):
        _compile(SANITIZED_LIB, SANITIZE)
    return SANITIZED_LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(LIB)
        d, f, i64, i, vp = ctypes.c_double, ctypes.c_float, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        sig = {
            "vnpo_cr_hypot": (d, [d, d]),
            "vnpo_cr_hypotf": (f, [f, f]),
            "vnpo_v1_hypot": (d, [d, d]),
            "vnpo_v1_hypotf": (f, [f, f]),
            "vnpo_cr_pow": (d, [d, d]),
            "vnpo_cr_powf": (f, [f, f]),
            "vnpo_v1_lp": (d, [d, d, d]),
            "vnpo_v1_lpf": (f, [f, f, f]),
            "vnpo_dnrm_acc": (d, [i64, vp]),
            "vnpo_snrm_acc": (f, [i64, vp]),
            "vnpo_dnrmf_R": (d, [i64, vp, i, i]),
            "vnpo_snrmf_R": (f, [i64, vp, i, i]),
            "vnpo_dnrmp_R": (d, [i64, vp, d, i]),
            "vnpo_snrmp_R": (f, [i64, vp, f, i]),
            "vnpo_dnrmf_Z": (d, [i64, vp, i, i, i]),
            "vnpo_snrmf_Z": (f, [i64, vp, i, i, i]),
            "vnpo_dnrmp_Z": (d, [i64, vp, d, i, i]),
            "vnpo_snrmp_Z": (f, [i64, vp, f, i, i]),
            "vnpo_trace": (i64, [i64, i, vp]),
            "vnpo_sumsq_exact": (i, [i64, vp, i, vp, i]),
            "vnpo_sa_limbs": (i, []),
            "vnpo_sa_bias": (i, []),
            "vnpo_pnorm_quad": (None, [i64, vp, i, d, i, vp, vp]),
            "vnpo_pnorm_R_quad": (None, [i64, vp, i, d, d, i, vp, vp]),
            "vnpo_powq2": (None, [d, d, vp, vp]),
            "vnpo_pow_ambiguous": (i64, []),
            "vnpo_pow_unresolved": (i64, []),
            "vnpo_mpfr_pow": (d, [d, d, i]),
            "vnpo_exact_failures": (i64, []),
            "vnpo_reset_counters": (None, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


# ---------------------------------------------------------------- scalar nodes
def cr_hypot(x, y):
    return _L().vnpo_cr_hypot(float(x), float(y))


def cr_hypotf(x, y):
    return float(np.float32(_L().vnpo_cr_hypotf(float(x), float(y))))


def v1_hypot(x, y):
    return _L().vnpo_v1_hypot(float(x), float(y))


def v1_hypotf(x, y):
    return float(np.float32(_L().vnpo_v1_hypotf(float(x), float(y))))


def cr_pow(x, y):
    return _L().vnpo_cr_pow(float(x), float(y))


def cr_powf(x, y):
    return float(np.float32(_L().vnpo_cr_powf(float(x), float(y))))


def v1_lp(p, x, y):
    return _L().vnpo_v1_lp(float(p), float(x), float(y))


def v1_lpf(p, x, y):
    return float(np.float32(_L().vnpo_v1_lpf(float(p), float(x), float(y))))


def powq(x, y):
    """binary128 x^y as an exact hi + lo pair of doubles (for pinning the pow evaluation)."""
    hi, lo = ctypes.c_double(), ctypes.c_double()
    _L().vnpo_powq2(float(x), float(y), ctypes.byref(hi), ctypes.byref(lo))
    return hi.value, lo.value


def mpfr_pow(x, y, prec=53):
    """GNU MPFR's correctly rounded pow (the oracle's fallback), for pinning cr_pow."""
    return _L().vnpo_mpfr_pow(float(x), float(y), int(prec))


def counters():
    L = _L()
    return {"pow_ambiguous": L.vnpo_pow_ambiguous(), "pow_unresolved": L.vnpo_pow_unresolved(),
            "exact_failures": L.vnpo_exact_failures()}


def reset_counters():
    _L().vnpo_reset_counters()


# ---------------------------------------------------------------- norms
def _prep(x):
    x = np.ascontiguousarray(x)
    if x.dtype not in (np.float64, np.float32):
        raise TypeError(x.dtype)
    return x


def _contract(x):
    """Returns the contract's value for empty / non-finite inputs, else None."""
    if x.size == 0:
        return x.dtype.type(0.0)
    if not np.all(np.isfinite(x)):
        if np.any(np.isnan(x)):
            return x.dtype.type(np.nan)
        return x.dtype.type(np.inf)
    return None


def nrmf(x, algo: str = "A", lanes: int | None = None, sort: bool = False, threads: int | None = None):
    """Frobenius norm by the paper's algorithm ``algo`` ('A', 'H' or 'Z')."""
    x = _prep(x)
    c = _contract(x)
    if c is not None:
        return c
    L = _L()
    t = threads or default_threads()
    single = x.dtype == np.float32
    n = x.size
    if algo in ("A", "H"):
        node = 0 if algo == "A" else 1
        fn = L.vnpo_snrmf_R if single else L.vnpo_dnrmf_R
        return x.dtype.type(fn(n, x.ctypes.data, node, t))
    if algo == "Z":
        P = lanes or (16 if single else 8)
        fn = L.vnpo_snrmf_Z if single else L.vnpo_dnrmf_Z
        return x.dtype.type(fn(n, x.ctypes.data, P, int(sort), t))
    raise ValueError(algo)


def nrmp(x, p: float, algo: str = "A", lanes: int | None = None, threads: int | None = None):
    """p-norm by the paper's recursion with the Listing 5 node ('A' = R, 'Z' = Z + A)."""
    x = _prep(x)
    if not (p > 0):
        raise ValueError("p must be > 0")
    c = _contract(x)
    if c is not None:
        return c
    L = _L()
    t = threads or default_threads()
    single = x.dtype == np.float32
    n = x.size
    if algo == "A":
        fn = L.vnpo_snrmp_R if single else L.vnpo_dnrmp_R
        return x.dtype.type(fn(n, x.ctypes.data, p, t))
    if algo == "Z":
        P = lanes or (16 if single else 8)
        fn = L.vnpo_snrmp_Z if single else L.vnpo_dnrmp_Z
        return x.dtype.type(fn(n, x.ctypes.data, p, P, t))
    raise ValueError(algo)


def nrm_acc(x):
    """Theorem 1's algorithm: g_i = fma(x_i, x_i, g_{i-1}) in the working precision, then
    sqrt(g_n) (no tree; its error bound grows linearly in n)."""
    x = _prep(x)
    L = _L()
    if x.dtype == np.float32:
        return np.float32(L.vnpo_snrm_acc(x.size, x.ctypes.data))
    return np.float64(L.vnpo_dnrm_acc(x.size, x.ctypes.data))


def schatten(a, m: int, n: int, lda: int, p: float):
    """Schatten p-norm of the m x n column-major matrix in a (leading dimension lda): the
    p-norm of its singular values (Sect. 4, ||G||_{S_p} = ||s||_p).  The singular values
    come from LAPACK (numpy.linalg.svd, a library step); the p-norm is the recursion A_p
    (A for p = 2)."""
    a = _prep(a)
    if m <= 0 or n <= 0:
        return a.dtype.type(0.0)
    G = np.lib.stride_tricks.as_strided(a, shape=(m, n), strides=(a.itemsize, lda * a.itemsize)).copy()
    sv = np.linalg.svd(G, compute_uv=False).astype(a.dtype)
    return nrmf(sv, "A") if p == 2.0 else nrmp(sv, p, "A")


def nrmf_complex(z, incz: int = 1, n: int | None = None, threads: int | None = None):
    """Frobenius norm of a complex vector.  |z_k|^2 = re^2 + im^2 (Sect. 1), so the norm is the
    recursion (A) over the real view (re_0, im_0, re_1, im_1, ...) of the n logical
    elements; element k is z[k incz] for incz >= 1, z[(n - 1 - k) |incz|] for incz <= -1."""
    z = np.asarray(z)
    if not np.iscomplexobj(z):
        raise TypeError("complex input expected")
    if incz == 0:
        raise ValueError("incz == 0")
    if n is None:
        n = (z.size + abs(incz) - 1) // abs(incz) if z.size else 0
    rdt = np.float32 if z.dtype == np.complex64 else np.float64
    if n <= 0:
        return rdt(0.0)
    idx = np.arange(n) * abs(incz)
    if incz < 0:
        idx = idx[::-1]
    zz = z[idx]
    real = np.empty(2 * n, dtype=rdt)
    real[0::2] = zz.real
    real[1::2] = zz.imag
    return nrmf(real, "A", threads=threads)


def nrm_mat(a, m: int, ncols: int, lda: int, p: float = 2.0, threads: int | None = None):
    """Frobenius (p = 2) or entrywise p-norm of the m x ncols column-major array stored in a
    with leading dimension lda (Sect. 3.1): an array stored contiguously (lda == m) is one
    vector; otherwise the norms of its columns are computed by the recursion (A) and then
    reduced by the same recursion, in column order.  Rows m .. lda-1 are never read."""
    a = _prep(a)
    if m <= 0 or ncols <= 0:
        return a.dtype.type(0.0)
    if lda < m:
        raise ValueError("lda < m")
    one = (lambda v: nrmf(v, "A", threads=threads)) if p == 2.0 else (lambda v: nrmp(v, p, "A", threads=threads))
    if lda == m:
        return one(a[:m * ncols])
    norms = np.array([one(a[j * lda:j * lda + m]) for j in range(ncols)], dtype=a.dtype)
    return one(norms)


def trace(n: int, lanes: int = 0):
    """Tree shape: list of (left, right) ids per node in completion order.

    Leaves are 1..n; the k-th node (0-based) has id 1000000 + k."""
    buf = np.zeros(2 * max(n + lanes, 1), dtype=np.int64)
    k = _L().vnpo_trace(n, lanes, buf.ctypes.data)
    return [(int(buf[2 * i]), int(buf[2 * i + 1])) for i in range(k)]


def exact_nrm2(x, threads: int | None = None):
    """RN(sqrt(sum x_i^2)) exactly: superaccumulated squares + exact integer square root."""
    x = _prep(x)
    c = _contract(x)
    if c is not None:
        return c
    L = _L()
    nl = L.vnpo_sa_limbs()
    limbs = np.zeros(nl, dtype=np.uint64)
    L.vnpo_sumsq_exact(x.size, x.ctypes.data, int(x.dtype == np.float32), limbs.ctypes.data,
                       threads or default_threads())
    N = exact.limbs_to_int(limbs)
    fmt = "f32" if x.dtype == np.float32 else "f64"
    return x.dtype.type(exact.rn_sqrt_dyadic(N, -L.vnpo_sa_bias(), fmt))


def ref_pnorm(x, p: float, threads: int | None = None):
    """binary128 reference (sum |x_i|^p)^(1/p) as (hi, lo) doubles (error ~1e-25 relative)."""
    x = _prep(x)
    hi, lo = ctypes.c_double(), ctypes.c_double()
    _L().vnpo_pnorm_quad(x.size, x.ctypes.data, int(x.dtype == np.float32), float(p),
                         threads or default_threads(), ctypes.byref(hi), ctypes.byref(lo))
    return hi.value, lo.value


def ref_pnorm_R(x, p: float, threads: int | None = None):
    """The p-norm recursion R evaluated in binary128 with the method's rounded exponents
    RN(p/2) and RN(1/p) (binary32 roundings for binary32 input), as (hi, lo) doubles."""
    x = _prep(x)
    if x.dtype == np.float32:
        hp, ip = float(np.float32(np.float32(p) * np.float32(0.5))), float(np.float32(1.0) / np.float32(p))
    else:
        hp, ip = p * 0.5, 1.0 / p
    hi, lo = ctypes.c_double(), ctypes.c_double()
    _L().vnpo_pnorm_R_quad(x.size, x.ctypes.data, int(x.dtype == np.float32), hp, ip, threads or default_threads(),
                           ctypes.byref(hi), ctypes.byref(lo))
    return hi.value, lo.value


def relerr(approx, ref, fmt: str) -> float:
    """Eq. (relerr): |ref - approx| / (ref * eps), ref rounded to the working precision."""
    e = 2.0 ** -53 if fmt == "f64" else 2.0 ** -24
    ref = float(ref)
    approx = float(approx)
    if ref == 0:
        return 0.0 if approx == 0 else math.inf
    return abs(ref - approx) / (ref * e)
