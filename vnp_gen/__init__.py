"""Seeded synthetic inputs shared by the GPU tests, the oracle and the benchmark.

No norm arithmetic lives here.  Three implementations of one definition
(SplitMix64 used counter-style; value kinds described in ``gen_host.c``):

* ``np_fill``      -- pure numpy, for small vectors and as the readable definition;
* ``host_fill``    -- C with OpenMP (``libvnp_gen_host.so``), for large host vectors;
* ``dev_fill``     -- HIP kernel (``libvnp_gen_dev.so``), for device-resident inputs.

Workload recipes (``RECIPES``) name the synthetic stand-ins for the benchmark
configurations: sizes, value distributions, exponent windows and seeds.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
HOST_LIB = os.path.join(_HERE, "libvnp_gen_host.so")
DEV_LIB = os.path.join(_HERE, "libvnp_gen_dev.so")

KIND_U11, KIND_EXP, KIND_U11EXP, KIND_U01 = 0, 1, 2, 3
KINDS = {"u11": KIND_U11, "exp": KIND_EXP, "u11exp": KIND_U11EXP, "u01": KIND_U01}

GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1

# name -> (n, kind, lo, hi, seed, stream).  Exponent windows for binary32 copies of
# the binary64 stress windows are the analogous ones of that format.
RECIPES = {
    "c0": dict(n=1 << 20, kind="u11", lo=0, hi=0, seed=0, stream=0),
    "c1": dict(n=1 << 30, kind="exp", lo=-20, hi=20, seed=0, stream=0),
    "c1_overflow_d": dict(n=1 << 30, kind="exp", lo=990, hi=1023, seed=1, stream=0),
    "c1_bigfinite_d": dict(n=1 << 30, kind="exp", lo=990, hi=1007, seed=1, stream=0),
    "c1_subnormal_d": dict(n=1 << 30, kind="exp", lo=-1074, hi=-1000, seed=2, stream=0),
    "c1_overflow_s": dict(n=1 << 30, kind="exp", lo=94, hi=127, seed=1, stream=0),
    "c1_subnormal_s": dict(n=1 << 30, kind="exp", lo=-149, hi=-104, seed=2, stream=0),
    "c2": dict(n=1 << 28, kind="exp", lo=-10, hi=10, seed=0, stream=0),
    "c3_values": dict(n=None, kind="u11exp", lo=-30, hi=30, seed=0, stream=1),
}


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * _M1) & _MASK
    z = ((z ^ (z >> 27)) * _M2) & _MASK
    return z ^ (z >> 31)


def key(seed: int, stream: int) -> int:
    return _mix((seed * GAMMA + _mix(stream)) & _MASK)


def _np_mix(z):
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def np_draws(n: int, i0: int, seed: int, stream: int) -> np.ndarray:
    """Raw 64-bit outputs i0..i0+n-1 of the (seed, stream) SplitMix64 stream."""
    k = np.uint64(key(seed, stream))
    i = np.arange(i0 + 1, i0 + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _np_mix(k + i * np.uint64(GAMMA))


def _exps(rb, lo, hi):
    span = np.uint64(hi - lo + 1)
    return (lo + ((rb >> np.uint64(32)) * span >> np.uint64(32)).astype(np.int64)).astype(np.int32)


def np_fill(n, dtype="f64", kind="u11", lo=0, hi=0, seed=0, stream=0, i0=0) -> np.ndarray:
    """Readable numpy definition of the generator (see gen_host.c)."""
    with np.errstate(over="ignore", under="ignore"):
        return _np_fill(n, dtype, kind, lo, hi, seed, stream, i0)


def _np_fill(n, dtype, kind, lo, hi, seed, stream, i0):
    kind = KINDS[kind] if isinstance(kind, str) else kind
    ra = np_draws(n, i0, seed, 2 * stream)
    rb = np_draws(n, i0, seed, 2 * stream + 1) if kind in (KIND_EXP, KIND_U11EXP) else None
    u53 = np.ldexp((ra >> np.uint64(11)).astype(np.float64), -53)
    if dtype in ("f64", np.float64):
        if kind == KIND_U11:
            return 2.0 * u53 - 1.0
        if kind == KIND_EXP:
            u = 0.5 + np.ldexp((ra >> np.uint64(12)).astype(np.float64), -53)
            u = np.where((ra >> np.uint64(10)) & np.uint64(1), -u, u)
            return np.ldexp(u, _exps(rb, lo, hi))
        if kind == KIND_U11EXP:
            return np.ldexp(2.0 * u53 - 1.0, _exps(rb, lo, hi))
        return u53
    if kind == KIND_U11:
        return (2.0 * u53 - 1.0).astype(np.float32)
    if kind == KIND_EXP:
        u = np.float32(0.5) + np.ldexp((ra >> np.uint64(41)).astype(np.float32), np.int32(-24))
        u = np.where((ra >> np.uint64(10)) & np.uint64(1), -u, u).astype(np.float32)
        return np.ldexp(u, _exps(rb, lo, hi)).astype(np.float32)
    if kind == KIND_U11EXP:
        w = (2.0 * u53 - 1.0).astype(np.float32)
        return np.ldexp(w, _exps(rb, lo, hi)).astype(np.float32)
    return np.ldexp((ra >> np.uint64(40)).astype(np.float32), np.int32(-24)).astype(np.float32)


_host = None
_dev = None


def _load_host():
    global _host
    if _host is None:
        if not os.path.exists(HOST_LIB):
            raise RuntimeError(f"{HOST_LIB} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(HOST_LIB)
        for name, ct in (("vnpg_fill_d", ctypes.c_double), ("vnpg_fill_s", ctypes.c_float)):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
                          ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.vnpg_draws.restype = None
        lib.vnpg_draws.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64]
        _host = lib
    return _host


def host_fill(n, dtype="f64", kind="u11", lo=0, hi=0, seed=0, stream=0, i0=0, out=None) -> np.ndarray:
    """Same values as np_fill, computed by the C generator (fast, multithreaded)."""
    lib = _load_host()
    kind = KINDS[kind] if isinstance(kind, str) else kind
    npdt = np.float64 if dtype in ("f64", np.float64) else np.float32
    if out is None:
        out = np.empty(n, dtype=npdt)
    assert out.dtype == npdt and out.flags.c_contiguous and out.size == n
    fn = lib.vnpg_fill_d if npdt is np.float64 else lib.vnpg_fill_s
    fn(out.ctypes.data, n, i0, seed, stream, kind, lo, hi)
    return out


def host_draws(n, i0, seed, stream) -> np.ndarray:
    lib = _load_host()
    out = np.empty(n, dtype=np.uint64)
    lib.vnpg_draws(out.ctypes.data, n, i0, seed, stream)
    return out


def _load_dev():
    global _dev
    if _dev is None:
        if not os.path.exists(DEV_LIB):
            raise RuntimeError(f"{DEV_LIB} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(DEV_LIB)
        for name in ("vnpg_dev_fill_d", "vnpg_dev_fill_s"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
                          ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.vnpg_dev_copy.restype = ctypes.c_int
        lib.vnpg_dev_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
        lib.vnpg_dev_read.restype = ctypes.c_int
        lib.vnpg_dev_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        _dev = lib
    return _dev


def dev_fill(t, kind="u11", lo=0, hi=0, seed=0, stream=0, i0=0):
    """Fill a contiguous CUDA (HIP) float32/float64 torch tensor in place on its current stream."""
    import torch

    lib = _load_dev()
    kind = KINDS[kind] if isinstance(kind, str) else kind
    assert t.is_cuda and t.is_contiguous()
    s = torch.cuda.current_stream(t.device).cuda_stream
    if t.dtype == torch.float64:
        rc = lib.vnpg_dev_fill_d(t.data_ptr(), t.numel(), i0, seed, stream, kind, lo, hi, s)
    elif t.dtype == torch.float32:
        rc = lib.vnpg_dev_fill_s(t.data_ptr(), t.numel(), i0, seed, stream, kind, lo, hi, s)
    else:
        raise TypeError(t.dtype)
    if rc != 0:
        raise RuntimeError(f"device fill failed: hip error {rc}")
    return t


def dev_fill_ptr(ptr, n, dtype="f64", kind="u11", lo=0, hi=0, seed=0, stream=0, i0=0, hip_stream=0):
    """Fill n elements at a raw device address (for buffers not owned by torch)."""
    lib = _load_dev()
    kind = KINDS[kind] if isinstance(kind, str) else kind
    fn = lib.vnpg_dev_fill_d if dtype in ("f64", np.float64) else lib.vnpg_dev_fill_s
    rc = fn(ptr, n, i0, seed, stream, kind, lo, hi, hip_stream)
    if rc != 0:
        raise RuntimeError(f"device fill failed: hip error {rc}")


def dev_copy(dst, src, nbytes, blocks=0, stream=0):
    rc = _load_dev().vnpg_dev_copy(dst, src, nbytes, blocks, stream)
    if rc != 0:
        raise RuntimeError(f"copy failed: {rc}")


def dev_read(src, nbytes, out, blocks, stream=0):
    rc = _load_dev().vnpg_dev_read(src, nbytes, out, blocks, stream)
    if rc != 0:
        raise RuntimeError(f"read failed: {rc}")


LOADGEN_LIB = os.path.join(_HERE, "libvnp_loadgen.so")


def run_load(server, arrival_s, reqs, copy=False):
    """Open-loop replay of requests (vnp.Request array) at arrival times arrival_s (seconds
    from start) against a vnp.Server (copy: submitted for admission by copy); returns
    (latency_s, values, status, wall_s)."""
    import paper_2509_06220_amd as vnp

    lg = ctypes.CDLL(LOADGEN_LIB)
    lg.vnpg_loadgen.restype = ctypes.c_int
    lg.vnpg_loadgen.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64] + [ctypes.c_void_p] * 6
    L = vnp.lib()
    fp = lambda f: ctypes.cast(f, ctypes.c_void_p).value  # noqa: E731
    n = len(arrival_s)
    arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
    lat = np.zeros(n)
    val = np.zeros(n)
    st = np.zeros(n, dtype=np.int32)
    wall = ctypes.c_double()
    raddr = reqs.ctypes.data if isinstance(reqs, np.ndarray) else ctypes.addressof(reqs)
    submit = L.vnp_server_submit_copy if copy else L.vnp_server_submit
    lg.vnpg_loadgen(server.handle, fp(submit), fp(L.vnp_server_wait), fp(L.vnp_server_clock_ns), n,
                    arr.ctypes.data, raddr, lat.ctypes.data, val.ctypes.data, st.ctypes.data,
                    ctypes.addressof(wall))
    return lat, val, st, wall.value


def request_array(count):
    """numpy structured array laid out like vnp_request (dtype, p, n, x, incx)."""
    import paper_2509_06220_amd as vnp

    R = vnp.Request
    dt = np.dtype({"names": ["dtype", "p", "n", "x", "incx"],
                   "formats": [np.int32, np.float64, np.int64, np.uint64, np.int64],
                   "offsets": [R.dtype.offset, R.p.offset, R.n.offset, R.x.offset, R.incx.offset],
                   "itemsize": ctypes.sizeof(R)})
    return np.zeros(count, dtype=dt)


def loop_plain(fn_name, offsets, x_ptr, esz, res_ptr, res_bytes, stream):
    """Issue one plain call per segment from native code (baseline of the batched mode)."""
    import paper_2509_06220_amd as vnp

    lg = ctypes.CDLL(LOADGEN_LIB)
    lg.vnpg_loop_plain.restype = ctypes.c_int
    lg.vnpg_loop_plain.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    fn = ctypes.cast(getattr(vnp.lib(), fn_name), ctypes.c_void_p).value
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    rc = lg.vnpg_loop_plain(fn, len(off) - 1, off.ctypes.data, x_ptr, esz, res_ptr, res_bytes, stream)
    if rc:
        raise RuntimeError(f"plain call failed with status {rc}")


def log_uniform_lengths(count, lo_log2, hi_log2, seed=0, stream=7):
    """L = floor(2^(a + (b-a) U)), U = u53 from the (seed, stream) draws: segment/request lengths."""
    ra = np_draws(count, 0, seed, stream)
    u = np.ldexp((ra >> np.uint64(11)).astype(np.float64), -53)
    return np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def recipe(name):
    return dict(RECIPES[name])


__all__ = ["np_fill", "host_fill", "dev_fill", "np_draws", "host_draws", "key", "RECIPES", "recipe",
           "log_uniform_lengths", "dev_copy", "dev_read", "dev_fill_ptr", "run_load", "request_array", "loop_plain",
           "KINDS"]
_ = math
