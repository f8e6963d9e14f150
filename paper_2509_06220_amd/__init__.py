"""vnp: recursive hypot-based vector norms on AMD MI355X (gfx950).

Thin ctypes binding over the C ABI in ``include/vnp.h`` (``libvnp.so``, built in-tree by
``paper_2509_06220_amd/build.py``).  Only argument marshalling happens here: torch
supplies device memory and the current HIP stream; every step of the computation runs
in the library's kernels.  If the library is missing the import of any entry point
fails loudly -- there is no fallback.

Method: Novakovic, "Recursive vectorized computation of the vector p-norm"
(arXiv 2509.06220): xNRMF (Sect. 1, 3) and xNRMP (Sect. 4).
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvnp.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "vnp.h")

F64, F32 = 0, 1
EAGAIN, ENOTFOUND, EPENDING, ECANCELED, ENOMEM = 100000, 100001, 100002, 100003, 100004


class VnpError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed with status {code}")
        self.code = code


_lib = None


def lib():
    """The loaded libvnp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no non-HIP implementation)")
        L = ctypes.CDLL(LIB_PATH)
        i64, vp, d, f, i = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_float, ctypes.c_int
        sig = {
            "vnp_dnrmf": [i64, vp, i64, vp, vp],
            "vnp_snrmf": [i64, vp, i64, vp, vp],
            "vnp_dnrmf_noalloc": [i64, vp, i64, vp, vp],
            "vnp_dnrmp": [i64, vp, i64, d, vp, vp],
            "vnp_snrmp": [i64, vp, i64, f, vp, vp],
            "vnp_dnrmf_batched": [i64, vp, i64, vp, vp, vp],
            "vnp_snrmf_batched": [i64, vp, i64, vp, vp, vp],
            "vnp_dnrmp_batched": [i64, vp, i64, vp, d, vp, vp],
            "vnp_snrmp_batched": [i64, vp, i64, vp, f, vp, vp],
            "vnp_plan_create": [vp, vp, vp],
            "vnp_plan_exec": [vp, vp],
            "vnp_plan_destroy": [vp],
            "vnp_plan_info": [vp, vp, vp, vp],
            "vnp_autotune_cache_clear": [],
            "vnp_dnrmf_cols": [i64, i64, vp, i64, vp, vp],
            "vnp_snrmf_cols": [i64, i64, vp, i64, vp, vp],
            "vnp_dschatten": [i64, i64, vp, i64, d, vp, vp],
            "vnp_sschatten": [i64, i64, vp, i64, f, vp, vp],
            "vnp_dznrmf": [i64, vp, i64, vp, vp],
            "vnp_scnrmf": [i64, vp, i64, vp, vp],
            "vnp_dnrmf_mat": [i64, i64, vp, i64, vp, vp],
            "vnp_snrmf_mat": [i64, i64, vp, i64, vp, vp],
            "vnp_dnrmp_mat": [i64, i64, vp, i64, d, vp, vp],
            "vnp_snrmp_mat": [i64, i64, vp, i64, f, vp, vp],
            "vnp_set_launch_shape": [i, i],
            "vnp_finalize": [],
            "vnp_server_create": [vp, vp],
            "vnp_server_destroy": [vp],
            "vnp_server_alloc": [vp, i64, vp],
            "vnp_server_free": [vp, vp],
            "vnp_server_submit": [vp, vp, vp],
            "vnp_server_submit_copy": [vp, vp, vp],
            "vnp_server_poll": [vp, ctypes.c_uint64, vp],
            "vnp_server_wait": [vp, ctypes.c_uint64, i64, vp],
            "vnp_server_get_stats": [vp, vp],
        }
        for name, args in sig.items():
            if hasattr(L, name):
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
        L.vnp_version.restype = ctypes.c_char_p
        L.vnp_version.argtypes = []
        L.vnp_tree_id.restype = ctypes.c_uint32
        L.vnp_tree_id.argtypes = [ctypes.c_int]
        L.vnp_tile_elems.restype = ctypes.c_int64
        L.vnp_tile_elems.argtypes = [ctypes.c_int]
        L.vnp_server_clock_ns.restype = ctypes.c_int64
        L.vnp_server_clock_ns.argtypes = []
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/vnp*.h."""
    names = []
    inc = os.path.dirname(HEADER)
    for fn in sorted(os.listdir(inc)):
        if fn.startswith("vnp") and fn.endswith(".h"):
            with open(os.path.join(inc, fn)) as f:
                txt = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(vnp_[a-z0-9_]+)\s*\(", txt, re.M)
    return names


def _check(name, rc):
    if rc != 0:
        raise VnpError(name, rc)


def _stream(t, stream):
    import torch

    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return torch.cuda.current_stream(t.device).cuda_stream


def _prep_vector(x, n, incx):
    import torch

    if not x.is_cuda:
        raise ValueError("x must be a device tensor")
    if x.dtype not in (torch.float64, torch.float32):
        raise TypeError(f"unsupported dtype {x.dtype}")
    if not x.is_contiguous():
        raise ValueError("pass the underlying contiguous storage and use incx for strides")
    if incx == 0:
        raise ValueError("incx must be nonzero")
    if n is None:
        n = (x.numel() + abs(incx) - 1) // abs(incx)
    if n > 0 and (n - 1) * abs(incx) >= x.numel():
        raise ValueError("n and incx reach past the end of x")
    return n


def nrmf(x, n=None, incx=1, out=None, stream=None):
    """Frobenius norm of the n elements x[0], x[incx], ... (BLAS stride rules)."""
    import torch

    n = _prep_vector(x, n, incx)
    if out is None:
        out = torch.empty((), dtype=x.dtype, device=x.device)
    fn = "vnp_dnrmf" if x.dtype == torch.float64 else "vnp_snrmf"
    _check(fn, getattr(lib(), fn)(n, x.data_ptr(), incx, out.data_ptr(), _stream(x, stream)))
    return out


def nrmp(x, p, n=None, incx=1, out=None, stream=None):
    """p-norm (p > 0; p = inf allowed) of the n elements x[0], x[incx], ..."""
    import torch

    n = _prep_vector(x, n, incx)
    if out is None:
        out = torch.empty((), dtype=x.dtype, device=x.device)
    fn = "vnp_dnrmp" if x.dtype == torch.float64 else "vnp_snrmp"
    _check(fn, getattr(lib(), fn)(n, x.data_ptr(), incx, float(p), out.data_ptr(), _stream(x, stream)))
    return out


def nrm_batched(x, offsets, p=2.0, out=None, stream=None):
    """Norms of the segments x[offsets[s]:offsets[s+1]] in one launch (offsets: device int64)."""
    import torch

    nseg = offsets.numel() - 1
    if out is None:
        out = torch.empty(max(nseg, 0), dtype=x.dtype, device=x.device)
    if offsets.dtype != torch.int64 or not offsets.is_cuda:
        raise TypeError("offsets must be a device int64 tensor")
    if not x.is_contiguous():
        raise ValueError("x must be contiguous")
    d = x.dtype == torch.float64
    s = _stream(x, stream)
    if p == 2.0:
        fn = "vnp_dnrmf_batched" if d else "vnp_snrmf_batched"
        rc = getattr(lib(), fn)(nseg, offsets.data_ptr(), x.numel(), x.data_ptr(), out.data_ptr(), s)
    else:
        fn = "vnp_dnrmp_batched" if d else "vnp_snrmp_batched"
        rc = getattr(lib(), fn)(nseg, offsets.data_ptr(), x.numel(), x.data_ptr(), float(p), out.data_ptr(), s)
    _check(fn, rc)
    return out


class _PlanDesc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("p", ctypes.c_double), ("nseg", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("h_offsets", ctypes.c_void_p), ("n_total", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("res", ctypes.c_void_p), ("autotune", ctypes.c_int)]


class Plan:
    """A batched workload captured once (autotuned shape, HIP graph) and replayed by run().

    autotune: 0 default shape; 1 (or True) the cached choice for this device, dtype, node
    kind, size class, alignment and tree id, else time the candidates and cache the choice;
    2 time and replace the cached choice (see vnp_autotune_cache_clear in vnp.h).
    The tensors passed here must stay alive (and keep their sizes) while the plan exists;
    their contents may change between runs."""

    def __init__(self, x, offsets, out=None, p=2.0, h_offsets=None, autotune=True, stream=None):
        import numpy as np
        import torch

        self._keep = [x, offsets]
        nseg = offsets.numel() - 1
        if out is None:
            out = torch.empty(max(nseg, 0), dtype=x.dtype, device=x.device)
        self.out = out
        self._keep.append(out)
        hoff = None
        if h_offsets is not None:
            hoff = np.ascontiguousarray(np.asarray(h_offsets, dtype=np.int64))
            self._keep.append(hoff)
        desc = _PlanDesc(F64 if x.dtype == torch.float64 else F32, float(p), nseg, offsets.data_ptr(),
                         hoff.ctypes.data if hoff is not None else None, x.numel(), x.data_ptr(), out.data_ptr(),
                         int(autotune))
        self._h = ctypes.c_void_p()
        _check("vnp_plan_create", lib().vnp_plan_create(ctypes.byref(self._h), ctypes.byref(desc),
                                                        _stream(x, stream)))
        self._x = x

    def run(self, stream=None):
        _check("vnp_plan_exec", lib().vnp_plan_exec(self._h, _stream(self._x, stream)))
        return self.out

    def info(self):
        b, w, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check("vnp_plan_info", lib().vnp_plan_info(self._h, ctypes.byref(b), ctypes.byref(w), ctypes.byref(t)))
        return {"blocks": b.value, "waves_per_block": w.value, "tiles_per_item": t.value}

    def close(self):
        if self._h:
            lib().vnp_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 -- interpreter shutdown
            pass


def nrmf_cols(A, m, ncols, lda, out=None, stream=None):
    """Column norms of the column-major m x ncols matrix stored in A with leading dimension lda."""
    import torch

    if out is None:
        out = torch.empty(ncols, dtype=A.dtype, device=A.device)
    fn = "vnp_dnrmf_cols" if A.dtype == torch.float64 else "vnp_snrmf_cols"
    _check(fn, getattr(lib(), fn)(m, ncols, A.data_ptr(), lda, out.data_ptr(), _stream(A, stream)))
    return out


def schatten(A, m, n, lda, p, out=None, stream=None):
    """Schatten p-norm of the column-major m x n matrix stored in A with leading dimension lda."""
    import torch

    if out is None:
        out = torch.empty((), dtype=A.dtype, device=A.device)
    fn = "vnp_dschatten" if A.dtype == torch.float64 else "vnp_sschatten"
    _check(fn, getattr(lib(), fn)(m, n, A.data_ptr(), lda, float(p), out.data_ptr(), _stream(A, stream)))
    return out


def nrmf_complex(z, n=None, incz=1, out=None, stream=None):
    """Frobenius norm of a complex vector (torch complex128 / complex64 tensor, or its real
    view as float64 / float32 pairs) of n elements with stride incz."""
    import torch

    if z.is_complex():
        z = torch.view_as_real(z)
    if not z.is_contiguous():
        raise ValueError("the storage must be contiguous (use incz for strides)")
    m = z.numel() // 2
    if n is None:
        n = (m + abs(incz) - 1) // abs(incz) if m else 0
    if n > 0 and (n - 1) * abs(incz) + 1 > m:
        raise ValueError("n and incz reach past the end of z")
    d = z.dtype == torch.float64
    if out is None:
        out = torch.empty((), dtype=z.dtype, device=z.device)
    fn = "vnp_dznrmf" if d else "vnp_scnrmf"
    _check(fn, getattr(lib(), fn)(n, z.data_ptr(), incz, out.data_ptr(), _stream(z, stream)))
    return out


def nrm_mat(A, m, ncols, lda, p=2.0, out=None, stream=None):
    """Frobenius (p = 2) or entrywise p-norm of the column-major m x ncols array stored in A
    with leading dimension lda (one value, a 0-d tensor)."""
    import torch

    if out is None:
        out = torch.empty((), dtype=A.dtype, device=A.device)
    d = A.dtype == torch.float64
    s = _stream(A, stream)
    if p == 2.0:
        fn = "vnp_dnrmf_mat" if d else "vnp_snrmf_mat"
        rc = getattr(lib(), fn)(m, ncols, A.data_ptr(), lda, out.data_ptr(), s)
    else:
        fn = "vnp_dnrmp_mat" if d else "vnp_snrmp_mat"
        rc = getattr(lib(), fn)(m, ncols, A.data_ptr(), lda, float(p), out.data_ptr(), s)
    _check(fn, rc)
    return out


class ServerConfig(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_int64), ("max_batch", ctypes.c_int), ("streams", ctypes.c_int),
                ("max_wait_us", ctypes.c_int), ("inject_failure_every", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("p", ctypes.c_double), ("n", ctypes.c_int64), ("x", ctypes.c_void_p),
                ("incx", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("status", ctypes.c_int), ("t_submit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "rejected", "batches", "launches",
                                              "failed_batches", "max_batch_seen", "pool_free_bytes", "pool_bytes",
                                              "pending", "in_flight", "host_launch_ns", "batch_ns",
                                              "batch_ns_max", "cancelled", "admission_waits",
                                              "admission_wait_ns", "admission_wait_ns_max")]


class Server:
    """Continuous-batching request server (include/vnp_server.h)."""

    def __init__(self, pool_bytes=1 << 30, max_batch=1024, streams=4, max_wait_us=0, inject_failure_every=0):
        self.cfg = ServerConfig(pool_bytes, max_batch, streams, max_wait_us, inject_failure_every)
        self._h = ctypes.c_void_p()
        _check("vnp_server_create", lib().vnp_server_create(ctypes.byref(self._h), ctypes.byref(self.cfg)))

    @property
    def handle(self):
        return self._h.value

    def alloc(self, nbytes):
        """Device pointer from the pool, or None when the pool is full (back-pressure)."""
        p = ctypes.c_void_p()
        rc = lib().vnp_server_alloc(self._h, int(nbytes), ctypes.byref(p))
        if rc == EAGAIN:
            return None
        _check("vnp_server_alloc", rc)
        return p.value

    def free(self, ptr):
        _check("vnp_server_free", lib().vnp_server_free(self._h, ctypes.c_void_p(ptr)))

    def submit(self, ptr, n, dtype=F64, p=2.0, incx=1, copy=False):
        """Queue a request on the payload at ptr; copy=True: the server copies the payload
        into its pool when it admits the request (vnp_server_submit_copy)."""
        req = Request(dtype, float(p), int(n), ptr, int(incx))
        t = ctypes.c_uint64()
        fn = "vnp_server_submit_copy" if copy else "vnp_server_submit"
        _check(fn, getattr(lib(), fn)(self._h, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def wait(self, ticket, timeout_us=-1):
        r = Result()
        rc = lib().vnp_server_wait(self._h, ticket, int(timeout_us), ctypes.byref(r))
        if rc == EPENDING:
            return None
        _check("vnp_server_wait", rc)
        return r

    def poll(self, ticket):
        r = Result()
        rc = lib().vnp_server_poll(self._h, ticket, ctypes.byref(r))
        if rc == EPENDING:
            return None
        _check("vnp_server_poll", rc)
        return r

    def stats(self):
        s = ServerStats()
        _check("vnp_server_get_stats", lib().vnp_server_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib().vnp_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 -- interpreter shutdown
            pass


def server_clock_ns():
    return lib().vnp_server_clock_ns()


def set_launch_shape(waves_per_block=0, tiles_per_wave=0):
    """Force a launch shape (tests / tuning); (0, 0) restores the automatic choice."""
    _check("vnp_set_launch_shape", lib().vnp_set_launch_shape(waves_per_block, tiles_per_wave))


def tree_id(dtype=F64):
    return lib().vnp_tree_id(dtype)


def autotune_cache_clear():
    """Drop the process's autotune records (a VNP_AUTOTUNE_CACHE file is read again)."""
    _check("vnp_autotune_cache_clear", lib().vnp_autotune_cache_clear())


def tile_elems(dtype=F64):
    return lib().vnp_tile_elems(dtype)


def version():
    return lib().vnp_version().decode()


def finalize():
    _check("vnp_finalize", lib().vnp_finalize())
