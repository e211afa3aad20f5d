"""Python binding of libmxfft.so (the C ABI in include/mxfft.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  Tensors are torch complex64 CUDA tensors of shape [batch, n, n]
(device memory); the current torch stream is used unless one is given.
"""
import ctypes
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmxfft.so")

E4M3, E5M2, FP16, BF16, FP32, E2M3, E3M2 = 0, 1, 2, 3, 4, 5, 6
FORMATS = {"e4m3": E4M3, "e5m2": E5M2, "fp16": FP16, "bf16": BF16, "fp32": FP32, "e2m3": E2M3, "e3m2": E3M2}
NO_PRESCALE, KEEP_SCALE, NORMALIZE, FUSED_ROUNDTRIP, DEBUG_CAPTURE, QUANTIZE_OUTPUT = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
OK, EINVAL, ENOMEM, EHIP, ENONFINITE, ERANGE, EBUDGET, EBUSY, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7, -8
INT32_MIN, INT32_MAX = -(2 ** 31), 2 ** 31 - 1

# Every entry point declared in include/mxfft.h.
EXPORTS = ("mxfft_params_default", "mxfft_plan", "mxfft_plan_destroy", "mxfft_forward", "mxfft_forward_static",
           "mxfft_inverse", "mxfft_roundtrip", "mxfft_plan_last_status", "mxfft_plan_profile",
           "mxfft_plan_profile_roles",
           "mxfft_plan_kernel_times", "mxfft_plan_device_bytes", "mxfft_status_string", "mxfft_version",
           "mxfft_plan_set_tuning", "mxfft_plan_get_tuning", "mxfft_tune", "mxfft_tune_cache_lookup",
           "mxfft_batch_create", "mxfft_batch_execute", "mxfft_batch_last_status", "mxfft_batch_group_tuning",
           "mxfft_batch_destroy", "mxfft_plan_bytes", "mxfft_serve_create", "mxfft_serve_submit",
           "mxfft_serve_wait", "mxfft_serve_poll", "mxfft_serve_hold", "mxfft_serve_stats", "mxfft_serve_destroy",
           "mxfft_rss",
           "mxfft_ssim", "mxfft_plan_capture")
TUNE_FORCE = 0x1
FORWARD, INVERSE, ROUNDTRIP = 0, 1, 2


# kernel roles reported by Plan.kernel_times (bit order of mxfft_plan_profile_roles)
ROLES = ("prescale_stats", "row_pass", "column_pass", "inverse_row_pass", "inverse_column_pass", "row_redo")


class Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("format", ctypes.c_int32), ("block", ctypes.c_int32),
                ("k_min", ctypes.c_int32), ("k_max", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("target", ctypes.c_double), ("tau_pct", ctypes.c_double), ("tau_min", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("lines", ctypes.c_int32), ("fast", ctypes.c_int32), ("ms", ctypes.c_double),
                ("single", ctypes.c_int32), ("stats", ctypes.c_int32), ("chunks", ctypes.c_int32)]


class Group(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("count", ctypes.c_int32), ("offset", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("inp", ctypes.c_void_p), ("out", ctypes.c_void_p), ("k_out", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("coils", ctypes.c_int32), ("op", ctypes.c_int32), ("params", Params),
                ("ready", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("t_submit_ms", ctypes.c_double),
                ("t_start_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double)]


class ServeCounters(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "submitted", "admitted", "completed", "rejected", "queued", "in_flight", "plan_bytes", "peak_plan_bytes",
        "plans_created", "plans_evicted", "budget", "coalesced_launches", "coalesced_requests")]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


class MxfftError(RuntimeError):
    def __init__(self, status, what):
        super().__init__("%s: %s (%d)" % (what, status_string(status), status))
        self.status = status


_lib = None


def lib():
    """Load libmxfft.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmxfft.so is not built: run __graft_entry__.build() (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
        L.mxfft_params_default.restype = None
        L.mxfft_params_default.argtypes = [ctypes.POINTER(Params)]
        L.mxfft_plan.restype = i32
        L.mxfft_plan.argtypes = [ctypes.POINTER(P), i32, i32, ctypes.POINTER(Params), P]
        L.mxfft_plan_destroy.restype = i32
        L.mxfft_plan_destroy.argtypes = [P]
        for name in ("mxfft_forward", "mxfft_forward_static", "mxfft_roundtrip"):
            getattr(L, name).restype = i32
            getattr(L, name).argtypes = [P, P, P, i32, P, P]
        L.mxfft_inverse.restype = i32
        L.mxfft_inverse.argtypes = [P, P, P, i32, P, P]
        L.mxfft_plan_last_status.restype = i32
        L.mxfft_plan_last_status.argtypes = [P, P]
        L.mxfft_plan_capture.restype = i32
        L.mxfft_plan_capture.argtypes = [P, P, P, P, i32, P]
        L.mxfft_plan_profile.restype = i32
        L.mxfft_plan_profile.argtypes = [P, i32]
        L.mxfft_plan_profile_roles.restype = i32
        L.mxfft_plan_profile_roles.argtypes = [P, ctypes.c_uint32]
        L.mxfft_plan_kernel_times.restype = i32
        L.mxfft_plan_kernel_times.argtypes = [P, ctypes.POINTER(KernelTime), i32, ctypes.POINTER(i32)]
        L.mxfft_plan_device_bytes.restype = ctypes.c_uint64
        L.mxfft_plan_device_bytes.argtypes = [P]
        L.mxfft_status_string.restype = ctypes.c_char_p
        L.mxfft_status_string.argtypes = [i32]
        L.mxfft_version.restype = i32
        L.mxfft_version.argtypes = []
        TP = ctypes.POINTER(Tuning)
        for name in ("mxfft_plan_set_tuning", "mxfft_plan_get_tuning"):
            getattr(L, name).restype = i32
            getattr(L, name).argtypes = [P, TP]
        L.mxfft_tune.restype = i32
        L.mxfft_tune.argtypes = [i32, ctypes.POINTER(Params), i32, ctypes.c_char_p, u32, TP, P]
        L.mxfft_tune_cache_lookup.restype = i32
        L.mxfft_tune_cache_lookup.argtypes = [ctypes.c_char_p, ctypes.c_char_p, i32, ctypes.POINTER(Params), TP]
        L.mxfft_batch_create.restype = i32
        L.mxfft_batch_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Group), i32, ctypes.POINTER(Params),
                                         ctypes.c_char_p, P]
        L.mxfft_batch_execute.restype = i32
        L.mxfft_batch_execute.argtypes = [P, i32, P, P, P, P]
        L.mxfft_batch_last_status.restype = i32
        L.mxfft_batch_last_status.argtypes = [P, P]
        L.mxfft_batch_group_tuning.restype = i32
        L.mxfft_batch_group_tuning.argtypes = [P, i32, TP]
        L.mxfft_batch_destroy.restype = i32
        L.mxfft_batch_destroy.argtypes = [P]
        L.mxfft_ssim.restype = i32
        L.mxfft_ssim.argtypes = [P, P, i32, i32, P, P]
        L.mxfft_rss.restype = i32
        L.mxfft_rss.argtypes = [P, i32, P, P, P, i32, i32, P, P]
        L.mxfft_plan_bytes.restype = i32
        L.mxfft_plan_bytes.argtypes = [i32, i32, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_uint64)]
        L.mxfft_serve_create.restype = i32
        L.mxfft_serve_create.argtypes = [ctypes.POINTER(P), ctypes.c_uint64, i32]
        L.mxfft_serve_submit.restype = i32
        L.mxfft_serve_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        for name in ("mxfft_serve_wait", "mxfft_serve_poll"):
            getattr(L, name).restype = i32
            getattr(L, name).argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result)]
        L.mxfft_serve_stats.restype = i32
        L.mxfft_serve_stats.argtypes = [P, ctypes.POINTER(ServeCounters)]
        L.mxfft_serve_hold.restype = i32
        L.mxfft_serve_hold.argtypes = [P, i32]
        L.mxfft_serve_destroy.restype = i32
        L.mxfft_serve_destroy.argtypes = [P]
        _lib = L
    return _lib


def status_string(st):
    return lib().mxfft_status_string(int(st)).decode()


def default_params():
    p = Params()
    lib().mxfft_params_default(ctypes.byref(p))
    return p


def make_params(fmt="e4m3", block=32, target=2.0 ** 7, tau=5.0, tau_min=2.0 ** -6,
                k_min=None, k_max=None, flags=0):
    p = default_params()
    p.format = FORMATS[fmt] if isinstance(fmt, str) else int(fmt)
    p.block = int(block)
    p.target = float(target)
    p.tau_pct = float(tau)
    p.tau_min = float(tau_min)
    p.k_min = INT32_MIN if k_min is None else int(k_min)
    p.k_max = INT32_MAX if k_max is None else int(k_max)
    p.flags = int(flags)
    return p


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_slices(x, n, what):
    if not (x.is_cuda and x.dtype == torch.complex64 and x.is_contiguous()):
        raise ValueError("%s must be a contiguous complex64 CUDA tensor" % what)
    if x.dim() != 3 or x.shape[1] != n or x.shape[2] != n:
        raise ValueError("%s must have shape [batch, %d, %d]" % (what, n, n))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """A plan for n x n slices and batches of up to max_batch slices."""

    def __init__(self, n, max_batch, stream=None, **params):
        self.n = int(n)
        self.max_batch = int(max_batch)
        self.params = make_params(**params)
        h = ctypes.c_void_p()
        st = lib().mxfft_plan(ctypes.byref(h), self.n, self.max_batch, ctypes.byref(self.params), _stream(stream))
        if st != OK:
            raise MxfftError(st, "mxfft_plan")
        self.handle = h

    def _kbuf(self, batch, k, device):
        if k is None:
            k = torch.empty(batch, dtype=torch.int32, device=device)
        if not (k.is_cuda and k.dtype == torch.int32 and k.numel() >= batch and k.is_contiguous()):
            raise ValueError("k must be a contiguous int32 CUDA tensor with >= batch entries")
        return k

    def forward(self, x, out=None, k_out=None, stream=None):
        """Eq. 1 forward transform; returns (out, k) with k the prescale per slice."""
        _check_slices(x, self.n, "x")
        out = torch.empty_like(x) if out is None else out
        _check_slices(out, self.n, "out")
        k_out = self._kbuf(x.shape[0], k_out, x.device)
        st = lib().mxfft_forward(self.handle, _ptr(x), _ptr(out), x.shape[0], _ptr(k_out), _stream(stream))
        if st != OK:
            raise MxfftError(st, "mxfft_forward")
        return out, k_out

    def forward_static(self, x, out=None, k_out=None, stream=None):
        """As forward, through mxfft_forward_static: no device allocation in
        the library; its workspace is the static array shared by every such
        call on the device (batch may exceed max_batch while it fits)."""
        _check_slices(x, self.n, "x")
        if out is None or k_out is None:
            raise ValueError("forward_static needs caller-allocated out and k_out")
        _check_slices(out, self.n, "out")
        k_out = self._kbuf(x.shape[0], k_out, x.device)
        st = lib().mxfft_forward_static(self.handle, _ptr(x), _ptr(out), x.shape[0], _ptr(k_out), _stream(stream))
        if st != OK:
            raise MxfftError(st, "mxfft_forward_static")
        return out, k_out

    def inverse(self, x, out=None, k_in=None, stream=None):
        _check_slices(x, self.n, "x")
        out = torch.empty_like(x) if out is None else out
        _check_slices(out, self.n, "out")
        if k_in is not None:
            k_in = self._kbuf(x.shape[0], k_in, x.device)
        st = lib().mxfft_inverse(self.handle, _ptr(x), _ptr(out), x.shape[0], _ptr(k_in), _stream(stream))
        if st != OK:
            raise MxfftError(st, "mxfft_inverse")
        return out

    def roundtrip(self, x, out=None, k_out=None, stream=None):
        _check_slices(x, self.n, "x")
        out = torch.empty_like(x) if out is None else out
        _check_slices(out, self.n, "out")
        k_out = self._kbuf(x.shape[0], k_out, x.device)
        st = lib().mxfft_roundtrip(self.handle, _ptr(x), _ptr(out), x.shape[0], _ptr(k_out), _stream(stream))
        if st != OK:
            raise MxfftError(st, "mxfft_roundtrip")
        return out, k_out

    def rss(self, x, coils, op=FORWARD, out=None, work=None, k_out=None, stream=None):
        """Eq. 1 root-sum-of-squares image of each reconstruction (coil-minor
        slices of x) after the forward transform or the round trip of every
        coil, fused into the last column pass; returns (rss, k)."""
        _check_slices(x, self.n, "x")
        if x.shape[0] % coils:
            raise ValueError("the batch must hold whole reconstructions of %d coils" % coils)
        recon = x.shape[0] // coils
        if out is None:
            out = torch.empty((recon, self.n, self.n), dtype=torch.float32, device=x.device)
        if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.shape == (recon, self.n, self.n)):
            raise ValueError("out must be a contiguous float32 CUDA tensor [recon, n, n]")
        if work is None and (op == ROUNDTRIP or self.params.format == FP32 or not self.tuning()["fast"]):
            work = torch.empty_like(x)
        k_out = self._kbuf(x.shape[0], k_out, x.device)
        st = lib().mxfft_rss(self.handle, int(op), _ptr(x), _ptr(work), _ptr(out), recon, int(coils), _ptr(k_out),
                             _stream(stream))
        if st != OK:
            raise MxfftError(st, "mxfft_rss")
        return out, k_out

    def capture(self, batch, trace=False, stream=None):
        """DEBUG_CAPTURE plans: the column pass's MX input of the last forward
        call (its first `batch` slices): element values complex64 [batch, n, n]
        and block exponents int32 [batch, n (columns), n / (B/2) (row blocks)];
        with trace, also int32 [batch, log2 n, n / B, 3]: (E_v, k_r, E_out)
        per stage and block of row 0's row pass."""
        cb = self.params.block // 2
        dev = torch.device("cuda", torch.cuda.current_device())
        mant = torch.empty((batch, self.n, self.n), dtype=torch.complex64, device=dev)
        exps = torch.empty((batch, self.n, self.n // cb), dtype=torch.int32, device=dev)
        tr = None
        if trace:
            tr = torch.empty((batch, self.n.bit_length() - 1, self.n // (2 * cb), 3), dtype=torch.int32, device=dev)
        st = lib().mxfft_plan_capture(self.handle, _ptr(mant), _ptr(exps), _ptr(tr), int(batch), _stream(stream))
        if st != OK:
            raise MxfftError(st, "mxfft_plan_capture")
        return (mant, exps, tr) if trace else (mant, exps)

    def last_status(self, stream=None):
        return lib().mxfft_plan_last_status(self.handle, _stream(stream))

    def profile(self, enable=True, roles=None):
        """Start (resetting) or stop event timing of the kernel launches: all
        of them, or only those whose role is named in `roles`."""
        if roles is None:
            st = lib().mxfft_plan_profile(self.handle, int(bool(enable)))
        else:
            mask = 0
            for r in roles:
                mask |= 1 << ROLES.index(r)
            st = lib().mxfft_plan_profile_roles(self.handle, mask if enable else 0)
        if st != OK:
            raise MxfftError(st, "mxfft_plan_profile")

    def kernel_times(self):
        """{role: (launches, total_ms)} accumulated while profiling."""
        buf = (KernelTime * 8)()
        n = ctypes.c_int32()
        st = lib().mxfft_plan_kernel_times(self.handle, buf, 8, ctypes.byref(n))
        if st != OK:
            raise MxfftError(st, "mxfft_plan_kernel_times")
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(min(n.value, 8))}

    def device_bytes(self):
        return lib().mxfft_plan_device_bytes(self.handle)

    def tuning(self):
        t = Tuning()
        st = lib().mxfft_plan_get_tuning(self.handle, ctypes.byref(t))
        if st != OK:
            raise MxfftError(st, "mxfft_plan_get_tuning")
        return {"lines": t.lines, "fast": bool(t.fast), "single": bool(t.single), "stats": t.stats, "chunks": t.chunks}

    def set_tuning(self, lines=0, single=False, stats=0, chunks=0):
        """Line kernels with `lines` per work-group, or (n <= 128, single=True)
        the single-launch kernel; stats=1: Alg. 1 as a separate read (with
        `chunks` work-groups per slice, 0 = by batch) where the row pass could
        gather it."""
        t = Tuning(int(lines), 0, 0.0, 1 if single else 0, int(stats), int(chunks))
        st = lib().mxfft_plan_set_tuning(self.handle, ctypes.byref(t))
        if st != OK:
            raise MxfftError(st, "mxfft_plan_set_tuning")

    def close(self):
        if getattr(self, "handle", None):
            lib().mxfft_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cpath(path):
    return None if path is None else os.fsencode(path)


def tune(n, sample=16, cache=None, force=False, stream=None, **params):
    """Autotune the launch choices for n x n plans of these parameters on
    `sample` slices (see mxfft_tune): lines and the single launch on the line
    kernels, the statistics read on the register-resident passes."""
    p = make_params(**params)
    t = Tuning()
    st = lib().mxfft_tune(int(n), ctypes.byref(p), int(sample), _cpath(cache), TUNE_FORCE if force else 0,
                          ctypes.byref(t), _stream(stream))
    if st != OK:
        raise MxfftError(st, "mxfft_tune")
    return {"lines": t.lines, "fast": bool(t.fast), "ms": t.ms, "single": bool(t.single),
            "stats": t.stats, "chunks": t.chunks}


def tune_cache_lookup(cache, arch, n, **params):
    """Host-only lookup in a tuning cache file; None when there is no entry."""
    p = make_params(**params)
    t = Tuning()
    st = lib().mxfft_tune_cache_lookup(_cpath(cache), arch.encode(), int(n), ctypes.byref(p), ctypes.byref(t))
    return None if st != OK else {"lines": t.lines, "ms": t.ms, "single": bool(t.single),
            "stats": t.stats, "chunks": t.chunks}


class Batch:
    """An uneven batch: groups [(n, count), ...] laid out one after another in
    a flat complex64 pool (or with explicit offsets: (n, count, offset)),
    executed as one HIP graph launch (mxfft_batch_*)."""

    def __init__(self, groups, tune_cache=None, stream=None, **params):
        self.params = make_params(**params)
        arr = (Group * len(groups))()
        off = 0
        self.groups = []
        for i, g in enumerate(groups):
            n, count = int(g[0]), int(g[1])
            o = int(g[2]) if len(g) > 2 else off
            arr[i] = Group(n, count, o)
            self.groups.append((n, count, o))
            off = max(off, o + count * n * n)
        self.pool_elems = off
        self.slices = sum(c for _, c, _ in self.groups)
        h = ctypes.c_void_p()
        st = lib().mxfft_batch_create(ctypes.byref(h), arr, len(groups), ctypes.byref(self.params),
                                      _cpath(tune_cache), _stream(stream))
        if st != OK:
            raise MxfftError(st, "mxfft_batch_create")
        self.handle = h

    def views(self, pool):
        """The [count, n, n] view of each group inside a flat pool."""
        return [pool[o:o + c * n * n].view(c, n, n) for n, c, o in self.groups]

    def execute(self, op, x, out=None, k_out=None, stream=None):
        if not (x.is_cuda and x.dtype == torch.complex64 and x.is_contiguous() and x.numel() >= self.pool_elems):
            raise ValueError("x must be a contiguous complex64 CUDA pool of >= %d values" % self.pool_elems)
        out = torch.empty_like(x) if out is None else out
        if not (out.is_cuda and out.dtype == torch.complex64 and out.is_contiguous() and out.numel() >= self.pool_elems):
            raise ValueError("out must be a contiguous complex64 CUDA pool of >= %d values" % self.pool_elems)
        if k_out is None and op != INVERSE:
            k_out = torch.empty(self.slices, dtype=torch.int32, device=x.device)
        if k_out is not None and not (k_out.is_cuda and k_out.dtype == torch.int32 and k_out.numel() >= self.slices):
            raise ValueError("k_out must be an int32 CUDA tensor with >= %d entries" % self.slices)
        st = lib().mxfft_batch_execute(self.handle, int(op), _ptr(x), _ptr(out), _ptr(k_out), _stream(stream))
        if st != OK:
            raise MxfftError(st, "mxfft_batch_execute")
        return out, k_out

    def forward(self, x, out=None, k_out=None, stream=None):
        return self.execute(FORWARD, x, out, k_out, stream)

    def last_status(self, stream=None):
        return lib().mxfft_batch_last_status(self.handle, _stream(stream))

    def group_tuning(self, g):
        t = Tuning()
        st = lib().mxfft_batch_group_tuning(self.handle, int(g), ctypes.byref(t))
        if st != OK:
            raise MxfftError(st, "mxfft_batch_group_tuning")
        return {"lines": t.lines, "fast": bool(t.fast), "ms": t.ms, "single": bool(t.single),
            "stats": t.stats, "chunks": t.chunks}

    def close(self):
        if getattr(self, "handle", None):
            lib().mxfft_batch_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_bytes(n, max_batch, **params):
    """Device bytes a plan would hold (host-only computation)."""
    p = make_params(**params)
    b = ctypes.c_uint64()
    st = lib().mxfft_plan_bytes(int(n), int(max_batch), ctypes.byref(p), ctypes.byref(b))
    if st != OK:
        raise MxfftError(st, "mxfft_plan_bytes")
    return b.value


class Server:
    """A request server (mxfft_serve_*): submit() from any thread, wait().

    A request runs on one of the server's streams.  submit() records an event
    on the submitting stream (the current torch stream unless one is given)
    that the request waits on, so work queued there before the call, such as
    writing x, is complete first; the tensors are kept referenced until the
    ticket is answered, so the caching allocator cannot hand their memory to
    other work while the request may still use it."""

    def __init__(self, budget_bytes, slots=4):
        h = ctypes.c_void_p()
        st = lib().mxfft_serve_create(ctypes.byref(h), int(budget_bytes), int(slots))
        if st != OK:
            raise MxfftError(st, "mxfft_serve_create")
        self.handle = h
        self._held = {}
        self._held_lock = threading.Lock()

    def submit(self, x, out, k_out=None, op=FORWARD, stream=None, **params):
        """Queue one request over x = [coils, n, n]; returns its ticket.  Raises
        MxfftError (status EBUDGET when its plan alone exceeds the budget)."""
        if not (x.is_cuda and x.dtype == torch.complex64 and x.is_contiguous() and x.dim() == 3):
            raise ValueError("x must be a contiguous complex64 CUDA tensor [coils, n, n]")
        if not (out.is_cuda and out.dtype == torch.complex64 and out.is_contiguous() and out.shape == x.shape):
            raise ValueError("out must be a contiguous complex64 CUDA tensor shaped like x")
        if k_out is not None and not (k_out.is_cuda and k_out.dtype == torch.int32 and k_out.numel() >= x.shape[0]):
            raise ValueError("k_out must be an int32 CUDA tensor with >= coils entries")
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream() if stream is None else stream)
        r = Request(x.data_ptr(), out.data_ptr(), None if k_out is None else k_out.data_ptr(),
                    int(x.shape[1]), int(x.shape[0]), int(op), make_params(**params), ready.cuda_event)
        t = ctypes.c_uint64()
        with self._held_lock:
            st = lib().mxfft_serve_submit(self.handle, ctypes.byref(r), ctypes.byref(t))
            if st == OK:
                self._held[t.value] = (x, out, k_out, ready)
        if st != OK:
            raise MxfftError(st, "mxfft_serve_submit")
        return t.value

    def _release(self, ticket):
        with self._held_lock:
            self._held.pop(int(ticket), None)

    @staticmethod
    def _res(r):
        return {"status": r.status, "slot": r.slot, "t_submit_ms": r.t_submit_ms, "t_start_ms": r.t_start_ms,
                "t_done_ms": r.t_done_ms}

    def wait(self, ticket):
        r = Result()
        st = lib().mxfft_serve_wait(self.handle, int(ticket), ctypes.byref(r))
        if st != OK:
            raise MxfftError(st, "mxfft_serve_wait")
        self._release(ticket)
        return self._res(r)

    def poll(self, ticket):
        """The result, or None while the request runs."""
        r = Result()
        st = lib().mxfft_serve_poll(self.handle, int(ticket), ctypes.byref(r))
        if st == EBUSY:
            return None
        if st != OK:
            raise MxfftError(st, "mxfft_serve_poll")
        self._release(ticket)
        return self._res(r)

    def hold(self, on=True):
        """Pause (on) or resume admissions; queued requests wait meanwhile."""
        st = lib().mxfft_serve_hold(self.handle, 1 if on else 0)
        if st != OK:
            raise MxfftError(st, "mxfft_serve_hold")

    def stats(self):
        c = ServeCounters()
        st = lib().mxfft_serve_stats(self.handle, ctypes.byref(c))
        if st != OK:
            raise MxfftError(st, "mxfft_serve_stats")
        return {name: getattr(c, name) for name, _ in ServeCounters._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().mxfft_serve_destroy(self.handle)   # finishes every request first
            self.handle = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ssim(x, ref, stream=None):
    """Mean SSIM of each image of x against ref (float32 CUDA [count, n, n]);
    returns a float64 CUDA tensor [count] (mxfft_ssim)."""
    for t, what in ((x, "x"), (ref, "ref")):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 3):
            raise ValueError("%s must be a contiguous float32 CUDA tensor [count, n, n]" % what)
    if x.shape != ref.shape:
        raise ValueError("x and ref must have the same shape")
    out = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    st = lib().mxfft_ssim(_ptr(x), _ptr(ref), int(x.shape[-1]), int(x.shape[0]), _ptr(out), _stream(stream))
    if st != OK:
        raise MxfftError(st, "mxfft_ssim")
    return out
