"""Python binding of libmxfft.so (the C ABI in include/mxfft.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  Tensors are torch complex64 CUDA tensors of shape [batch, n, n]
(device memory); the current torch stream is used unless one is given.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmxfft.so")

E4M3, E5M2, FP16, BF16, FP32 = 0, 1, 2, 3, 4
FORMATS = {"e4m3": E4M3, "e5m2": E5M2, "fp16": FP16, "bf16": BF16, "fp32": FP32}
NO_PRESCALE, KEEP_SCALE, NORMALIZE = 0x1, 0x2, 0x4
OK, EINVAL, ENOMEM, EHIP, ENONFINITE, ERANGE, EBUDGET, EBUSY, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7, -8
INT32_MIN, INT32_MAX = -(2 ** 31), 2 ** 31 - 1

# Every entry point declared in include/mxfft.h.
EXPORTS = ("mxfft_params_default", "mxfft_plan", "mxfft_plan_destroy", "mxfft_forward",
           "mxfft_inverse", "mxfft_roundtrip", "mxfft_plan_last_status", "mxfft_plan_profile",
           "mxfft_plan_profile_roles",
           "mxfft_plan_kernel_times", "mxfft_plan_device_bytes", "mxfft_status_string", "mxfft_version")


# kernel roles reported by Plan.kernel_times (bit order of mxfft_plan_profile_roles)
ROLES = ("prescale_stats", "row_pass", "column_pass", "inverse_row_pass", "inverse_column_pass", "row_redo")


class Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("format", ctypes.c_int32), ("block", ctypes.c_int32),
                ("k_min", ctypes.c_int32), ("k_max", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("target", ctypes.c_double), ("tau_pct", ctypes.c_double), ("tau_min", ctypes.c_double)]


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
        for name in ("mxfft_forward", "mxfft_roundtrip"):
            getattr(L, name).restype = i32
            getattr(L, name).argtypes = [P, P, P, i32, P, P]
        L.mxfft_inverse.restype = i32
        L.mxfft_inverse.argtypes = [P, P, P, i32, P, P]
        L.mxfft_plan_last_status.restype = i32
        L.mxfft_plan_last_status.argtypes = [P, P]
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

    def close(self):
        if getattr(self, "handle", None):
            lib().mxfft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
