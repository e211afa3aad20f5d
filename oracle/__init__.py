"""CPU oracle for the MX-scaled mixed-precision FFT (test infrastructure only).

Plain, slow, obviously correct CPU implementation (C, in ``mxfft_oracle.c``) of
the paper's method: the global power-of-two prescale (Alg. 1), the MX-scaled
complex butterfly (Alg. 2), iterative radix-2 passes with stage-wise MX
re-encoding, and the 2D forward / inverse / round-trip transforms of Eq. 1.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the two
share no code.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mxfft_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libmxfft_oracle.so")

E4M3, E5M2, FP16, BF16, E6M23, E2M3, E3M2 = 0, 1, 2, 3, 4, 5, 6
MODE_MX, MODE_FP32, MODE_FP16, MODE_BF16 = 0, 1, 2, 3
OK, EINVAL, ENONFINITE, ERANGE = 0, -1, -4, -5
NO_PRESCALE, KEEP_SCALE, NORMALIZE, FUSED_RT, QUANTIZE_OUT = 1, 2, 4, 8, 32
FORWARD, INVERSE, ROUNDTRIP = 0, 1, 2
INT32_MIN = -(2 ** 31)
INT32_MAX = 2 ** 31 - 1

FMT_NAMES = {"e4m3": E4M3, "e5m2": E5M2, "fp16": FP16, "bf16": BF16, "e6m23": E6M23, "e2m3": E2M3, "e3m2": E3M2}


def build(force=True):
    """Compile the oracle with gcc (no fused multiply-add, IEEE semantics)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i, d, lg, u = ctypes.c_int, ctypes.c_double, ctypes.c_long, ctypes.c_uint
        L.orc_quantize.restype = d
        L.orc_quantize.argtypes = [i, d]
        L.orc_quantize_array.restype = None
        L.orc_quantize_array.argtypes = [i, P, P, lg]
        L.orc_encode_code.restype = i
        L.orc_encode_code.argtypes = [i, d]
        L.orc_decode_code.restype = d
        L.orc_decode_code.argtypes = [i, i]
        L.orc_mx_encode.restype = i
        L.orc_mx_encode.argtypes = [i, P, i, P]
        L.orc_twiddle64.restype = None
        L.orc_twiddle64.argtypes = [i, i, i, P, P]
        L.orc_mx_butterfly.restype = None
        L.orc_mx_butterfly.argtypes = [i, i, P, P, P, i, P, P, P]
        L.orc_prescale.restype = i
        L.orc_prescale.argtypes = [P, lg, d, d, d, i, i, P]
        L.orc_transform.restype = i
        L.orc_transform.argtypes = [i, i, i, i, i, lg, P, P, P, i, d, d, d, i, i, u, i]
        L.orc_pass_lines.restype = i
        L.orc_pass_lines.argtypes = [i, i, i, i, i, lg, P, P]
        L.orc_column_encode.restype = i
        L.orc_column_encode.argtypes = [i, i, i, P, P, P]
        L.orc_fft2_f64.restype = i
        L.orc_fft2_f64.argtypes = [i, lg, i, P]
        L.orc_fft1_f64.restype = i
        L.orc_fft1_f64.argtypes = [i, lg, i, P]
        L.orc_fmt_info.restype = i
        L.orc_fmt_info.argtypes = [i, P, P, P, P, P]
        L.orc_rss.restype = i
        L.orc_rss.argtypes = [P, lg, i, lg, P]
        L.orc_ssim.restype = i
        L.orc_ssim.argtypes = [P, P, i, d, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def fmt_info(f):
    vals = [ctypes.c_int() for _ in range(4)] + [ctypes.c_double()]
    lib().orc_fmt_info(f, *[ctypes.byref(v) for v in vals])
    e, m, emin, emax, mx = (v.value for v in vals)
    return {"ebits": e, "mbits": m, "emin": emin, "emax": emax, "maxval": mx}


def quantize(f, x):
    """Q_F applied elementwise (round to nearest even, saturate or overflow)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    q = np.empty_like(x)
    lib().orc_quantize_array(f, _ptr(x), _ptr(q), x.size)
    return q


def encode_code(f, q):
    return lib().orc_encode_code(f, float(q))


def decode_code(f, c):
    return lib().orc_decode_code(f, int(c))


def mx_encode(f, vals):
    """EncodeBlockMX + MantissasBlock: returns (E, element values)."""
    v = np.ascontiguousarray(vals, dtype=np.float64)
    m = np.empty_like(v)
    E = lib().orc_mx_encode(f, _ptr(v), v.size, _ptr(m))
    return E, m


def twiddle64(j, m, inverse=False):
    wr, wi = ctypes.c_double(), ctypes.c_double()
    lib().orc_twiddle64(j, m, int(inverse), ctypes.byref(wr), ctypes.byref(wi))
    return complex(wr.value, wi.value)


def mx_butterfly(f, u, v, x, Ew):
    """Alg. 2 on one block. u, v: complex64 arrays (cb values); x: complex128
    twiddle element values; Ew: twiddle block exponent. Returns (y0, y1, (Ev, kr, Eout))."""
    u = np.ascontiguousarray(u, dtype=np.complex64)
    v = np.ascontiguousarray(v, dtype=np.complex64)
    xx = np.ascontiguousarray(x, dtype=np.complex128)
    cb = u.size
    y0 = np.empty(cb, np.complex64)
    y1 = np.empty(cb, np.complex64)
    tr = np.zeros(3, np.int32)
    lib().orc_mx_butterfly(f, cb, _ptr(u), _ptr(v), _ptr(xx), int(Ew), _ptr(y0), _ptr(y1), _ptr(tr))
    return y0, y1, tuple(int(t) for t in tr)


def prescale(x, target=2.0 ** 7, tau=5.0, tau_min=2.0 ** -6, k_min=INT32_MIN, k_max=INT32_MAX):
    """Alg. 1 on one slice (complex64 array of any shape). Returns (status, k)."""
    x = np.ascontiguousarray(x, dtype=np.complex64)
    k = ctypes.c_int32()
    st = lib().orc_prescale(_ptr(x), x.size, target, tau, tau_min, k_min, k_max, ctypes.byref(k))
    return st, k.value


def transform(x, op=FORWARD, mode=MODE_MX, fmt=E4M3, B=32, kp=None, target=2.0 ** 7, tau=5.0,
              tau_min=2.0 ** -6, k_min=INT32_MIN, k_max=INT32_MAX, flags=0, nthreads=1):
    """2D transform of complex64 slices [batch, N, N] (or [N, N]).

    op: FORWARD, INVERSE or ROUNDTRIP.  kp: for INVERSE, per-slice exponents
    already applied to the input (the round-trip hand-off); otherwise None.
    Returns (status, out complex64, kp int32[batch])."""
    x = np.asarray(x)
    squeeze = x.ndim == 2
    x = np.ascontiguousarray(x.reshape((-1,) + x.shape[-2:]), dtype=np.complex64)
    batch, N = x.shape[0], x.shape[-1]
    out = np.empty_like(x)
    if kp is None:
        k = np.zeros(batch, np.int32)
        given = 0
    else:
        k = np.ascontiguousarray(np.broadcast_to(np.asarray(kp, np.int32), (batch,)))
        given = 1
    st = lib().orc_transform(op, mode, fmt, B, N, batch, _ptr(x), _ptr(out), _ptr(k), given,
                             target, tau, tau_min, k_min, k_max, flags, nthreads)
    if squeeze:
        out = out[0]
    return st, out, k


def pass_lines(a, mode=MODE_MX, fmt=E4M3, B=32, inverse=False, trace=False):
    """One 1D pass over each row of a [lines, N] complex64 array. With trace,
    also returns int32[L, N/B, 3] = (Ev, kr, Eout) per stage and block of row 0."""
    a = np.ascontiguousarray(a, dtype=np.complex64).copy()
    lines, N = a.reshape(-1, a.shape[-1]).shape
    L = N.bit_length() - 1
    tr = np.zeros((L, max(N // B, 1), 3), np.int32) if trace else None
    st = lib().orc_pass_lines(mode, fmt, B, N, int(inverse), lines, _ptr(a), _ptr(tr) if trace else None)
    assert st == OK, st
    return (a, tr) if trace else a


def column_encode(a, fmt=E4M3, B=32):
    """MX encode of every column's pass input (blocks of B/2 rows): returns
    (element values complex128 [N, N], exponents int32 [N cols, N/(B/2)])."""
    a = np.ascontiguousarray(a, dtype=np.complex64)
    N = a.shape[-1]
    mant = np.empty((N, N), np.complex128)
    E = np.empty((N, N // (B // 2)), np.int32)
    st = lib().orc_column_encode(fmt, B, N, _ptr(a), _ptr(mant), _ptr(E))
    assert st == OK, st
    return mant, E


def fft2_f64(x, inverse=False):
    """Unnormalised radix-2 2D FFT in FP64 (rows then columns)."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    N = a.shape[-1]
    batch = a.size // (N * N)
    assert lib().orc_fft2_f64(N, batch, int(inverse), _ptr(a)) == OK
    return a


def fft1_f64(x, inverse=False):
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    N = a.shape[-1]
    assert lib().orc_fft1_f64(N, a.size // N, int(inverse), _ptr(a)) == OK
    return a


def rss(T, coils):
    """Eq. 1 root-sum-of-squares over coils: T complex64 [recon * coils, n, n]
    (coil-minor) -> float32 [recon, n, n] (FP32, coils summed in order)."""
    a = np.ascontiguousarray(T, dtype=np.complex64)
    n = a.shape[-1]
    recon = a.size // (coils * n * n)
    out = np.empty((recon, n, n), np.float32)
    assert lib().orc_rss(_ptr(a), recon, int(coils), n * n, _ptr(out)) == OK
    return out


def ssim(x, y, L=None):
    """Mean SSIM of image x against reference y (Wang et al. 2004 form;
    L defaults to the reference's maximum)."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    b = np.ascontiguousarray(y, dtype=np.float32)
    L = float(b.max()) if L is None else float(L)
    out = ctypes.c_double()
    st = lib().orc_ssim(_ptr(a), _ptr(b), a.shape[-1], L, ctypes.byref(out))
    assert st == OK, st
    return out.value
