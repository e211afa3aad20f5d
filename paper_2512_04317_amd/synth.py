"""Seeded synthetic multi-coil k-space (stand-in for the fastMRI / SKM-TEA data).

The paper evaluates on fully sampled multi-coil k-space (Sec. 2.3); those
datasets are not available here, so every input is generated from a recipe:

* image: 10 additive ellipses on the grid u, v = (j - N/2)/(N/2) in [-1, 1)
  (field of view 2), centres ~ U(-0.6, 0.6)^2, semi-axes ~ U(0.05, 0.45),
  angle ~ U(0, pi), intensity ~ U[0.1, 1], times a smooth random phase
  exp(i * sum_{1 <= p+q <= 2} c_pq u^p v^q) with c_pq ~ U(-pi/2, pi/2);
* coil maps: S_c = exp(-|r - r_c|^2 / (2 sigma^2)) * exp(i theta_c), centres on
  a ring of radius 0.8 (0.4 FOV) at theta_c = 2 pi c / C + theta_0,
  theta_0 ~ U(0, 2 pi) per slice, sigma = 0.8 (0.4 FOV); one coil means S = 1;
* k-space: K = FFT2(image * S_c) in complex128 (no shifts), plus complex
  Gaussian noise with per-component std sigma_n / sqrt(2), sigma_n = 1e-3 max|K|
  per coil slice, then rounded to complex64.

Seeds: image of (workload, slice) from default_rng([20251204, workload, slice]);
coil map and noise of coil c from default_rng([20251204, workload, slice, c + 1]);
the ring offset theta_0 from default_rng([20251204, workload, slice, 0]).

This module only builds inputs; it holds none of the transform's arithmetic and
serves the tests, the smoke check and the benchmark alike.
"""
import numpy as np

SEED = 20251204


def _grid(N):
    ax = (np.arange(N, dtype=np.float64) - N / 2) / (N / 2)
    v, u = np.meshgrid(ax, ax, indexing="ij")   # v: row coordinate, u: column coordinate
    return u, v


def phantom(N, rng, n_ellipses=10):
    """Complex image: additive random ellipses times a smooth random phase."""
    u, v = _grid(N)
    mag = np.zeros((N, N), np.float64)
    for _ in range(n_ellipses):
        cx, cy = rng.uniform(-0.6, 0.6, size=2)
        a, b = rng.uniform(0.05, 0.45, size=2)
        th = rng.uniform(0.0, np.pi)
        val = rng.uniform(0.1, 1.0)
        c, s = np.cos(th), np.sin(th)
        xr = (u - cx) * c + (v - cy) * s
        yr = -(u - cx) * s + (v - cy) * c
        mag += val * ((xr / a) ** 2 + (yr / b) ** 2 <= 1.0)
    phase = np.zeros_like(mag)
    for p in range(3):
        for q in range(3):
            if 1 <= p + q <= 2:
                phase += rng.uniform(-np.pi / 2, np.pi / 2) * u ** p * v ** q
    return mag * np.exp(1j * phase)


def coil_map(N, c, C, theta0):
    u, v = _grid(N)
    th = 2 * np.pi * c / C + theta0
    rc = 0.8
    cx, cy = rc * np.cos(th), rc * np.sin(th)
    sigma = 0.8
    return np.exp(-((u - cx) ** 2 + (v - cy) ** 2) / (2 * sigma ** 2)) * np.exp(1j * th)


def kspace_slice(N, config, slice_idx, coils):
    """k-space of one slice: complex64 [coils, N, N]."""
    img = phantom(N, np.random.default_rng([SEED, config, slice_idx]))
    out = np.empty((coils, N, N), np.complex64)
    theta0 = np.random.default_rng([SEED, config, slice_idx, 0]).uniform(0, 2 * np.pi)
    for c in range(coils):
        rng = np.random.default_rng([SEED, config, slice_idx, c + 1])
        S = np.ones((N, N)) if coils == 1 else coil_map(N, c, coils, theta0)
        K = np.fft.fft2(img * S)
        sig = 1e-3 * np.abs(K).max()
        noise = rng.normal(0.0, sig / np.sqrt(2), size=(2, N, N))
        K = K + noise[0] + 1j * noise[1]
        out[c] = K.astype(np.complex64)
    return out


def kspace_batch(N, config, slices, coils, first_slice=0, workers=1):
    """complex64 [slices * coils, N, N]: slice-major, coil-minor.  `workers`
    threads build slices concurrently (numpy's FFT releases the GIL); the
    result does not depend on it."""
    out = np.empty((slices * coils, N, N), np.complex64)

    def one(s):
        out[s * coils:(s + 1) * coils] = kspace_slice(N, config, first_slice + s, coils)

    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(one, range(slices)))
    else:
        for s in range(slices):
            one(s)
    return out


def random_complex(shape, seed, scale=1.0, dist="normal"):
    """Plain seeded complex64 test data (normal or heavy-tailed magnitudes)."""
    rng = np.random.default_rng([SEED, 99, seed])
    if dist == "normal":
        z = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    elif dist == "lognormal":
        z = np.exp(rng.normal(0, 3, size=shape)) * np.exp(2j * np.pi * rng.uniform(size=shape))
    else:
        raise ValueError(dist)
    return (scale * z).astype(np.complex64)


# Workloads: single-coil 64^2, 8-coil 256^2 and 16-coil 512^2 k-space stacks.
# The second field of each seed names the workload.
WORKLOADS = {
    "kspace64_1x1": dict(N=64, config=1, slices=1, coils=1),
    "kspace256_32x8": dict(N=256, config=2, slices=32, coils=8),
    "kspace512_64x16": dict(N=512, config=3, slices=64, coils=16),
}
