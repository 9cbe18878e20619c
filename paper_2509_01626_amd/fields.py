"""Seeded synthetic scientific fields (inputs only; no compressor arithmetic).

The paper evaluates on simulation outputs (cosmology, accelerator physics,
plasma and turbulence; Table 2) that are not available here. These generators
produce fields with the same shapes and comparable structure:

* ``bumps``: a sum of random 3-D Gaussian bumps plus small white noise (smooth,
  localized features);
* ``spectral``: an isotropic power-law field with random phases,
  P(|k|) ~ |k|^-alpha, normalized to zero mean and unit variance
  (turbulence-like; alpha = 5/3);
* ``grf``: a Gaussian random field (filtered white noise, random amplitudes)
  with P(k) ~ k^-alpha, unit variance;
* ``lognormal``: exp of a unit-variance Gaussian random field (a density-like
  field with a heavy upper tail).

Every generator is deterministic in its seed (numpy PCG64), computes in
float64 and returns C-ordered float32 of shape (nz, ny, nx).
"""
import numpy as np

try:
    import scipy.fft as _fft

    def _rfftn(a):
        return _fft.rfftn(a, workers=-1)

    def _irfftn(a, s):
        return _fft.irfftn(a, s=s, workers=-1)
except ImportError:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)


def bumps(dims, seed, n_bumps=32, sigma=(4.0, 16.0), noise=1e-3):
    """Sum of ``n_bumps`` Gaussian bumps: centers uniform in the box, widths
    uniform in ``sigma`` (voxels), amplitudes N(0,1); plus N(0, noise^2)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = dims
    c = rng.uniform(0, 1, size=(n_bumps, 3)) * np.array([nz, ny, nx], dtype=np.float64)
    sg = rng.uniform(sigma[0], sigma[1], size=n_bumps)
    amp = rng.standard_normal(n_bumps)
    z = np.arange(nz, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    x = np.arange(nx, dtype=np.float64)
    out = np.zeros(dims, dtype=np.float64)
    for i in range(n_bumps):
        k = -0.5 / (sg[i] * sg[i])
        gz = np.exp(k * (z - c[i, 0]) ** 2)
        gy = np.exp(k * (y - c[i, 1]) ** 2)
        gx = np.exp(k * (x - c[i, 2]) ** 2)
        out += amp[i] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    out += noise * rng.standard_normal(dims)
    return np.ascontiguousarray(out, dtype=np.float32)


def _kmag(dims):
    nz, ny, nx = dims
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.rfftfreq(nx) * nx
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    return np.sqrt(k2)


def _power_filter(dims, W, alpha, random_phase):
    k = _kmag(dims)
    with np.errstate(divide="ignore"):
        amp = np.where(k > 0, k ** (-alpha / 2.0), 0.0)
    if random_phase:
        mag = np.abs(W)
        W = np.where(mag > 0, W / np.where(mag > 0, mag, 1.0), 0.0)
    W = W * amp
    W[0, 0, 0] = 0.0
    return W


def _normalize(f):
    f = f - f.mean()
    sd = f.std()
    if sd > 0:
        f = f / sd
    return f


def spectral(dims, alpha=5.0 / 3.0, seed=0):
    """Random-phase field with isotropic power spectrum P(|k|) ~ |k|^-alpha
    (integer wavenumbers, zero mode removed), zero mean, unit variance."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(dims)
    W = _power_filter(dims, _rfftn(white), alpha, random_phase=True)
    f = _irfftn(W, dims)
    return np.ascontiguousarray(_normalize(f), dtype=np.float32)


def grf(dims, alpha, seed=0):
    """Gaussian random field: white noise filtered to P(k) ~ k^-alpha, unit
    variance."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(dims)
    W = _power_filter(dims, _rfftn(white), alpha, random_phase=False)
    f = _irfftn(W, dims)
    return np.ascontiguousarray(_normalize(f), dtype=np.float32)


def lognormal(dims, alpha=2.0, seed=0):
    """Density-like field exp(G), G a unit-variance Gaussian random field with
    P(k) ~ k^-alpha."""
    g = grf(dims, alpha, seed).astype(np.float64)
    return np.ascontiguousarray(np.exp(g), dtype=np.float32)


def batch_fields(n_fields=256, lo=32, hi=256, seed=1000):
    """Descriptors of a batch of uneven fields: dims per axis uniform in
    [lo, hi], even index -> bumps, odd -> k^-5/3 spectral, relative error bound
    log-uniform in [1e-4, 1e-2]. Returns a list of (kind, dims, seed, eb)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_fields):
        dims = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        eb = float(10 ** rng.uniform(-4, -2))
        out.append(("bumps" if i % 2 == 0 else "spectral", dims, seed + i, eb))
    return out


def make(kind, dims, seed):
    if kind == "bumps":
        return bumps(dims, seed)
    if kind == "spectral":
        return spectral(dims, 5.0 / 3.0, seed)
    raise ValueError(kind)
