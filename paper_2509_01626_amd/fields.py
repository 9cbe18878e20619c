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


# ---- device-side generators (large benchmark inputs) ------------------------------
# The same recipes computed with torch on a GPU (float64, then float32), seeded
# with torch's Philox generator: realizations differ from the numpy versions
# above, statistics do not. Used where host generation of many or very large
# fields would dominate a benchmark run; a field's values are copied to the host
# whenever the CPU oracle has to check it.

def _tgen(seed, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def bumps_t(dims, seed, device, n_bumps=32, sigma=(4.0, 16.0), noise=1e-3):
    import torch
    g = _tgen(seed, device)
    f64 = torch.float64
    ext = torch.tensor(dims, dtype=f64, device=device)
    c = torch.rand(n_bumps, 3, generator=g, device=device, dtype=f64) * ext
    sg = sigma[0] + (sigma[1] - sigma[0]) * torch.rand(n_bumps, generator=g, device=device,
                                                       dtype=f64)
    amp = torch.randn(n_bumps, generator=g, device=device, dtype=f64)
    ax = [torch.arange(n, device=device, dtype=f64) for n in dims]
    k = -0.5 / (sg * sg)
    gz = torch.exp(k[:, None] * (ax[0][None, :] - c[:, 0:1]) ** 2) * amp[:, None]
    gy = torch.exp(k[:, None] * (ax[1][None, :] - c[:, 1:2]) ** 2)
    gx = torch.exp(k[:, None] * (ax[2][None, :] - c[:, 2:3]) ** 2)
    # sum_i gz_i (x) gy_i (x) gx_i as one product over the bump index
    gyx = (gy[:, :, None] * gx[:, None, :]).reshape(n_bumps, -1)
    out = torch.matmul(gz.t().contiguous(), gyx).reshape(dims)
    out += noise * torch.randn(dims, generator=g, device=device, dtype=f64)
    return out.to(torch.float32).contiguous()


def _kmag_t(dims, device):
    import torch
    nz, ny, nx = dims
    f64 = torch.float64
    kz = torch.fft.fftfreq(nz, d=1.0 / nz, device=device, dtype=f64)
    ky = torch.fft.fftfreq(ny, d=1.0 / ny, device=device, dtype=f64)
    kx = torch.fft.rfftfreq(nx, d=1.0 / nx, device=device, dtype=f64)
    return torch.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)


def _filtered_t(dims, alpha, seed, device, random_phase, dtype):
    import torch
    g = _tgen(seed, device)
    white = torch.randn(dims, generator=g, device=device, dtype=dtype)
    W = torch.fft.rfftn(white)
    del white
    k = _kmag_t(dims, device).to(dtype)
    amp = torch.where(k > 0, k.clamp_min(1e-30) ** (-alpha / 2.0), torch.zeros_like(k))
    del k
    if random_phase:
        mag = W.abs()
        W = torch.where(mag > 0, W / torch.where(mag > 0, mag, torch.ones_like(mag)),
                        torch.zeros_like(W))
        del mag
    W = W * amp
    del amp
    W[0, 0, 0] = 0
    f = torch.fft.irfftn(W, s=dims)
    del W
    f = f - f.mean()
    sd = f.std()
    if sd > 0:
        f = f / sd
    return f


def spectral_t(dims, alpha, seed, device, dtype=None):
    import torch
    return _filtered_t(dims, alpha, seed, device, True,
                       dtype or torch.float64).to(torch.float32).contiguous()


def spectral64_t(dims, alpha, seed, device):
    """spectral_t kept in float64 (a double-precision field, for the float64
    path)."""
    import torch
    return _filtered_t(dims, alpha, seed, device, True, torch.float64).contiguous()


def grf_t(dims, alpha, seed, device, dtype=None):
    import torch
    return _filtered_t(dims, alpha, seed, device, False,
                       dtype or torch.float64).to(torch.float32).contiguous()


def lognormal_t(dims, alpha, seed, device, dtype=None):
    import torch
    g = _filtered_t(dims, alpha, seed, device, False, dtype or torch.float64)
    return torch.exp(g).to(torch.float32).contiguous()


def spectral_crop_t(dims, alpha, seed, device):
    """spectral_t synthesized on the power-of-two cube that holds `dims` and
    cropped to `dims`, then normalized again: every field of a batch of uneven
    shapes reuses one of a few FFT sizes."""
    import torch
    side = 1
    while side < max(dims):
        side *= 2
    f = _filtered_t((side, side, side), alpha, seed, device, True, torch.float64)
    f = f[:dims[0], :dims[1], :dims[2]]
    f = f - f.mean()
    sd = f.std()
    if sd > 0:
        f = f / sd
    return f.to(torch.float32).contiguous()


def make_t(kind, dims, seed, device):
    if kind == "bumps":
        return bumps_t(dims, seed, device)
    if kind == "spectral":
        return spectral_crop_t(dims, 5.0 / 3.0, seed, device)
    raise ValueError(kind)
