"""Random initial yield-perturbation fields phi0 (Section 3.2.2, the two
distributions the paper uses, plus the log-normal and inclusion fields of the
synthetic workloads).

All fields are cell-centred on the initial Eulerian mesh, shaped (nz, ny, nx),
and generated on the host from a numpy PCG64 generator.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_field(shape, a, seed):
    """phi0 ~ U(1-a, 1+a) independently per cell (Section 3.2.2, uniform)."""
    return _rng(seed).uniform(1.0 - a, 1.0 + a, size=shape)


def correlated_normal(shape, spacing, corr_len, seed):
    """Zero-mean, unit-variance Gaussian field with covariance
    exp(-r^2 / (2 l^2)): white noise filtered in Fourier space by
    exp(-|k|^2 l^2 / 4), then normalised to the sample mean and std.
    `spacing` is (dz, dy, dx)."""
    rng = _rng(seed)
    w = rng.standard_normal(size=shape)
    spec = np.fft.rfftn(w)
    kz = 2 * np.pi * np.fft.fftfreq(shape[0], d=spacing[0])
    ky = 2 * np.pi * np.fft.fftfreq(shape[1], d=spacing[1])
    kx = 2 * np.pi * np.fft.rfftfreq(shape[2], d=spacing[2])
    k2 = (kz[:, None, None] ** 2 + ky[None, :, None] ** 2
          + kx[None, None, :] ** 2)
    spec *= np.exp(-k2 * corr_len ** 2 / 4.0)
    g = np.fft.irfftn(spec, s=shape, axes=(0, 1, 2))
    g -= g.mean()
    s = g.std()
    if s > 0:
        g /= s
    return g


def gaussian_field(shape, spacing, corr_len, std, seed):
    """Rectified Gaussian phi0 ~ N^R(1, std^2) with spatial correlation
    (Section 3.2.2, rectified Gaussian: negative values set to 0)."""
    g = correlated_normal(shape, spacing, corr_len, seed)
    return np.maximum(1.0 + std * g, 0.0)


def lognormal_field(shape, spacing, corr_len, sigma, seed):
    """Log-normal phi0 = exp(sigma g - sigma^2/2), mean 1."""
    g = correlated_normal(shape, spacing, corr_len, seed)
    return np.exp(sigma * g - 0.5 * sigma * sigma)


def inclusion_field(n, lo, hi, box_lo, box_hi, n_incl, r_min, r_max, factor,
                    seed):
    """phi0 = `factor` at cell centres inside any of `n_incl` spheres with
    radius ~ U(r_min, r_max) and centres uniform in [box_lo, box_hi], else 1
    (overlaps are not compounded).  n = (nx, ny, nz); lo/hi/box in (x,y,z)."""
    rng = _rng(seed)
    nx, ny, nz = n
    dx = [(hi[k] - lo[k]) / n[k] for k in range(3)]
    radii = rng.uniform(r_min, r_max, size=n_incl)
    centres = np.stack([rng.uniform(box_lo[k], box_hi[k], size=n_incl)
                        for k in range(3)], axis=1)
    inside = np.zeros((nz, ny, nx), dtype=bool)
    for c, r in zip(centres, radii):
        idx = []
        for k in range(3):
            i0 = int(np.floor((c[k] - r - lo[k]) / dx[k] - 0.5)) - 1
            i1 = int(np.ceil((c[k] + r - lo[k]) / dx[k] - 0.5)) + 2
            i0 = max(i0, 0)
            i1 = min(i1, n[k])
            idx.append((i0, i1))
        if any(a >= b for a, b in idx):
            continue
        xs = lo[0] + (np.arange(idx[0][0], idx[0][1]) + 0.5) * dx[0]
        ys = lo[1] + (np.arange(idx[1][0], idx[1][1]) + 0.5) * dx[1]
        zs = lo[2] + (np.arange(idx[2][0], idx[2][1]) + 0.5) * dx[2]
        d2 = ((zs[:, None, None] - c[2]) ** 2 + (ys[None, :, None] - c[1]) ** 2
              + (xs[None, None, :] - c[0]) ** 2)
        inside[idx[2][0]:idx[2][1], idx[1][0]:idx[1][1],
               idx[0][0]:idx[0][1]] |= d2 <= r * r
    out = np.ones((nz, ny, nx))
    out[inside] = factor
    return out
