"""Seeded high-contrast media on an n x n cell grid.

The paper's own permeability fields exist only as figures (Section 5), so the
workloads use synthetic stand-ins with the same structure: a background plus
straight high-conductivity channels (channelised media, Section 3.2) and small
inclusions, at contrast 1e2..1e6 (Section 5). kappa[iy, ix] is the value on
cell (ix, iy).
"""
import numpy as np


def _channel_rows(rng, n, n_c, count):
    """Pick `count` distinct coarse rows, and a uniform fine row inside each."""
    m = n // n_c
    coarse = rng.choice(n_c, size=count, replace=False)
    fine = coarse * m + rng.integers(0, m, size=count)
    return np.sort(coarse), np.sort(fine)


def straight_channels(n, n_c, n_h, n_v, contrast, rng, background=None):
    """Background (default 1) plus n_h horizontal and n_v vertical full-span
    channels one cell wide, at most one per coarse row / column."""
    kappa = np.ones((n, n)) if background is None else np.array(background, dtype=np.float64)
    ch_rows_c, ch_rows = _channel_rows(rng, n, n_c, n_h)
    ch_cols_c, ch_cols = _channel_rows(rng, n, n_c, n_v)
    kappa[ch_rows, :] = contrast
    kappa[:, ch_cols] = contrast
    return kappa, ch_rows_c, ch_cols_c


def gaussian_field(n, corr_len, rng):
    """Unit-variance stationary Gaussian field on the cell grid with Gaussian
    covariance exp(-r^2 / (2 l^2)), made by FFT filtering of white noise."""
    white = rng.standard_normal((n, n))
    k = np.fft.fftfreq(n, d=1.0 / n)  # integer wave numbers on the unit square
    kx, ky = np.meshgrid(k, k, indexing="xy")
    # spectral density of the Gaussian covariance (up to a constant)
    amp = np.exp(-((2 * np.pi) ** 2) * (kx ** 2 + ky ** 2) * corr_len ** 2 / 4.0)
    g = np.real(np.fft.ifft2(np.fft.fft2(white) * amp))
    g -= g.mean()
    g /= g.std()
    return g


def lognormal_channels(n, n_c, sigma, corr_len, n_h, n_v, contrast, incl_frac, rng):
    """exp(sigma*g) background, full-span channels of value `contrast`, and
    2x2-cell inclusions of value `contrast` in a fraction of the channel-free
    coarse elements (at most one per element)."""
    back = np.exp(sigma * gaussian_field(n, corr_len, rng))
    kappa, rows_c, cols_c = straight_channels(n, n_c, n_h, n_v, contrast, rng, back)
    m = n // n_c
    free = [(ey, ex) for ey in range(n_c) for ex in range(n_c)
            if ey not in set(rows_c.tolist()) and ex not in set(cols_c.tolist())]
    n_incl = int(round(incl_frac * len(free)))
    pick = rng.choice(len(free), size=n_incl, replace=False)
    for p in pick:
        ey, ex = free[p]
        iy = ey * m + rng.integers(1, m - 2)
        ix = ex * m + rng.integers(1, m - 2)
        kappa[iy:iy + 2, ix:ix + 2] = contrast
    return kappa
