"""Seeded field generators (inputs only; no part of the diffusion scheme)."""
import numpy as np


def _rng(seed):
    return np.random.default_rng(np.random.PCG64(int(seed)))


def ring(n, t_in=10.0, t_out=0.1):
    """Ring test of section 3.1 on [-1,1]^2 with n x n cells.

    b = (-y, x)/r at cell centres, b = 0 for r > 1 (conduction vanishes
    outside r = 1).  T = t_in for 0.5 < r < 0.7 and 11pi/12 < theta < 13pi/12,
    t_out elsewhere.  theta = atan2(y, x) taken in [0, 2 pi) so that the patch
    around theta = pi is not cut by the branch line.
    Returns (bx, by, T0, h).
    """
    h = 2.0 / n
    c = -1.0 + (np.arange(n) + 0.5) * h
    x, y = np.meshgrid(c, c, indexing="xy")  # shape (ny, nx)
    r = np.hypot(x, y)
    with np.errstate(invalid="ignore", divide="ignore"):
        bx = np.where(r > 0, -y / r, 0.0)
        by = np.where(r > 0, x / r, 0.0)
    outside = r > 1.0
    bx[outside] = 0.0
    by[outside] = 0.0
    theta = np.mod(np.arctan2(y, x), 2.0 * np.pi)
    hot = (r > 0.5) & (r < 0.7) & (theta > 11.0 * np.pi / 12.0) & (theta < 13.0 * np.pi / 12.0)
    T0 = np.where(hot, t_in, t_out).astype(np.float64)
    return bx, by, T0, h


def sovinec(n):
    """Smooth test of section 3.2 on [-0.5, 0.5]^2 with n x n cells: flux
    function psi = cos(pi x) cos(pi y), B = grad psi x z_hat =
    (dpsi/dy, -dpsi/dx), b = B/|B| (b = 0 where |B| < 1e-12 max |B|, i.e. at
    the centre for odd n), source Q = 2 pi^2 psi (so b lies along the
    contours of Q), T0 = 0.  Returns (bx, by, Q, psi, h)."""
    h = 1.0 / n
    c = -0.5 + (np.arange(n) + 0.5) * h
    x, y = np.meshgrid(c, c, indexing="xy")
    psi = np.cos(np.pi * x) * np.cos(np.pi * y)
    Bx = -np.pi * np.cos(np.pi * x) * np.sin(np.pi * y)
    By = np.pi * np.sin(np.pi * x) * np.cos(np.pi * y)
    m = np.hypot(Bx, By)
    ok = m > 1e-12 * m.max()
    safe = np.where(ok, m, 1.0)
    bx = np.where(ok, Bx / safe, 0.0)
    by = np.where(ok, By / safe, 0.0)
    Q = 2.0 * np.pi ** 2 * psi
    return bx, by, Q, psi, h


def _modes(ndim, kmax2):
    """Integer wave vectors m with 1 <= |m|^2 <= kmax2, one of each +-m pair."""
    k = int(np.floor(np.sqrt(kmax2)))
    rng1 = np.arange(-k, k + 1)
    grids = np.meshgrid(*([rng1] * ndim), indexing="ij")
    m = np.stack([g.ravel() for g in grids], axis=1)
    m2 = (m ** 2).sum(axis=1)
    keep = (m2 >= 1) & (m2 <= kmax2)
    m = m[keep]
    # keep the half space: first nonzero component positive
    first = np.array([row[np.nonzero(row)[0][0]] for row in m])
    return m[first > 0]


def _spectral_eval(shape, modes, amps, factors):
    """Evaluate sum_m Re[amp_m * factor_m * exp(2 pi i m.x)] at cell centres.

    shape: grid shape in (.., ny, nx) order; modes are (mx, my[, mz]).
    Cell centres sit at (i + 1/2)/n_axis on the unit interval.
    """
    ndim = len(shape)
    spec = np.zeros(shape, dtype=np.complex128)
    n_xyz = tuple(reversed(shape))
    for m, a, f in zip(modes, amps, factors):
        phase = np.exp(1j * np.pi * sum(m[q] / n_xyz[q] for q in range(ndim)))
        idx = tuple(int(m[q]) % n_xyz[q] for q in reversed(range(ndim)))
        spec[idx] += a * f * phase
    field = np.fft.ifftn(spec) * np.prod(shape)
    return field.real


def grf_unit_field_2d(nx, ny, seed, kmax2=64, lx=1.0, ly=1.0):
    """b = grad A_z x z_hat / |.| with A_z a flat-spectrum Gaussian random
    potential on the periodic box [0,lx) x [0,ly); modes 1 <= |m|^2 <= kmax2.

    grad A_z x z_hat = (dA/dy, -dA/dx).  b = 0 where |B| < 1e-12 max |B|.
    Returns (bx, by) with shape (ny, nx).
    """
    rng = _rng(seed)
    modes = _modes(2, kmax2)
    amps = rng.standard_normal(len(modes)) + 1j * rng.standard_normal(len(modes))
    kx = 2j * np.pi * modes[:, 0] / lx
    ky = 2j * np.pi * modes[:, 1] / ly
    dAdx = _spectral_eval((ny, nx), modes, amps, kx)
    dAdy = _spectral_eval((ny, nx), modes, amps, ky)
    Bx, By = dAdy, -dAdx
    mag = np.hypot(Bx, By)
    tiny = mag < 1e-12 * mag.max()
    with np.errstate(invalid="ignore", divide="ignore"):
        bx = np.where(tiny, 0.0, Bx / mag)
        by = np.where(tiny, 0.0, By / mag)
    return bx, by


def curl_unit_field_3d(n, seed, kmax2=36):
    """b = curl A / |curl A| on the periodic unit cube (n^3 cells), A with three
    independent flat-spectrum Gaussian random components, 1 <= |m|^2 <= kmax2.
    Returns (bx, by, bz) with shape (n, n, n) in (z, y, x) order.
    """
    rng = _rng(seed)
    modes = _modes(3, kmax2)
    shape = (n, n, n)
    amp = [rng.standard_normal(len(modes)) + 1j * rng.standard_normal(len(modes)) for _ in range(3)]
    ik = [2j * np.pi * modes[:, q] for q in range(3)]
    # curl A = (dAz/dy - dAy/dz, dAx/dz - dAz/dx, dAy/dx - dAx/dy)
    Bx = _spectral_eval(shape, modes, amp[2] * ik[1] - amp[1] * ik[2], np.ones(len(modes)))
    By = _spectral_eval(shape, modes, amp[0] * ik[2] - amp[2] * ik[0], np.ones(len(modes)))
    Bz = _spectral_eval(shape, modes, amp[1] * ik[0] - amp[0] * ik[1], np.ones(len(modes)))
    mag = np.sqrt(Bx * Bx + By * By + Bz * Bz)
    tiny = mag < 1e-12 * mag.max()
    with np.errstate(invalid="ignore", divide="ignore"):
        out = tuple(np.where(tiny, 0.0, B / mag) for B in (Bx, By, Bz))
    return out


def blobs_2d(nx, ny, seed, nblobs=8, rmin=0.05, rmax=0.2, width=0.01, amp=0.5, base=1.0,
             lx=1.0, ly=1.0):
    """T = base + amp * sum_k 0.5 [1 - tanh((d_k - R_k)/width)] on the periodic
    box [0,lx) x [0,ly); centres uniform, R_k ~ U[rmin, rmax], d_k the
    minimum-image distance from the cell centre.  Shape (ny, nx)."""
    rng = _rng(seed)
    cx = rng.uniform(0.0, lx, nblobs)
    cy = rng.uniform(0.0, ly, nblobs)
    R = rng.uniform(rmin, rmax, nblobs)
    x = (np.arange(nx) + 0.5) * (lx / nx)
    y = (np.arange(ny) + 0.5) * (ly / ny)
    X, Y = np.meshgrid(x, y, indexing="xy")
    T = np.full((ny, nx), float(base))
    for k in range(nblobs):
        dx = np.abs(X - cx[k])
        dx = np.minimum(dx, lx - dx)
        dy = np.abs(Y - cy[k])
        dy = np.minimum(dy, ly - dy)
        d = np.hypot(dx, dy)
        T += amp * 0.5 * (1.0 - np.tanh((d - R[k]) / width))
    return T


def smoothed_normal(shape, seed, sigma_cells=4.0):
    """White noise smoothed by a periodic Gaussian of sigma_cells cells, then
    re-standardised to zero mean and unit variance."""
    rng = _rng(seed)
    w = rng.standard_normal(shape)
    spec = np.fft.fftn(w)
    filt = np.ones(shape)
    for ax, n in enumerate(shape):
        f = np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[ax] = n
        filt = filt * np.exp(-2.0 * np.pi ** 2 * sigma_cells ** 2 * f ** 2).reshape(sh)
    g = np.fft.ifftn(spec * filt).real
    g -= g.mean()
    g /= g.std()
    return g


def lognormal_3d(n, seed, sigma_ln=0.3, sigma_cells=4.0):
    """T = exp(sigma_ln * g), g smoothed unit-variance noise on n^3 cells."""
    return np.exp(sigma_ln * smoothed_normal((n, n, n), seed, sigma_cells))


def chi_field_2d(nx, ny, seed, amp=0.5, sigma_cells=4.0):
    """Per-cell diffusivity chi = exp(amp * g), g smoothed unit-variance noise
    (amp = 0.5 is a log-normal with variance 0.25)."""
    return np.exp(amp * smoothed_normal((ny, nx), seed, sigma_cells))


def gaussian_pulse_x(nx, ny, sigma0, x0=0.5, t=0.0, chi=1.0, base=1.0):
    """Spreading Gaussian along x on the periodic unit square (independent of
    y): T = base + (sigma0/sigma_t) exp(-(x - x0)^2 / (2 sigma_t^2)),
    sigma_t^2 = sigma0^2 + 2 chi t.  Nearest periodic image only (sigma small)."""
    st = np.sqrt(sigma0 ** 2 + 2.0 * chi * t)
    x = (np.arange(nx) + 0.5) / nx
    dx = x - x0
    dx = dx - np.round(dx)
    row = base + (sigma0 / st) * np.exp(-dx ** 2 / (2.0 * st ** 2))
    return np.tile(row, (ny, 1))
