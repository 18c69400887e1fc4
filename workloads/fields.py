"""Random fields and vectors for the synthetic workloads.

Every generator takes an explicit seed and uses numpy's PCG64 bit generator, so
the same call returns the same array on every machine.  Arrays over the grid are
indexed ``[k, j, i]`` (z, y, x) and flatten to the natural unknown ordering
``r = (k * ny + j) * nx + i`` used throughout the solver's interface.

Grid: vertex-centred finite differences on the unit cube with homogeneous
Dirichlet boundary conditions; unknown ``i`` of an axis with ``n`` points sits
at ``(i + 1) * h`` with ``h = 1 / (n + 1)`` (the model problem of Section 2.2.1
of the paper, discretised with the 7-point stencil).
"""
import numpy as np
import scipy.fft as sfft

# Seed assignment for the named workloads (one stream per role).
SEEDS = {
    "kappa": 0, "rhs": 1, "velocity": 2, "speed": 2,
    "obs_cells": 3, "obs_noise": 4, "fd_dirs": 5, "kappa_true": 6, "perturb27": 7,
}


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def grid_h(n):
    """Mesh width of an axis with ``n`` interior points on [0, 1]."""
    return 1.0 / (n + 1)


def _padded_shape(shape, corr, hs):
    # Zero padding of at least four correlation lengths keeps the periodic
    # wrap-around of the FFT filter from coupling opposite faces of the cube.
    return tuple(sfft.next_fast_len(int(n + np.ceil(4.0 * corr / h))) for n, h in zip(shape, hs))


def _gaussian_kernel_hat(pshape, corr, hs):
    """FFT of exp(-r^2 / (2 corr^2)) sampled on the periodic padded grid."""
    axes = []
    for p, h in zip(pshape, hs):
        idx = np.arange(p)
        d = np.minimum(idx, p - idx) * h
        axes.append(np.exp(-d * d / (2.0 * corr * corr)))
    ker = axes[0][:, None, None] * axes[1][None, :, None] * axes[2][None, None, :]
    return np.real(sfft.fftn(ker))


def _filtered_noise(shape, corr, rng, count=1):
    """Stationary Gaussian fields with squared-exponential covariance.

    White N(0, 1) noise on a zero-padded periodic grid is filtered with the
    square root of the covariance spectrum; returns the padded fields (before
    cropping) so derivatives can be taken spectrally.
    """
    hs = [grid_h(n) for n in shape]
    pshape = _padded_shape(shape, corr, hs)
    khat = np.sqrt(np.maximum(_gaussian_kernel_hat(pshape, corr, hs), 0.0))
    out = []
    for _ in range(count):
        w = rng.standard_normal(pshape)
        out.append(np.real(sfft.ifftn(sfft.fftn(w) * khat)))
    return out, pshape, hs


def _normalise(g):
    g = g - g.mean()
    return g / g.std()


def gaussian_random_field(shape, corr=0.2, seed=0):
    """Zero-mean, unit-std Gaussian random field on the node grid.

    ``shape`` is (nz, ny, nx).  Squared-exponential covariance with the given
    correlation length; the sample mean and std are removed exactly.
    """
    shape = tuple(int(s) for s in shape)
    (g,), _, _ = _filtered_noise(shape, corr, _rng(seed))
    g = g[: shape[0], : shape[1], : shape[2]]
    return _normalise(g)


def lognormal_kappa(n, seed=SEEDS["kappa"], corr=0.2):
    """kappa = exp(g) with g a unit-std Gaussian random field; shape (n, n, n)."""
    return np.exp(gaussian_random_field((n, n, n), corr, seed))


def rhs_normal(N, nrhs=1, seed=SEEDS["rhs"]):
    """Right-hand sides with i.i.d. N(0, 1) entries, column-major (N, nrhs)."""
    f = _rng(seed).standard_normal((nrhs, N)).T
    return np.ascontiguousarray(f[:, 0]) if nrhs == 1 else np.asfortranarray(f)


def divergence_free_velocity(kappa, seed=SEEDS["velocity"], corr=0.2, peclet=1.0):
    """Random divergence-free velocity b = curl(psi), shape (3, nz, ny, nx).

    psi has three independent Gaussian-random-field components; the curl is
    taken spectrally on the padded periodic grid and sampled at the nodes.  The
    field is scaled so that the largest cell Peclet number
    max_{r,d} |b_d(r)| h_d / (2 kappa_r) equals ``peclet``.
    Component order is (x, y, z).
    """
    nz, ny, nx = kappa.shape
    psis, pshape, hs = _filtered_noise((nz, ny, nx), corr, _rng(seed), count=3)
    # axis 0 = z, 1 = y, 2 = x; wavenumbers in physical units
    kz = 2j * np.pi * sfft.fftfreq(pshape[0], d=hs[0])[:, None, None]
    ky = 2j * np.pi * sfft.fftfreq(pshape[1], d=hs[1])[None, :, None]
    kx = 2j * np.pi * sfft.fftfreq(pshape[2], d=hs[2])[None, None, :]
    px, py, pz = (sfft.fftn(p) for p in psis)
    bx = np.real(sfft.ifftn(ky * pz - kz * py))
    by = np.real(sfft.ifftn(kz * px - kx * pz))
    bz = np.real(sfft.ifftn(kx * py - ky * px))
    b = np.stack([bx, by, bz])[:, :nz, :ny, :nx]
    hvec = np.array([hs[2], hs[1], hs[0]])[:, None, None, None]
    pe = np.max(np.abs(b) * hvec / (2.0 * kappa[None]))
    return b * (peclet / pe)


def helmholtz_speed(n, seed=SEEDS["speed"], corr=0.1, amp=0.3):
    """Wave speed c(x) = 1 + amp * s(x) for the indefinite Helmholtz workload.

    s is uniform(-1, 1) white noise smoothed with a Gaussian of the given
    correlation length (FFT convolution on a padded grid), rescaled so that
    max |s| = 1.
    """
    shape = (n, n, n)
    hs = [grid_h(n)] * 3
    pshape = _padded_shape(shape, corr, hs)
    w = _rng(seed).uniform(-1.0, 1.0, pshape)
    khat = _gaussian_kernel_hat(pshape, corr, hs)
    s = np.real(sfft.ifftn(sfft.fftn(w) * khat))[:n, :n, :n]
    s = s / np.max(np.abs(s))
    return 1.0 + amp * s


def helmholtz_omega(n, points_per_wavelength=10.0):
    """Angular frequency giving the stated points per wavelength at c = 1."""
    return 2.0 * np.pi * (n + 1) / points_per_wavelength


def observation_cells(N, count=512, seed=SEEDS["obs_cells"]):
    """Distinct observed unknowns, sampled without replacement, sorted."""
    return np.sort(_rng(seed).choice(N, size=count, replace=False)).astype(np.int64)


def observation_noise(count=512, seed=SEEDS["obs_noise"]):
    return _rng(seed).standard_normal(count)


def fd_directions(kappa, count=8, seed=SEEDS["fd_dirs"]):
    """Relative perturbation directions v_i = kappa * z_i with z ~ N(0, 1)."""
    z = _rng(seed).standard_normal((count,) + kappa.shape)
    return z * kappa[None]
