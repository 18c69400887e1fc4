"""7- and 27-point stencils of the synthetic workloads, in the solver's input layout.

Layout: ``coef[7, nz, ny, nx]`` float64 with slot order
``C, W(i-1), E(i+1), S(j-1), N(j+1), B(k-1), T(k+1)`` so that, for the natural
index r = (k*ny + j)*nx + i,

    (A u)_r = C u_r + W u_{r-1} + E u_{r+1} + S u_{r-nx} + N u_{r+nx}
              + B u_{r-nx*ny} + T u_{r+nx*ny}.

Entries that would reach outside the grid are zero.  Grouping the unknowns by
plane k gives the block-tridiagonal matrix of Eq. (originalMatrix): D_k is the
5-point operator of plane k, E_k = diag(B[k]) and F_k = diag(T[k]).

Discretisation (the paper leaves the variable-coefficient scheme open):
vertex-centred, h = 1/(n+1); the coefficient on the face between nodes r and s
is the harmonic mean 2 k_r k_s / (k_r + k_s); a face to the Dirichlet boundary
uses k_r; (A u)_r = h^-2 [ sum_s k_rs (u_r - u_s) + n_b(r) k_r u_r ].
Convection is first-order upwind; Helmholtz is -Lap_h - (omega / c)^2.
"""
import numpy as np

from . import fields

SLOT_NAMES = ("C", "W", "E", "S", "N", "B", "T")
# (slot of the lower neighbour, slot of the upper neighbour, array axis) for x, y, z
_DIRS = ((1, 2, 2), (3, 4, 1), (5, 6, 0))


def _shift_lower(a, axis):
    """Value of the lower neighbour along ``axis`` (NaN where outside)."""
    out = np.full_like(a, np.nan)
    sl_dst = [slice(None)] * 3
    sl_src = [slice(None)] * 3
    sl_dst[axis] = slice(1, None)
    sl_src[axis] = slice(None, -1)
    out[tuple(sl_dst)] = a[tuple(sl_src)]
    return out


def _shift_upper(a, axis):
    out = np.full_like(a, np.nan)
    sl_dst = [slice(None)] * 3
    sl_src = [slice(None)] * 3
    sl_dst[axis] = slice(None, -1)
    sl_src[axis] = slice(1, None)
    out[tuple(sl_dst)] = a[tuple(sl_src)]
    return out


def diffusion_coef(kappa):
    """Stencil of -div(kappa grad u) with harmonic-mean face coefficients."""
    kappa = np.asarray(kappa, dtype=np.float64)
    nz, ny, nx = kappa.shape
    hs = {2: fields.grid_h(nx), 1: fields.grid_h(ny), 0: fields.grid_h(nz)}
    coef = np.zeros((7,) + kappa.shape)
    for lo, up, ax in _DIRS:
        ih2 = 1.0 / hs[ax] ** 2
        for slot, nb in ((lo, _shift_lower(kappa, ax)), (up, _shift_upper(kappa, ax))):
            inside = ~np.isnan(nb)
            kf = np.where(inside, 2.0 * kappa * np.where(inside, nb, 1.0)
                          / (kappa + np.where(inside, nb, 1.0)), kappa)
            coef[0] += ih2 * kf
            coef[slot] = np.where(inside, -ih2 * kf, 0.0)
    return coef


def add_upwind_convection(coef, b):
    """Add b . grad u, first-order upwind; ``b`` has shape (3, nz, ny, nx) in (x, y, z) order."""
    coef = coef.copy()
    nz, ny, nx = coef.shape[1:]
    hs = {2: fields.grid_h(nx), 1: fields.grid_h(ny), 0: fields.grid_h(nz)}
    for comp, (lo, up, ax) in enumerate(_DIRS):
        bd = b[comp]
        pos = np.maximum(bd, 0.0) / hs[ax]
        neg = np.minimum(bd, 0.0) / hs[ax]
        coef[0] += pos - neg
        lower_inside = ~np.isnan(_shift_lower(np.zeros_like(bd), ax))
        upper_inside = ~np.isnan(_shift_upper(np.zeros_like(bd), ax))
        coef[lo] += np.where(lower_inside, -pos, 0.0)
        coef[up] += np.where(upper_inside, neg, 0.0)
    return coef


def helmholtz_coef(c, omega):
    """Stencil of -Lap_h u - (omega / c)^2 u (indefinite for large omega)."""
    coef = diffusion_coef(np.ones_like(c, dtype=np.float64))
    coef[0] -= (omega / c) ** 2
    return coef


# ---------------------------------------------------------------- 27 points
# Layout coef[27, nz, ny, nx]: slot s = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) holds
# the coupling to the neighbour at offset (dx, dy, dz), so that
#     (A u)_r = sum_s coef[s][r] u_{r + dx + dy nx + dz nx ny};
# slot 13 is the centre.  D_k (dz = 0) and E_k, F_k (dz = -1, +1) are then
# 9-point plane operators.  Entries reaching outside the grid are zero.


def slot27(dx, dy, dz):
    return 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)


def _outside27(shape):
    """Boolean [27, nz, ny, nx]: the neighbour of a slot lies outside the grid."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((27,) + tuple(shape), bool)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                out[slot27(dx, dy, dz)] = ((i + dx < 0) | (i + dx >= nx) | (j + dy < 0) | (j + dy >= ny)
                                           | (k + dz < 0) | (k + dz >= nz))
    return out


def fem_q1_coef(shape, wavenumber=0.0):
    """27-point stencil of the trilinear (Q1) finite-element discretisation of
    -lap u - wavenumber^2 u on the unit cube with Dirichlet boundaries
    (Section 5.3): K - wavenumber^2 M on the interior nodes of a uniform grid.

    Per axis the assembled linear-element stencils are stiffness
    [-1, 2, -1] / h and mass [1, 4, 1] h / 6; the 3D stencils are their tensor
    products, K = Kx My Mz + Mx Ky Mz + Mx My Kz and M = Mx My Mz.
    """
    nz, ny, nx = shape
    axes = []
    for n in (nx, ny, nz):
        h = fields.grid_h(n)
        axes.append((np.array([-1.0, 2.0, -1.0]) / h, np.array([1.0, 4.0, 1.0]) * h / 6.0))
    (kx, mx), (ky, my), (kz, mz) = axes
    coef = np.zeros((27,) + tuple(shape))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                a, b, c = dx + 1, dy + 1, dz + 1
                v = kx[a] * my[b] * mz[c] + mx[a] * ky[b] * mz[c] + mx[a] * my[b] * kz[c]
                v -= wavenumber ** 2 * mx[a] * my[b] * mz[c]
                coef[slot27(dx, dy, dz)] = v
    coef[_outside27(shape)] = 0.0
    return coef


def perturbed_q1_coef(shape, seed=fields.SEEDS["perturb27"], spread=0.3, centre=1.35):
    """A nonsymmetric 27-point operator with the Q1 pattern: every off-centre
    entry of the Q1 Laplacian scaled by (1 + spread * xi), xi uniform on
    [-1, 1] per entry, the centre by ``centre``; strictly diagonally dominant
    (the Q1 Laplacian's off-centre magnitudes sum to its centre), hence
    nonsingular."""
    coef = fem_q1_coef(shape)
    rng = fields._rng(seed)
    xi = rng.uniform(-1.0, 1.0, coef.shape)
    off = np.ones(27, bool)
    off[13] = False
    coef[off] *= 1.0 + spread * xi[off]
    coef[13] *= centre
    return coef


def helmholtz27_wavenumber(n):
    """Wavenumber of the 27-point Helmholtz workload: n / 2 (16, 32, 64 at
    n = 32, 64, 128, the paper's choice of about 12 points per wavelength)."""
    return n / 2.0


PROBLEMS = ("poisson", "convdiff", "helmholtz", "laplace", "fem_poisson27", "fem_helmholtz27", "nonsym27")


def problem(kind, n, seed=None):
    """Coefficient array of a named workload on an n^3 grid.

    ``poisson``: -div(kappa grad u), kappa lognormal (seed 0 unless given).
    ``convdiff``: the same diffusion plus divergence-free upwind convection at
    cell Peclet <= 1 (velocity seed 2).  ``helmholtz``: -Lap u - (omega/c)^2 u
    with c = 1 + 0.3 * smoothed noise (seed 2), 10 points per wavelength.
    ``laplace``: kappa = 1 (the constant-coefficient special case).
    27-point (coef[27, ...]): ``fem_poisson27`` the trilinear finite-element
    Laplacian, ``fem_helmholtz27`` -(lap u + k^2 u) with k = n / 2 (Section
    5.3), ``nonsym27`` the perturbed nonsymmetric Q1 pattern (seed 7).
    """
    if kind == "fem_poisson27":
        return fem_q1_coef((n, n, n))
    if kind == "fem_helmholtz27":
        return fem_q1_coef((n, n, n), helmholtz27_wavenumber(n))
    if kind == "nonsym27":
        return perturbed_q1_coef((n, n, n), seed=fields.SEEDS["perturb27"] if seed is None else seed)
    if kind == "laplace":
        return diffusion_coef(np.ones((n, n, n)))
    if kind == "helmholtz":
        c = fields.helmholtz_speed(n, seed=fields.SEEDS["speed"] if seed is None else seed)
        return helmholtz_coef(c, fields.helmholtz_omega(n))
    kappa = fields.lognormal_kappa(n, seed=fields.SEEDS["kappa"] if seed is None else seed)
    coef = diffusion_coef(kappa)
    if kind == "poisson":
        return coef
    if kind == "convdiff":
        return add_upwind_convection(coef, fields.divergence_free_velocity(kappa))
    raise ValueError(f"unknown problem {kind!r}")
