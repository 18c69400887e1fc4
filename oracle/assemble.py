"""Sparse assembly of the model operators and the residual metric (oracle).

Two routes to the same matrix, written independently of the input generators:

* ``operator_from_fields`` loops over grid faces and boundary faces
  (model problem of Section 2.2.1, Eq. probSta; convection-diffusion of
  Section 5.2 with a random velocity; Helmholtz of Section 5.3 with a
  7-point Laplacian and a variable wave speed).
* ``operator_from_coef`` reads a 7-point coefficient array (the solver's
  input format) entry by entry.

``plane_blocks`` cuts the matrix into the plane blocks of Eq. originalMatrix
and ``relres`` is the accuracy metric of Section 5, ||A x - b|| / ||b||.
"""
import numpy as np
import scipy.sparse as sp


def _h(n):
    return 1.0 / (n + 1)


def operator_from_fields(shape, kappa=None, velocity=None, speed=None, omega=None):
    """CSR matrix of -div(kappa grad u) [+ b.grad u upwind] [- (omega/c)^2 u].

    shape = (nz, ny, nx); kappa defaults to 1; velocity is (3, nz, ny, nx) in
    (x, y, z) component order.  Face coefficient: harmonic mean of the two
    nodal values; boundary faces use the nodal value (Dirichlet u = 0).
    """
    nz, ny, nx = shape
    N = nx * ny * nz
    kap = np.ones(N) if kappa is None else np.asarray(kappa, dtype=np.float64).reshape(N)
    k_idx, j_idx, i_idx = np.unravel_index(np.arange(N), (nz, ny, nx))
    coords = (i_idx, j_idx, k_idx)
    dims = (nx, ny, nz)
    strides = (1, nx, nx * ny)
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    for d in range(3):
        h2 = _h(dims[d]) ** 2
        has_up = coords[d] < dims[d] - 1
        r = np.nonzero(has_up)[0]
        s = r + strides[d]
        kf = 2.0 * kap[r] * kap[s] / (kap[r] + kap[s]) / h2
        np.add.at(diag, r, kf)
        np.add.at(diag, s, kf)
        rows += [r, s]
        cols += [s, r]
        vals += [-kf, -kf]
        nb = (coords[d] == 0).astype(float) + (coords[d] == dims[d] - 1).astype(float)
        diag += nb * kap / h2
    if velocity is not None:
        for d in range(3):
            h = _h(dims[d])
            b = np.asarray(velocity[d], dtype=np.float64).reshape(N)
            bp, bm = np.maximum(b, 0.0) / h, np.minimum(b, 0.0) / h
            diag += bp - bm
            lo = np.nonzero(coords[d] > 0)[0]
            rows.append(lo)
            cols.append(lo - strides[d])
            vals.append(-bp[lo])
            up = np.nonzero(coords[d] < dims[d] - 1)[0]
            rows.append(up)
            cols.append(up + strides[d])
            vals.append(bm[up])
    if speed is not None:
        diag -= (omega / np.asarray(speed, dtype=np.float64).reshape(N)) ** 2
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A.tocsr()


def operator_from_coef(coef):
    """CSR matrix of a 7-point coefficient array coef[7, nz, ny, nx].

    Slot order C, W(i-1), E(i+1), S(j-1), N(j+1), B(k-1), T(k+1).  Raises if a
    coefficient reaching outside the grid is nonzero.
    """
    coef = np.asarray(coef, dtype=np.float64)
    _, nz, ny, nx = coef.shape
    N = nx * ny * nz
    k_idx, j_idx, i_idx = np.unravel_index(np.arange(N), (nz, ny, nx))
    offsets = {0: 0, 1: -1, 2: 1, 3: -nx, 4: nx, 5: -nx * ny, 6: nx * ny}
    inside = {
        0: np.ones(N, bool), 1: i_idx > 0, 2: i_idx < nx - 1, 3: j_idx > 0,
        4: j_idx < ny - 1, 5: k_idx > 0, 6: k_idx < nz - 1,
    }
    rows, cols, vals = [], [], []
    for slot in range(7):
        c = coef[slot].reshape(N)
        ok = inside[slot]
        if np.any(c[~ok] != 0.0):
            raise ValueError(f"stencil slot {slot} reaches outside the grid")
        r = np.nonzero(ok)[0]
        rows.append(r)
        cols.append(r + offsets[slot])
        vals.append(c[r])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A.tocsr()


def plane_blocks(A, nx, ny, nz):
    """Dense D_k and the diagonals of E_k, F_k of the block-tridiagonal A.

    E_k couples plane k to plane k-1 and F_k to plane k+1 (Eq. originalMatrix);
    for a 7-point stencil both are diagonal, which is checked.
    """
    M = nx * ny
    A = sp.csr_matrix(A)
    D, E, F = [], [], []
    for k in range(nz):
        rows = slice(k * M, (k + 1) * M)
        D.append(A[rows, rows].toarray())
        for lst, kk in ((E, k - 1), (F, k + 1)):
            if 0 <= kk < nz:
                blk = A[rows, kk * M:(kk + 1) * M].toarray()
                dg = np.diag(blk).copy()
                if np.any(blk - np.diag(dg)):
                    raise ValueError("plane coupling is not diagonal")
                lst.append(dg)
            else:
                lst.append(None)
    return D, E, F


def relres(A, x, b):
    """||b - A x||_2 / ||b||_2 column by column (Section 5 accuracy metric)."""
    r = b - A @ x
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)
