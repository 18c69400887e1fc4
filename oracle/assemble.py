"""Sparse assembly of the model operators and the residual metric (oracle).

Two routes to the same matrix, written independently of the input generators:

* ``operator_from_fields`` loops over grid faces and boundary faces
  (model problem of Section 2.2.1, Eq. probSta; convection-diffusion of
  Section 5.2 with a random velocity; Helmholtz of Section 5.3 with a
  7-point Laplacian and a variable wave speed).
* ``operator_from_coef`` reads a 7- or 27-point coefficient array (the
  solver's input format) entry by entry.
* ``fem_q1_operator`` assembles the trilinear finite-element matrix of
  Section 5.3 (-lap u - k^2 u) element by element from the 8 x 8 element
  stiffness and mass matrices.

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


def _offsets27(nx, ny, N, i_idx, j_idx, k_idx):
    """Neighbour offset and in-grid mask of the 27 slots, slot
    9 (dz + 1) + 3 (dy + 1) + (dx + 1) for the neighbour at (dx, dy, dz)."""
    offsets, inside = {}, {}
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                s = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                offsets[s] = dx + dy * nx + dz * nx * ny
                inside[s] = ((i_idx + dx >= 0) & (i_idx + dx < nx) & (j_idx + dy >= 0) & (j_idx + dy < ny)
                             & (k_idx + dz >= 0) & (k_idx + dz < N // (nx * ny)))
    return offsets, inside


def operator_from_coef(coef):
    """CSR matrix of a 7-point coefficient array coef[7, nz, ny, nx] or a
    27-point one coef[27, nz, ny, nx].

    7 points: slot order C, W(i-1), E(i+1), S(j-1), N(j+1), B(k-1), T(k+1).
    27 points: slot 9 (dz + 1) + 3 (dy + 1) + (dx + 1) couples node (i, j, k)
    to (i + dx, j + dy, k + dz).  Raises if a coefficient reaching outside the
    grid is nonzero.
    """
    coef = np.asarray(coef, dtype=np.float64)
    ns, nz, ny, nx = coef.shape
    N = nx * ny * nz
    k_idx, j_idx, i_idx = np.unravel_index(np.arange(N), (nz, ny, nx))
    if ns == 27:
        offsets, inside = _offsets27(nx, ny, N, i_idx, j_idx, k_idx)
    elif ns == 7:
        offsets = {0: 0, 1: -1, 2: 1, 3: -nx, 4: nx, 5: -nx * ny, 6: nx * ny}
        inside = {
            0: np.ones(N, bool), 1: i_idx > 0, 2: i_idx < nx - 1, 3: j_idx > 0,
            4: j_idx < ny - 1, 5: k_idx > 0, 6: k_idx < nz - 1,
        }
    else:
        raise ValueError("coefficient arrays have 7 or 27 slots")
    rows, cols, vals = [], [], []
    for slot in range(ns):
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


def plane_blocks(A, nx, ny, nz, diagonal=True):
    """Dense D_k and the couplings E_k, F_k of the block-tridiagonal A.

    E_k couples plane k to plane k-1 and F_k to plane k+1 (Eq. originalMatrix).
    diagonal=True (7-point stencils): E_k, F_k are returned as their
    diagonals, and that they are diagonal is checked; diagonal=False (27-point
    stencils, whose couplings are 9-point plane operators): dense M x M.
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
                if not diagonal:
                    lst.append(blk)
                    continue
                dg = np.diag(blk).copy()
                if np.any(blk - np.diag(dg)):
                    raise ValueError("plane coupling is not diagonal")
                lst.append(dg)
            else:
                lst.append(None)
    return D, E, F


def fem_q1_operator(shape, wavenumber=0.0):
    """CSR matrix of the trilinear (Q1) finite-element discretisation of
    -lap u - wavenumber^2 u on the unit cube, Dirichlet boundaries (Section
    5.3), assembled element by element.

    The grid has shape = (nz, ny, nx) interior nodes at (i + 1) h per axis,
    h = 1/(n + 1); every cell of the (n + 1)^3 cells is an element whose
    8 x 8 stiffness and mass matrices are Kronecker products of the linear
    element matrices (1/h)[[1, -1], [-1, 1]] and (h/6)[[2, 1], [1, 2]]; rows and
    columns of boundary nodes are dropped (u = 0 there).
    """
    nz, ny, nx = shape
    dims = (nx, ny, nz)
    kel, mel = [], []
    for n in dims:
        h = _h(n)
        kel.append(np.array([[1.0, -1.0], [-1.0, 1.0]]) / h)
        mel.append(np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0)
    # local node (a, b, c) in {0,1}^3 -> index a + 2 b + 4 c (x fastest)
    kron3 = lambda ex, ey, ez: np.kron(ez, np.kron(ey, ex))
    Kloc = (kron3(kel[0], mel[1], mel[2]) + kron3(mel[0], kel[1], mel[2]) + kron3(mel[0], mel[1], kel[2]))
    Aloc = Kloc - wavenumber ** 2 * kron3(mel[0], mel[1], mel[2])
    corners = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]
    rows, cols, vals = [], [], []
    # cell (ci, cj, ck) spans grid lines ci..ci+1 (line 0 and line n+1 are the boundary)
    ci, cj, ck = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    for la, (a, b, c) in enumerate(corners):
        ia, ja, ka = ci + a - 1, cj + b - 1, ck + c - 1       # interior index of the corner node
        oka = (ia >= 0) & (ia < nx) & (ja >= 0) & (ja < ny) & (ka >= 0) & (ka < nz)
        ga = (ka * ny + ja) * nx + ia
        for lb, (a2, b2, c2) in enumerate(corners):
            ib, jb, kb = ci + a2 - 1, cj + b2 - 1, ck + c2 - 1
            okb = (ib >= 0) & (ib < nx) & (jb >= 0) & (jb < ny) & (kb >= 0) & (kb < nz)
            ok = oka & okb
            gb = (kb * ny + jb) * nx + ib
            rows.append(ga[ok])
            cols.append(gb[ok])
            vals.append(np.full(int(ok.sum()), Aloc[la, lb]))
    N = nx * ny * nz
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A.tocsr()


def relres(A, x, b):
    """||b - A x||_2 / ||b||_2 column by column (Section 5 accuracy metric)."""
    r = b - A @ x
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)
