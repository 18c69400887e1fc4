// Stencil-side kernels: input validation, the level-0 conversion of plane
// blocks, ordering permutations, FP64 residuals and vector operations.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace acr {

struct Grid {
  int nx, ny, nz;
  int ns = 7;   // stencil slots: 7, or 27 (slot 9 (dz+1) + 3 (dy+1) + (dx+1) for the offset (dx, dy, dz))
  __host__ __device__ int64_t M() const { return (int64_t)nx * ny; }
  __host__ __device__ int64_t N() const { return M() * nz; }
};

// Entry of a plane's 5-point operator that falls inside a dense leaf.
struct LeafEnt { int leaf, a, b, n, slot, nat; };
// Entry coupling two sibling clusters (the exact low-rank cut couplings).
struct CutEnt { int r, c, slot, nat; };
// Entry of a 9-point plane operator coupling two sibling clusters, in the
// exact factors U (rows x k, a selection) and V (cols x k, the couplings):
// column j of block `blk` selects row r and holds the coupling to column c.
struct Cut9Ent { int blk, j, r, c, slot, nat; };

void launch_validate(Grid g, const double* coef, int* flags, hipStream_t s);
template <class T>
void launch_conv_leaves(Grid g, const double* coef, const LeafEnt* ents, int nent, T* const* leafptr, int nleaf,
                        hipStream_t s);
void launch_cut_rank(Grid g, const double* coef, const CutEnt* ents, const int* blk_first, int nblk, double eps,
                     int* ranks, hipStream_t s);
template <class T>
void launch_cut_fill(Grid g, const double* coef, const CutEnt* ents, const int* blk_first, int nblk, double eps,
                     T* const* uptr, T* const* vptr, const int* rows, const int* cols, hipStream_t s);
template <class T>
void launch_diag(Grid g, const double* coef, int slot, const int* perm, T* out, hipStream_t s);
// exact factors of the cut couplings of 9-point plane operators: for every
// plane k and entry e, U[k][blk][r + j rows] = 1, V[k][blk][c + j cols] = coef
// (U, V zeroed before; null pointers are skipped)
template <class T>
void launch_cut9_fill(Grid g, const double* coef, const Cut9Ent* ents, int nent, int nblk, T* const* uptr,
                      T* const* vptr, const int* rows, const int* cols, hipStream_t s);
// W[k][c][pos] = b[k*M + perm[pos] + c*ldb]  (and the inverse)
template <class T>
void launch_perm_in(Grid g, int nrhs, const double* b, int64_t ldb, const int* perm, T* W, hipStream_t s);
template <class T>
void launch_perm_out(Grid g, int nrhs, const T* W, const int* perm, double* x, int64_t ldx, hipStream_t s);
// r = b - op(A) x, FP64, natural order
void launch_residual(Grid g, const double* coef, const double* x, const double* b, double* r, int transpose,
                     hipStream_t s);
// partial sums of <x_i, y> for i < nvec (x_i = X + i*ldx) into part[nvec][nblocks]
void launch_multidot(int64_t n, int nvec, const double* X, int64_t ldx, const double* y, double* part,
                     int nblocks, hipStream_t s);
// out[i] = sum_b part[i][b]
void launch_reduce_parts(int nvec, const double* part, int nblocks, double* out, hipStream_t s);
// y -= X h (h device, nvec entries); y = alpha x + beta y
void launch_gemv_sub(int64_t n, int nvec, const double* X, int64_t ldx, const double* h, double* y,
                     hipStream_t s);
void launch_axpby(int64_t n, double alpha, const double* x, double beta, double* y, hipStream_t s);
void launch_scale_copy(int64_t n, const double* x, const double* alpha_dev, int invert, double* y,
                       hipStream_t s);
void launch_assemble(Grid g, const double* kappa, double* coef, hipStream_t s);
void launch_kappa_grad(Grid g, const double* kappa, const double* u, const double* lam, double* grad,
                       hipStream_t s);

}  // namespace acr
