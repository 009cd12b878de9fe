// Memory-bound FP64 kernels of the Krylov engine (see engkern.hip) and the
// small dense FP64 solvers (see dense.hip).  Vector blocks are row-major:
// vector j of a block at base + j * ld.
#pragma once

#include "common.hpp"

namespace rid {

// Scratch for the two-pass reductions (owned by the caller).
struct RedScratch {
  double* part;      // >= gram_part_elems(m, n, N)
  size_t part_elems;
};

size_t gram_part_elems(int m, int n, long N);

// C[i * ldc + j] = sum_k V[i][k] W[j][k] for i < m, j < n (f64, two passes).
void gram(const double* V, long ldv, int m, const double* W, long ldw, int n, long N, double* C, int ldc,
          const RedScratch& rs, hipStream_t s);
// Out[j][k] = beta * Out[j][k] + alpha * sum_i c[i * csi + j * csj] V[i][k] for j < n.
void combo(const double* V, long ldv, int m, const double* c, int csi, int csj, int n, long N, double alpha,
           double beta, double* Out, long ldo, hipStream_t s);
// out_j = a_j - sh[idx_j] * b_j - c_j  (idx device, null = identity; c may be null).
void resid3(const double* a, const double* b, const double* c, long ld, int n, long N, const double* sh,
            double* out, long ldo, hipStream_t s);
// Projected-matrix update after appending columns [m0, m): for i < m and
// j in [m0, m): a[i][j] = a[j][i] = (c1[i][j-m0] + c2[i][j-m0]) / 2, where
// c1 = V^T (op V_new) and c2 = (op V)^T V_new (each m x (m - m0), row-major).
void proj_update(double* a, int lda, int m, int m0, const double* c1, const double* c2, hipStream_t s);
// out[j] = ||W_j||_2 for j < n.
void col_norms(const double* W, long ldw, int n, long N, double* out, const RedScratch& rs, hipStream_t s);
// W_j *= sc[j] (device scalars); if inv: W_j /= sc[j] (zero left unscaled).
void scale_cols(double* W, long ldw, int n, long N, const double* sc, int inv, hipStream_t s);
// R_j = AX_j - om[j] X_j  (om device).
void residual(const double* AX, const double* X, long ld, int n, long N, const double* om, double* R,
              hipStream_t s);
// Pair residuals: R1_j = P_j - om[j] Z'_j, R2_j = M_j - om[j] Z_j.
void residual_pair(const double* Pz, const double* Zp, const double* Mzp, const double* Z, long ld, int n, long N,
                   const double* om, double* R1, double* R2, hipStream_t s);
// out_j = r_j / g(de - sh[j]) with the +-1e-8 denominator guard; idx (device,
// optional) selects source columns: out_j uses r_{idx[j]}, sh[idx[j]].
void diag_tda(const double* de, const double* r, long ldr, int n, long N, const double* sh, const int* idx,
              double* out, long ldo, hipStream_t s);
// Pair form of the diagonal preconditioner:
// d1 = (de r1 + s r2) / (g(de - s)(de + s)), d2 = (s r1 + de r2) / (...).
void diag_pair(const double* de, const double* r1, const double* r2, long ldr, int n, long N, const double* sh,
               const int* idx, double* d1, double* d2, long ldo, hipStream_t s);
// out_j = a * x_j + b * y_j (per-column device coefficients a[j], b[j]; null = 0).
void axpby_cols(const double* x, const double* y, long ld, int n, long N, const double* a, const double* b,
                double* out, long ldo, hipStream_t s);
// Copy columns: dst_j = src_{idx[j]} (idx device, null = identity).
void gather_cols(const double* src, long lds, const int* idx, int n, long N, double* dst, long ldd, hipStream_t s);
// Unit vectors: out_j = e_{pos[j]} (pos device).
void unit_vectors(const int* pos, int n, long N, double* out, long ldo, hipStream_t s);
// Elementwise cast f64 -> f64 negation helper: dst = alpha * src.
void scale_copy(const double* src, long n, double alpha, double* dst, hipStream_t s);
// dst = src / r if the device scalar r >= tol, else 0.
void accept_scale(const double* src, long n, const double* r, double tol, double* dst, hipStream_t s);
// out[0, n) = diagonal of l (n x n, leading dim ldl), out[n, 2n) = nrm[0, n),
// out[2n] = info[0]: the figures a Cholesky-QR step checks, for one read.
void chol_check_pack(const double* l, int n, int ldl, const double* nrm, const int* info, double* out, hipStream_t s);

// ---- small dense FP64 (dense.hip) -------------------------------------------
// Symmetric eigen-decomposition of a (m x m, leading dim lda) by cyclic
// Jacobi in one workgroup; a is overwritten.  w[m] ascending, q (m x m,
// row-major, q[i * m + j] = component i of eigenvector j); work >= m*m + m.
void small_eigh(double* a, int m, int lda, double* w, double* q, double* work, hipStream_t s);
// The k lowest eigenpairs of symmetric a (m x m, lda; destroyed): w[k]
// ascending, q[i * ldq + t] = component i of eigenvector t.  work >=
// small_syevx_work(m, k) doubles.  m is at most kMaxProjected.
constexpr int kMaxProjected = 1024;  // largest projected dimension of the dense eigen/Cholesky kernels
size_t small_syevx_work(int m, int k);
void small_syevx(double* a, int m, int lda, int k, double* w, double* q, int ldq, double* work, hipStream_t s);
// Cholesky a = L L^T in place (lower triangle, upper zeroed); info[0] = 0 on
// success, j+1 if the j-th pivot is not positive (that pivot is replaced by
// 1 and the factorisation goes on).  One wavefront for m <= 64, panels of
// 16 columns in LDS for m <= 512, column by column beyond.
void small_chol(double* a, int m, int lda, int* info, hipStream_t s);
// Batched dense solve with partial pivoting: for b < nb, solve
// M_b y_b = g_b where M_b is m x m at mats + b * m * m (row-major; destroyed)
// and g_b at rhs + b * m (overwritten by y_b).  A pivot below 1e-300 in
// magnitude is replaced by +-1e-300.
void small_lu_solve(double* mats, double* rhs, int m, int nb, hipStream_t s);
// The same for column-major matrices, one workgroup per system: in LDS up
// to 128 unknowns, by 16-column panels up to 512, a column at a time beyond
// (the three give bit-identical solutions).
void small_lu_solve_cm(double* mats, double* rhs, int m, int nb, hipStream_t s);
// Pair systems of the inner full-TDDFT solve (see dense.hip): build the
// nsys column-major matrices and right-hand sides, and write the solutions
// back into g (rows of length 2m: y then y').
void pair_systems_build(const double* P, const double* tp, const double* tm, int ld, int m, const int* sys_b,
                        const int* sys_type, const double* sys_shift, int nsys, const double* g, int ldg,
                        const double* tg, double* mats, double* rhs, hipStream_t s);
void pair_systems_unpack(double* g, int ldg, const double* sol, const double* yt, const int* sys_b,
                         const int* sys_type, const double* sys_shift, int nsys, int m, hipStream_t s);
// C (m x n) = alpha * op(A) op(B) + beta * C, row-major, op = transpose if t*.
void small_gemm(int ta, int tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
                double beta, double* C, int ldc, hipStream_t s);
// G = L^{-1} for lower-triangular L (m x m).
void small_trinv_lower(const double* L, int m, int ldl, double* G, int ldg, hipStream_t s);
// mats_b = t - sh_b^2 w for b < nb (m x m each, contiguous).
void build_schur(const double* t, int ldt, const double* w, int ldw, int m, const double* sh, int nb, double* mats,
                 hipStream_t s);
// out_b = x_b + sh_b y_b for nb rows of length m.
void rows_axpy(const double* x, int ldx, const double* y, int ldy, const double* sh, int nb, int m, double* out,
               int ldo, hipStream_t s);
// Symmetrise in place: a = (a + a^T) / 2 over the leading m x m block.
void small_symmetrize(double* a, int m, int lda, hipStream_t s);
// Build shifted systems for the inner solves: for b < nb,
//   single: M_b = t - sh[b] I  (m x m)
//   pair:   M_b = [[tp, -sh[b] I], [-sh[b] I, tm]]  (2m x 2m)
void build_shifted(const double* t, const double* tm, int m, int ld, const double* sh, int nb, int pair,
                   double* mats, hipStream_t s);
// Copy a (rows x cols) block with leading dims (device to device).
void copy_block(const double* src, int lds, int rows, int cols, double* dst, int ldd, hipStream_t s);

}  // namespace rid
