// Launch wrappers of the kernels in ops.hip (weights, reductions, closure, GMRES pieces).
#pragma once

#include <algorithm>

#include "internal.hpp"

namespace bae {

// Sparse map from densities on gamma- to source weights on gamma- u E (internal order).
struct CSR {
    int64_t rows = 0;
    int64_t padded_rows = 0;   // weights past `rows` are written as zero
    int32_t* rowptr = nullptr;
    int32_t* col = nullptr;
    double* coef = nullptr;
};

// Dirichlet closure rows in gamma- (lexicographic) order: internal target indices of q
// and of its partner p, and the weight t.
struct Closure {
    int64_t n = 0;
    int32_t* tq = nullptr;
    int32_t* tp = nullptr;
    double* t = nullptr;
};

// Device-resident GMRES state for up to `cap` right-hand sides, basis capacity m.
struct KrylovState {
    int m = 0;                 // max iterations (basis m+1 vectors)
    int64_t n = 0;             // vector length
    int64_t ld_rhs = 0;        // (m+1) * n
    double* V = nullptr;       // [rhs][m+1][n]
    double* H = nullptr;       // [rhs][m][m+1]  column-major Hessenberg
    double* cs = nullptr;      // [rhs][m]
    double* sn = nullptr;
    double* g = nullptr;       // [rhs][m+1]
    double* hist = nullptr;    // [rhs][m]
    double* beta = nullptr;    // [rhs]
    int32_t* done = nullptr;   // [rhs]
    int32_t* kdone = nullptr;  // [rhs]
};

void launch_weights(const CSR& B, const double* q, int64_t ldq, void* w, int64_t ldw, int nrhs, int prec,
                    hipStream_t st);
void launch_reduce_scatter(const double* part, int chunks, int64_t nt, const int32_t* pos, double* out, int64_t ldo,
                           int nrhs, double scale, hipStream_t st);
// vsum: scratch [nrhs][nt] for the chunk-reduced sums
void launch_closure(const double* part, int chunks, int64_t nt, const Closure& cl, double* aq, int64_t lda, int nrhs,
                    double* vsum, hipStream_t st);
// The direct formulation's system rows (Sec. 3.1) from the chunk partials of its LGF sum:
// v + (sum) on gamma+, the Dirichlet rows of v on gamma-; v and aq in [gamma+; gamma-] order.
void launch_direct_closure(const double* part, int chunks, int64_t nt, const int32_t* tinv, int64_t ngp,
                           const int32_t* partner, const double* t, const double* v, int64_t ldv, double* aq,
                           int64_t lda, int nrhs, double* vsum, hipStream_t st);
int dot_blocks(int64_t n);
// h[r][j] (+)= <X[r][j], y[r]> for j < nj; partial: scratch [nrhs][maxj][dot_blocks(n)].
void launch_dots(const double* X, int64_t ldx_vec, int64_t ldx_rhs, int nj, const double* y, int64_t ldy, int64_t n,
                 int nrhs, const int32_t* done, double* partial, int maxj, double* h, int64_t ldh, int accumulate,
                 hipStream_t st);
// The slices only: partial[r][j][b] (b < dot_blocks(n)), summed by the consumers below.
void launch_dot_slices(const double* X, int64_t ldx_vec, int64_t ldx_rhs, int nj, const double* y, int64_t ldy,
                       int64_t n, int nrhs, const int32_t* done, double* partial, int maxj, hipStream_t st);
// y[r] -= sum_j c[r][j] X[r][j] with c the summed slices of cpart; with npart non-null also
// the slices of ||y[r]||^2 (npart[r][b], b < norm_blocks(n)).
void launch_subtract_combination(const double* X, int64_t ldx_vec, int64_t ldx_rhs, const double* cpart, int maxj,
                                 int nj, int64_t n, int nrhs, const int32_t* done, double* y, int64_t ldy,
                                 double* npart, hipStream_t st);
int norm_blocks(int64_t n);
// out[r][l] = sum_{j < kin} X[r][j] M[r][j][l], l < kout; M [nrhs][kin][kout] on the device.
void launch_basis_transform(const double* X, int64_t ldx_vec, int64_t ldx_rhs, int kin, const double* M, int kout,
                            int64_t n, int nrhs, double* out, int64_t ldo_vec, int64_t ldo_rhs, hipStream_t st);
void launch_combination(const double* X, int64_t ldx_vec, int64_t ldx_rhs, const double* c, int64_t ldc,
                        const int32_t* nj, int64_t n, int nrhs, double* y, int64_t ldy, int accumulate,
                        hipStream_t st);
void launch_normalize(double* V, int64_t ldv_vec, int64_t ldv_rhs, int k, int64_t n, const double* npart,
                      const int32_t* done, int nrhs, hipStream_t st);
void launch_givens(const KrylovState& K, const double* pA, const double* pB, int maxj, const double* npart, int k,
                   double tol, int nrhs, hipStream_t st);
// The closing launch of Arnoldi step k: V[k+1] = wv / ||w||, the next source weights from
// that vector (precision prec, into w with leading dimension ldw) and the Givens update.
// host_flag (optional, device-mapped host memory): receives done[r] of every RHS.
void launch_finish(const KrylovState& K, const double* wv, int64_t ldwv, const double* pA, const double* pB, int maxj,
                   const double* npart, int k, double tol, const CSR& B, void* w, int64_t ldw, int prec, int nrhs,
                   int32_t* host_flag, hipStream_t st);
void launch_gmres_init(const double* r0, int64_t ldr, const KrylovState& K, int64_t n, const double* nrm2, int nrhs,
                       hipStream_t st);
void launch_axpby(double a, const double* x, int64_t ldx, double b, double* y, int64_t ldy, int64_t n, int nrhs,
                  hipStream_t st);
void launch_gather(const double* x, int64_t ldx, const int32_t* idx, int64_t n, double* y, int64_t ldy, int nrhs,
                   double scale, hipStream_t st);
// b = g - Phi u_p on gamma- (up: [nrhs][ngp + ngm] in [gamma+; gamma-] order, or null);
// a non-finite g sets *bad.
void launch_rhs(const double* g, int64_t ldg, const double* up, int64_t ldu, const int32_t* partner, const double* t,
                int64_t ngp, int64_t ngm, double* b, int64_t ldb, int nrhs, int32_t* bad, hipStream_t st);
void launch_finite_check(const double* x, int64_t ldx, int64_t n, int nrhs, int32_t* bad, hipStream_t st);
// y[r][idx[i]] = x[r][i]
void launch_scatter(const double* x, int64_t ldx, const int32_t* idx, int64_t n, double* y, int64_t ldy, int nrhs,
                    hipStream_t st);
void launch_fill(double* y, int64_t n, double v, hipStream_t st);
void launch_fill_int(int32_t* y, int64_t n, int32_t v, hipStream_t st);
void launch_to_float(const double* x, float* y, int64_t n, hipStream_t st);

}  // namespace bae
