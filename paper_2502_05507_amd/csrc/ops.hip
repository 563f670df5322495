// Device kernels around the LGF sum: double-layer weights, chunk reduction, the
// hat-function closure Phi, and the FP64 GMRES building blocks (dot products, classical
// Gram-Schmidt with re-orthogonalisation, Givens rotations) for several right-hand
// sides at once.  Everything here is memory-latency bound and small next to the LGF sum.
#include "ops.hpp"

namespace bae {

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n, int per = kThreads) { return (unsigned)((n + per - 1) / per); }

// w[r][s] = sum_{j in row s} coef[j] q[r][col[j]]   (Sec. 3.2: w(n) = |D_n| q(n), w(k) = -sum q)
// Rows in [ns, npad) are the padding sources of the last block: weight zero.
template <typename Real>
__global__ void weights_kernel(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                               const double* __restrict__ coef, int64_t ns, int64_t npad,
                               const double* __restrict__ q, int64_t ldq, Real* __restrict__ w, int64_t ldw) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= npad) return;
    double acc = 0.0;
    if (s < ns) {
        const double* qr = q + r * ldq;
        for (int j = rowptr[s]; j < rowptr[s + 1]; ++j) acc = fma(coef[j], qr[col[j]], acc);
    }
    w[r * ldw + s] = (Real)acc;
}

// out[r][pos[t]] = scale * sum_c part[r][c][t]  (+ add[r][pos[t]] when add != null)
// out[r][pos(t)] = scale * sum over chunks of part[r][c][t].  A block covers 64 targets
// with 4 chunk lanes (chunk c goes to lane c mod 4; every load is a coalesced 512-byte row),
// the lane sums combined in a fixed order, so results do not vary between runs.
__global__ __launch_bounds__(256) void reduce_chunks_kernel(const double* __restrict__ part, int chunks, int64_t nt,
                                                            int64_t ldp, const int32_t* __restrict__ pos,
                                                            double* __restrict__ out, int64_t ldo, double scale) {
    __shared__ double sh[4][64];
    const int tl = threadIdx.x & 63, cl = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * 64 + tl;
    const int r = blockIdx.y;
    double acc = 0.0;
    if (t < nt) {
        const double* p = part + r * ldp + t;
        for (int c = cl; c < chunks; c += 4) acc += p[(int64_t)c * nt];
    }
    sh[cl][tl] = acc;
    __syncthreads();
    if (cl == 0 && t < nt) out[r * ldo + (pos ? pos[t] : t)] = scale * (((sh[0][tl] + sh[1][tl]) + sh[2][tl]) + sh[3][tl]);
}

// aq[r][i] = (1 - t_i) v(q_i) + t_i v(p_i), v the reduced sum at the internal target indices
// of q_i and of its partner p_i (Sec. 2.1 eq. "bc", hat functions).
__global__ void closure_kernel(const double* __restrict__ v, int64_t ldv, const int32_t* __restrict__ tq,
                               const int32_t* __restrict__ tp, const double* __restrict__ tw, int64_t n,
                               double* __restrict__ aq, int64_t lda) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= n) return;
    const double t = tw[i];
    aq[r * lda + i] = (1.0 - t) * v[r * ldv + tq[i]] + t * v[r * ldv + tp[i]];
}

// The direct system (Sec. 3.1, eq. "direct_sys") from the reduced LGF sums vsum (internal
// target order, [nrhs][nt]): rows on gamma+ (j < ngp) v[j] + vsum[tinv[j]]; rows on gamma-
// (j = ngp + q) the Dirichlet row (1 - t_q) v[j] + t_q v[partner_q].
__global__ void direct_closure_kernel(const double* __restrict__ vsum, int64_t nt, const int32_t* __restrict__ tinv,
                                      int64_t ngp, const int32_t* __restrict__ partner,
                                      const double* __restrict__ tw, const double* __restrict__ v, int64_t ldv,
                                      double* __restrict__ aq, int64_t lda) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (j >= nt) return;
    const double* vr = v + r * ldv;
    double y;
    if (j < ngp) {
        y = vr[j] + vsum[r * nt + tinv[j]];
    } else {
        const int64_t q = j - ngp;
        const double t = tw[q];
        y = (1.0 - t) * vr[j] + t * vr[partner[q]];
    }
    aq[r * lda + j] = y;
}

__device__ inline double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
    return s;
}

// partial[r][j][b] = sum over slice b of X[r][j][i] * y[r][i]; j < nj (grid y), b < nb.
// The consumers add the nb slices themselves, always in the same order (no finalize
// launch, no cross-block synchronisation, deterministic results).
__global__ void dots_kernel(const double* __restrict__ X, int64_t ldx_vec, int64_t ldx_rhs,
                            const double* __restrict__ y, int64_t ldy, int64_t n, int nb,
                            const int32_t* __restrict__ done, double* __restrict__ partial, int maxj) {
    __shared__ double sh[kThreads / 64];
    const int b = blockIdx.x, j = blockIdx.y, r = blockIdx.z;
    if (done && done[r]) return;
    const int64_t per = (n + nb - 1) / nb;
    const int64_t lo = b * per, hi = min(n, lo + per);
    const double* x = X + r * ldx_rhs + j * ldx_vec;
    const double* yy = y + r * ldy;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) acc = fma(x[i], yy[i], acc);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[((int64_t)r * maxj + j) * nb + b] = s;
}

// Sum of nb partial results in a fixed order: eight independent running sums, so that
// eight loads are in flight at a time (one sum would wait on every load in turn).
__device__ inline double slice_sum(const double* p, int nb) {
    double t[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 8 <= nb; k += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] += p[k + u];
    }
    for (int u = 0; k < nb; ++k, ++u) t[u] += p[k];
    return ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
}

// The same by the whole block (every thread calls it and gets the sum), for the longer
// lists of norm slices: strided partial sums, then a wavefront tree and the wavefronts'
// sums in order.
__device__ double block_slice_sum(const double* p, int nb) {
    __shared__ double ws[kThreads / 64];
    double t = 0.0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) t += p[k];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    __syncthreads();   // an earlier call's readers are done with ws
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
    __syncthreads();
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += ws[w];
    return sum;
}

// h[r][j] (+)= sum_b partial[r][j][b]   (the few places that need h itself)
__global__ void dots_finalize_kernel(const double* __restrict__ partial, int nb, int nj, int maxj,
                                     const int32_t* __restrict__ done, double* __restrict__ h, int64_t ldh,
                                     int accumulate) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (j >= nj || (done && done[r])) return;
    const double s = slice_sum(partial + ((int64_t)r * maxj + j) * nb, nb);
    h[r * ldh + j] = accumulate ? h[r * ldh + j] + s : s;
}

// y[r][i] -= sum_{j < nj} c[r][j] X[r][j][i], c[r][j] = the nb dot-product slices of
// cpart summed by every block into LDS.  With npart, also the block's sum of the squared
// results goes to npart[r][blockIdx.x] (slices of ||y[r]||^2).
__global__ void subtract_combination_kernel(const double* __restrict__ X, int64_t ldx_vec, int64_t ldx_rhs,
                                            const double* __restrict__ cpart, int nb, int maxj, int nj, int64_t n,
                                            const int32_t* __restrict__ done, double* __restrict__ y,
                                            int64_t ldy, double* __restrict__ npart) {
    extern __shared__ double cl[];   // nj coefficients
    __shared__ double sh[kThreads / 64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (done && done[r]) return;
    for (int j = threadIdx.x; j < nj; j += blockDim.x) cl[j] = slice_sum(cpart + ((int64_t)r * maxj + j) * nb, nb);
    __syncthreads();
    double v2 = 0.0;
    if (i < n) {
        const double* x = X + r * ldx_rhs + i;
        double acc = 0.0;
        for (int j = 0; j < nj; ++j) acc = fma(cl[j], x[j * ldx_vec], acc);
        const double v = y[r * ldy + i] - acc;
        y[r * ldy + i] = v;
        v2 = v * v;
    }
    if (!npart) return;
    const double s = block_sum(v2, sh);
    if (threadIdx.x == 0) npart[(int64_t)r * gridDim.x + blockIdx.x] = s;
}

// y[r][i] (+)= sum_{j < nj[r]} c[r][j] X[r][j][i]
__global__ void combination_kernel(const double* __restrict__ X, int64_t ldx_vec, int64_t ldx_rhs,
                                   const double* __restrict__ c, int64_t ldc, const int32_t* __restrict__ nj,
                                   int64_t n, double* __restrict__ y, int64_t ldy, int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= n) return;
    const double* x = X + r * ldx_rhs + i;
    const double* cr = c + r * ldc;
    double acc = 0.0;
    for (int j = 0; j < nj[r]; ++j) acc = fma(cr[j], x[j * ldx_vec], acc);
    y[r * ldy + i] = accumulate ? y[r * ldy + i] + acc : acc;
}

// out[r][l] = sum_{j < kin} X[r][j] M[r][j][l] for l < kout (a change of basis of a few
// vectors; M is small and row-major per RHS).
__global__ void basis_transform_kernel(const double* __restrict__ X, int64_t ldx_vec, int64_t ldx_rhs, int kin,
                                       const double* __restrict__ M, int kout, int64_t n, double* __restrict__ out,
                                       int64_t ldo_vec, int64_t ldo_rhs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= n) return;
    const double* x = X + r * ldx_rhs + i;
    const double* mr = M + (int64_t)r * kin * kout;
    for (int l = 0; l < kout; ++l) {
        double acc = 0.0;
        for (int j = 0; j < kin; ++j) acc = fma(x[j * ldx_vec], mr[j * kout + l], acc);
        out[r * ldo_rhs + l * ldo_vec + i] = acc;
    }
}

// Scale w = V[k+1] to unit length; ||w||^2 is the sum of its nn slices npart[r][*].
__global__ void normalize_kernel(double* __restrict__ V, int64_t ldv_vec, int64_t ldv_rhs, int k, int64_t n,
                                 const double* __restrict__ npart, int nn, const int32_t* __restrict__ done) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (done && done[r]) return;
    const double nr = sqrt(block_slice_sum(npart + (int64_t)r * nn, nn));
    if (i < n && nr > 0.0) V[r * ldv_rhs + (int64_t)(k + 1) * ldv_vec + i] /= nr;
}

// Givens update of column k (Saad-Schultz) for RHS r by one block, residual estimate,
// convergence / breakdown flag.  H is column-major per RHS: H[r][k][i], i <= k+1.  The
// column is the sum of the Gram-Schmidt passes' coefficients, each the sum of its nb
// dot-product slices (pA, and pB when there is a second pass; summed by the block's
// threads); H[k+1][k] = ||w|| from the nn norm slices.  The rotations themselves are
// sequential (thread 0).
struct GivensArgs {
    double* Hc;
    int64_t ldh_col, ldh_rhs;
    const double *pA, *pB;
    int nb, maxj;
    const double* npart;
    int nn;
    double *cs, *sn;
    int64_t ldcs;
    double* g;
    int64_t ldg;
    const double* beta;
    double* hist;
    int64_t ldhist;
    int32_t *done, *kdone;
    int k;
    double tol;
};

// The previous rotations are applied to the new column in chunks staged in LDS: the
// rotations are a sequential chain, and with their operands in global memory every step
// would wait on a load (0.3 us each, 25 us at k = 85).
constexpr int kGivensChunk = 256;

__device__ void givens_block(const GivensArgs& a, int r) {
    __shared__ double hk1s, carry;
    __shared__ double hc[kGivensChunk], cc[kGivensChunk], sc[kGivensChunk];
    const int k = a.k;
    double* h = a.Hc + r * a.ldh_rhs + (int64_t)k * a.ldh_col;
    const double* c = a.cs + r * a.ldcs;
    const double* s = a.sn + r * a.ldcs;
    auto hval = [&](int i) {
        const double h1 = slice_sum(a.pA + ((int64_t)r * a.maxj + i) * a.nb, a.nb);
        return a.pB ? h1 + slice_sum(a.pB + ((int64_t)r * a.maxj + i) * a.nb, a.nb) : h1;
    };
    const double hk1_all = sqrt(block_slice_sum(a.npart + (int64_t)r * a.nn, a.nn));
    if (threadIdx.x == 0) {
        hk1s = hk1_all;
        carry = hval(0);   // the entry the next rotation takes as its x
    }
    // rotation i mixes entries i and i + 1; chunk [i0, i1) of rotations
    for (int i0 = 0; i0 < k; i0 += kGivensChunk) {
        const int i1 = min(k, i0 + kGivensChunk);
        __syncthreads();
        for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) {
            hc[i - i0] = hval(i + 1);
            cc[i - i0] = c[i];
            sc[i - i0] = s[i];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double x = carry;
            for (int i = i0; i < i1; ++i) {
                const double y = hc[i - i0], ci = cc[i - i0], si = sc[i - i0];
                hc[i - i0] = ci * x + si * y;   // final entry i
                x = -si * x + ci * y;
            }
            carry = x;
        }
        __syncthreads();
        for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) h[i] = hc[i - i0];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double hk1 = hk1s;
    double* cw = a.cs + r * a.ldcs;
    double* sw = a.sn + r * a.ldcs;
    const double x = carry, y = hk1;
    const double rr = hypot(x, y);
    double* gr = a.g + r * a.ldg;
    if (rr == 0.0) {          // exact breakdown of a singular system: stop here
        a.done[r] = 1;
        a.kdone[r] = k;
        return;
    }
    cw[k] = x / rr;
    sw[k] = y / rr;
    h[k] = rr;
    h[k + 1] = 0.0;
    gr[k + 1] = -sw[k] * gr[k];
    gr[k] = cw[k] * gr[k];
    const double est = fabs(gr[k + 1]) / a.beta[r];
    a.hist[r * a.ldhist + k] = est;
    a.kdone[r] = k + 1;
    if (est <= a.tol || hk1 == 0.0) a.done[r] = 1;
}

__global__ void givens_kernel(const GivensArgs a) {
    const int r = blockIdx.x;
    if (a.done[r]) return;
    givens_block(a, r);
}

// The closing launch of an Arnoldi step (one row of blocks per RHS): the orthogonalised
// vector w (in wv) scaled by 1/||w|| into V[k+1] (blocks [0, nbn)); the same scaled vector
// mapped to the next operator's source weights (Sec. 3.2; blocks [nbn, nbn + nbw)), so the
// next step starts with the LGF sum; the Givens update (last block).  ||w|| is the sum of
// the norm slices, formed by every block alike.
template <typename Real>
__global__ void finish_kernel(double* __restrict__ V, int64_t ldv_vec, int64_t ldv_rhs, const double* __restrict__ wv,
                              int64_t ldwv, int64_t n, int nbn, int nbw, const int32_t* __restrict__ rowptr,
                              const int32_t* __restrict__ col, const double* __restrict__ coef, int64_t ns,
                              int64_t npad, Real* __restrict__ w, int64_t ldw, const GivensArgs ga,
                              int32_t* host_flag) {
    const int r = blockIdx.y;
    const int b = blockIdx.x;
    if (b == nbn + nbw) {
        if (!ga.done[r]) givens_block(ga, r);
        // the convergence flag straight into host memory (no copy launch per step)
        if (threadIdx.x == 0 && host_flag)
            __hip_atomic_store(host_flag + r, ga.done[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return;
    }
    if (ga.done[r]) return;
    const double nr = sqrt(block_slice_sum(ga.npart + (int64_t)r * ga.nn, ga.nn));
    const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
    const double* x = wv + r * ldwv;
    if (b < nbn) {
        const int64_t i = (int64_t)b * blockDim.x + threadIdx.x;
        if (i < n) V[r * ldv_rhs + (int64_t)(ga.k + 1) * ldv_vec + i] = inv > 0.0 ? x[i] * inv : x[i];
        return;
    }
    const int64_t sidx = (int64_t)(b - nbn) * blockDim.x + threadIdx.x;
    if (sidx >= npad) return;
    double acc = 0.0;
    if (sidx < ns)
        for (int j = rowptr[sidx]; j < rowptr[sidx + 1]; ++j) acc = fma(coef[j], x[col[j]] * inv, acc);
    w[r * ldw + sidx] = (Real)acc;
}

// beta = sqrt(nrm2); V[0] = r0 / beta; g[0] = beta; done = beta == 0
__global__ void gmres_init_kernel(const double* __restrict__ r0, int64_t ldr, double* __restrict__ V,
                                  int64_t ldv_rhs, int64_t n, const double* __restrict__ nrm2,
                                  double* __restrict__ beta, double* __restrict__ g, int64_t ldg,
                                  int32_t* __restrict__ done, int32_t* __restrict__ kdone) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const double b = sqrt(nrm2[r]);
    if (i == 0) {
        beta[r] = b;
        g[r * ldg] = b;
        done[r] = b == 0.0;
        kdone[r] = 0;
    }
    if (i < n) V[r * ldv_rhs + i] = b > 0.0 ? r0[r * ldr + i] / b : 0.0;
}

__global__ void axpby_kernel(double a, const double* __restrict__ x, int64_t ldx, double b,
                             double* __restrict__ y, int64_t ldy, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i < n) y[r * ldy + i] = a * x[r * ldx + i] + b * y[r * ldy + i];
}

__global__ void gather_kernel(const double* __restrict__ x, int64_t ldx, const int32_t* __restrict__ idx,
                              int64_t n, double* __restrict__ y, int64_t ldy, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i < n) y[r * ldy + i] = scale * x[r * ldx + idx[i]];
}

// b[r][q] = g[r][q] - ((1 - t_q) up[r][ngp + q] + t_q up[r][partner_q])  (Sec. 3.4: the
// right-hand side g - Phi u_p; up on gamma in [gamma+; gamma-] order, or null for u_p = 0).
// A non-finite g sets *bad (system scope: it may be mapped host memory).
__global__ void rhs_kernel(const double* __restrict__ g, int64_t ldg, const double* __restrict__ up, int64_t ldu,
                           const int32_t* __restrict__ partner, const double* __restrict__ t, int64_t ngp,
                           int64_t ngm, double* __restrict__ b, int64_t ldb, int32_t* __restrict__ bad) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= ngm) return;
    const double gv = g[r * ldg + q];
    if (!isfinite(gv)) __hip_atomic_store(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    double v = gv;
    if (up) v -= (1.0 - t[q]) * up[r * ldu + ngp + q] + t[q] * up[r * ldu + partner[q]];
    b[r * ldb + q] = v;
}

// *bad = 1 (system scope) if any of x[r][i], i < n, is not finite.
__global__ void finite_check_kernel(const double* __restrict__ x, int64_t ldx, int64_t n, int32_t* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i < n && !isfinite(x[r * ldx + i])) __hip_atomic_store(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// y[r][idx[i]] = x[r][i]
__global__ void scatter_kernel(const double* __restrict__ x, int64_t ldx, const int32_t* __restrict__ idx, int64_t n,
                               double* __restrict__ y, int64_t ldy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i < n) y[r * ldy + idx[i]] = x[r * ldx + i];
}

__global__ void fill_kernel(double* __restrict__ y, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

__global__ void fill_int_kernel(int32_t* __restrict__ y, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

__global__ void to_float_kernel(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

}  // namespace

#define LAUNCH_CHECK() BAE_HIP_CHECK(hipGetLastError())

void launch_weights(const CSR& B, const double* q, int64_t ldq, void* w, int64_t ldw, int nrhs, int prec,
                    hipStream_t st) {
    if (B.padded_rows == 0) return;
    dim3 grid(blocks_for(B.padded_rows), nrhs);
    if (prec == BAE_PREC_FP64)
        weights_kernel<double><<<grid, kThreads, 0, st>>>(B.rowptr, B.col, B.coef, B.rows, B.padded_rows, q, ldq,
                                                          (double*)w, ldw);
    else
        weights_kernel<float><<<grid, kThreads, 0, st>>>(B.rowptr, B.col, B.coef, B.rows, B.padded_rows, q, ldq,
                                                         (float*)w, ldw);
    LAUNCH_CHECK();
}

void launch_reduce_scatter(const double* part, int chunks, int64_t nt, const int32_t* pos, double* out, int64_t ldo,
                           int nrhs, double scale, hipStream_t st) {
    if (nt == 0) return;
    dim3 grid((unsigned)((nt + 63) / 64), nrhs);
    reduce_chunks_kernel<<<grid, 256, 0, st>>>(part, chunks, nt, (int64_t)chunks * nt, pos, out, ldo, scale);
    LAUNCH_CHECK();
}

void launch_closure(const double* part, int chunks, int64_t nt, const Closure& cl, double* aq, int64_t lda, int nrhs,
                    double* vsum, hipStream_t st) {
    if (cl.n == 0) return;
    launch_reduce_scatter(part, chunks, nt, nullptr, vsum, nt, nrhs, 1.0, st);
    dim3 grid(blocks_for(cl.n), nrhs);
    closure_kernel<<<grid, kThreads, 0, st>>>(vsum, nt, cl.tq, cl.tp, cl.t, cl.n, aq, lda);
    LAUNCH_CHECK();
}

void launch_direct_closure(const double* part, int chunks, int64_t nt, const int32_t* tinv, int64_t ngp,
                           const int32_t* partner, const double* t, const double* v, int64_t ldv, double* aq,
                           int64_t lda, int nrhs, double* vsum, hipStream_t st) {
    if (nt == 0) return;
    launch_reduce_scatter(part, chunks, nt, nullptr, vsum, nt, nrhs, 1.0, st);
    direct_closure_kernel<<<dim3(blocks_for(nt), nrhs), kThreads, 0, st>>>(vsum, nt, tinv, ngp, partner, t, v, ldv,
                                                                           aq, lda);
    LAUNCH_CHECK();
}

int dot_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(64, (n + 2047) / 2048)); }

void launch_dots(const double* X, int64_t ldx_vec, int64_t ldx_rhs, int nj, const double* y, int64_t ldy, int64_t n,
                 int nrhs, const int32_t* done, double* partial, int maxj, double* h, int64_t ldh, int accumulate,
                 hipStream_t st) {
    const int nb = dot_blocks(n);
    launch_dot_slices(X, ldx_vec, ldx_rhs, nj, y, ldy, n, nrhs, done, partial, maxj, st);
    dots_finalize_kernel<<<dim3(blocks_for(nj, 64), nrhs), 64, 0, st>>>(partial, nb, nj, maxj, done, h, ldh,
                                                                         accumulate);
    LAUNCH_CHECK();
}

void launch_dot_slices(const double* X, int64_t ldx_vec, int64_t ldx_rhs, int nj, const double* y, int64_t ldy,
                       int64_t n, int nrhs, const int32_t* done, double* partial, int maxj, hipStream_t st) {
    const int nb = dot_blocks(n);
    dots_kernel<<<dim3(nb, nj, nrhs), kThreads, 0, st>>>(X, ldx_vec, ldx_rhs, y, ldy, n, nb, done, partial, maxj);
    LAUNCH_CHECK();
}

void launch_subtract_combination(const double* X, int64_t ldx_vec, int64_t ldx_rhs, const double* cpart, int maxj,
                                 int nj, int64_t n, int nrhs, const int32_t* done, double* y, int64_t ldy,
                                 double* npart, hipStream_t st) {
    const int nb = dot_blocks(n);
    subtract_combination_kernel<<<dim3(blocks_for(n), nrhs), kThreads, sizeof(double) * nj, st>>>(
        X, ldx_vec, ldx_rhs, cpart, nb, maxj, nj, n, done, y, ldy, npart);
    LAUNCH_CHECK();
}

int norm_blocks(int64_t n) { return (int)blocks_for(n); }

void launch_combination(const double* X, int64_t ldx_vec, int64_t ldx_rhs, const double* c, int64_t ldc,
                        const int32_t* nj, int64_t n, int nrhs, double* y, int64_t ldy, int accumulate,
                        hipStream_t st) {
    combination_kernel<<<dim3(blocks_for(n), nrhs), kThreads, 0, st>>>(X, ldx_vec, ldx_rhs, c, ldc, nj, n, y, ldy,
                                                                        accumulate);
    LAUNCH_CHECK();
}

void launch_normalize(double* V, int64_t ldv_vec, int64_t ldv_rhs, int k, int64_t n, const double* npart,
                      const int32_t* done, int nrhs, hipStream_t st) {
    normalize_kernel<<<dim3(blocks_for(n), nrhs), kThreads, 0, st>>>(V, ldv_vec, ldv_rhs, k, n, npart,
                                                                      norm_blocks(n), done);
    LAUNCH_CHECK();
}

static GivensArgs givens_args(const KrylovState& K, const double* pA, const double* pB, int maxj, const double* npart,
                              int k, double tol) {
    return GivensArgs{K.H, K.m + 1, (int64_t)(K.m + 1) * K.m, pA, pB, dot_blocks(K.n), maxj, npart, norm_blocks(K.n),
                      K.cs, K.sn, K.m, K.g, K.m + 1, K.beta, K.hist, K.m, K.done, K.kdone, k, tol};
}

void launch_givens(const KrylovState& K, const double* pA, const double* pB, int maxj, const double* npart, int k,
                   double tol, int nrhs, hipStream_t st) {
    givens_kernel<<<nrhs, kThreads, 0, st>>>(givens_args(K, pA, pB, maxj, npart, k, tol));
    LAUNCH_CHECK();
}

void launch_finish(const KrylovState& K, const double* wv, int64_t ldwv, const double* pA, const double* pB, int maxj,
                   const double* npart, int k, double tol, const CSR& B, void* w, int64_t ldw, int prec, int nrhs,
                   int32_t* host_flag, hipStream_t st) {
    const int nbn = (int)blocks_for(K.n), nbw = (int)blocks_for(B.padded_rows);
    const dim3 grid(nbn + nbw + 1, nrhs);
    const GivensArgs ga = givens_args(K, pA, pB, maxj, npart, k, tol);
    if (prec == BAE_PREC_FP64)
        finish_kernel<double><<<grid, kThreads, 0, st>>>(K.V, K.n, K.ld_rhs, wv, ldwv, K.n, nbn, nbw, B.rowptr, B.col,
                                                          B.coef, B.rows, B.padded_rows, (double*)w, ldw, ga,
                                                          host_flag);
    else
        finish_kernel<float><<<grid, kThreads, 0, st>>>(K.V, K.n, K.ld_rhs, wv, ldwv, K.n, nbn, nbw, B.rowptr, B.col,
                                                         B.coef, B.rows, B.padded_rows, (float*)w, ldw, ga,
                                                         host_flag);
    LAUNCH_CHECK();
}

void launch_basis_transform(const double* X, int64_t ldx_vec, int64_t ldx_rhs, int kin, const double* M, int kout,
                            int64_t n, int nrhs, double* out, int64_t ldo_vec, int64_t ldo_rhs, hipStream_t st) {
    if (n == 0 || kout == 0) return;
    basis_transform_kernel<<<dim3(blocks_for(n), nrhs), kThreads, 0, st>>>(X, ldx_vec, ldx_rhs, kin, M, kout, n, out,
                                                                          ldo_vec, ldo_rhs);
    LAUNCH_CHECK();
}

void launch_gmres_init(const double* r0, int64_t ldr, const KrylovState& K, int64_t n, const double* nrm2, int nrhs,
                       hipStream_t st) {
    gmres_init_kernel<<<dim3(blocks_for(std::max<int64_t>(n, 1)), nrhs), kThreads, 0, st>>>(
        r0, ldr, K.V, K.ld_rhs, n, nrm2, K.beta, K.g, K.m + 1, K.done, K.kdone);
    LAUNCH_CHECK();
}

void launch_axpby(double a, const double* x, int64_t ldx, double b, double* y, int64_t ldy, int64_t n, int nrhs,
                  hipStream_t st) {
    if (n == 0) return;
    axpby_kernel<<<dim3(blocks_for(n), nrhs), kThreads, 0, st>>>(a, x, ldx, b, y, ldy, n);
    LAUNCH_CHECK();
}

void launch_gather(const double* x, int64_t ldx, const int32_t* idx, int64_t n, double* y, int64_t ldy, int nrhs,
                   double scale, hipStream_t st) {
    if (n == 0) return;
    gather_kernel<<<dim3(blocks_for(n), nrhs), kThreads, 0, st>>>(x, ldx, idx, n, y, ldy, scale);
    LAUNCH_CHECK();
}

void launch_rhs(const double* g, int64_t ldg, const double* up, int64_t ldu, const int32_t* partner, const double* t,
                int64_t ngp, int64_t ngm, double* b, int64_t ldb, int nrhs, int32_t* bad, hipStream_t st) {
    if (ngm == 0) return;
    rhs_kernel<<<dim3(blocks_for(ngm), nrhs), kThreads, 0, st>>>(g, ldg, up, ldu, partner, t, ngp, ngm, b, ldb, bad);
    LAUNCH_CHECK();
}

void launch_finite_check(const double* x, int64_t ldx, int64_t n, int nrhs, int32_t* bad, hipStream_t st) {
    if (n == 0) return;
    finite_check_kernel<<<dim3(blocks_for(n), nrhs), kThreads, 0, st>>>(x, ldx, n, bad);
    LAUNCH_CHECK();
}

void launch_scatter(const double* x, int64_t ldx, const int32_t* idx, int64_t n, double* y, int64_t ldy, int nrhs,
                    hipStream_t st) {
    if (n == 0) return;
    scatter_kernel<<<dim3(blocks_for(n), nrhs), kThreads, 0, st>>>(x, ldx, idx, n, y, ldy);
    LAUNCH_CHECK();
}

void launch_fill(double* y, int64_t n, double v, hipStream_t st) {
    if (n == 0) return;
    fill_kernel<<<blocks_for(n), kThreads, 0, st>>>(y, n, v);
    LAUNCH_CHECK();
}

void launch_fill_int(int32_t* y, int64_t n, int32_t v, hipStream_t st) {
    if (n == 0) return;
    fill_int_kernel<<<blocks_for(n), kThreads, 0, st>>>(y, n, v);
    LAUNCH_CHECK();
}

void launch_to_float(const double* x, float* y, int64_t n, hipStream_t st) {
    if (n == 0) return;
    to_float_kernel<<<blocks_for(n), kThreads, 0, st>>>(x, y, n);
    LAUNCH_CHECK();
}

}  // namespace bae
