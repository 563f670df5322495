// The particular solution on the finite grid (Algorithm 1, first step): u_p = G_h[chi_{M+} f],
// G_h the inverse of the 7-point operator L_h u = (6 + s) u(m) - sum of the six neighbours on
// the N^3 interior nodes of the box with u = 0 on its boundary nodes (Sec. 2.1).
//
// The sine vectors diagonalise L_h: with the DST-I matrix S[m][l] = sin(pi (m+1)(l+1) / (N+1))
// (symmetric, S S = (N+1)/2 I) applied along each axis,
//   u = (2/(N+1))^3 S_3 S_2 S_1 [ (S_1 S_2 S_3 q) / lambda ],
//   lambda(k) = (6 + s) - 2 (cos(pi k1/(N+1)) + cos(pi k2/(N+1)) + cos(pi k3/(N+1))).
// Each S along an axis is a dense contraction: the grid viewed as an N x N^2 matrix times S
// from the left (a GEMM on the FP64 matrix cores), then a transpose to N^2 x N that rotates the axes, so
// three passes transform every axis and return the original order.  O(N^4) work: at
// N = 255, six passes of 8.5e9 flops.
#include "internal.hpp"
#include "ops.hpp"

namespace bae {
namespace {

constexpr int kTile = 64;     // GEMM output tile (rows x columns)
constexpr int kTileK = 16;    // contraction chunk
constexpr int kTr = 32;       // transpose tile

__global__ void dst_matrix_kernel(int N, double* __restrict__ S) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * N) return;
    const int m = (int)(i / N), l = (int)(i % N);
    // reduce (m+1)(l+1) modulo 2(N+1) first, so the sine's argument stays below 2 pi
    const int64_t r = ((int64_t)(m + 1) * (l + 1)) % (2 * (int64_t)(N + 1));
    S[i] = sin(M_PI * (double)r / (double)(N + 1));
}

// C[m][p] = sum_l S[m][l] B[l][p], m < N, p < P; S N x N, B and C N x P, row-major, on the
// FP64 matrix cores (v_mfma_f64_16x16x4).  A block of 4 wavefronts owns a 64 x 64 tile of C,
// each wavefront 32 x 32 as 2 x 2 MFMA tiles; chunks of 16 along l are staged in LDS, the
// next chunk's loads in flight while the current one is contracted.
// Operand layouts (16x16x4 f64, measured on gfx950): A[i][k] in lane 16k + i, B[k][j] in
// lane 16k + j; D[i][j] in lane 16v' + j, element v, with i = v' + 4v.
using V4d = __attribute__((__vector_size__(4 * sizeof(double)))) double;
__global__ __launch_bounds__(256) void gemm_s_kernel(const double* __restrict__ S, const double* __restrict__ B,
                                                     double* __restrict__ C, int N, int64_t P) {
    __shared__ double As[kTileK][kTile + 1];   // As[l][m] = S[m0 + m][l0 + l]
    __shared__ double Bs[kTileK][kTile + 1];   // Bs[l][p] = B[l0 + l][p0 + p]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int wm = (w >> 1) * 32, wp = (w & 1) * 32;
    const int m0 = blockIdx.y * kTile;
    const int64_t p0 = (int64_t)blockIdx.x * kTile;
    V4d acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][u][v] = 0.0;
    // the chunk's operands: 4 + 4 values per thread, loaded one chunk ahead of their use
    double ra[4], rb[4];
    auto load = [&](int l0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = threadIdx.x + 256 * r;
            const int m = e / kTileK, l = e % kTileK;
            ra[r] = (m0 + m < N && l0 + l < N) ? S[(int64_t)(m0 + m) * N + l0 + l] : 0.0;
            const int lb = e / kTile, pb = e % kTile;
            rb[r] = (l0 + lb < N && p0 + pb < P) ? B[(int64_t)(l0 + lb) * P + p0 + pb] : 0.0;
        }
    };
    load(0);
    for (int l0 = 0; l0 < N; l0 += kTileK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = threadIdx.x + 256 * r;
            As[e % kTileK][e / kTileK] = ra[r];
            Bs[e / kTile][e % kTile] = rb[r];
        }
        __syncthreads();
        if (l0 + kTileK < N) load(l0 + kTileK);
#pragma unroll
        for (int kk = 0; kk < kTileK; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) a[t] = As[kk + kq][wm + 16 * t + i];
#pragma unroll
            for (int u = 0; u < 2; ++u) b[u] = Bs[kk + kq][wp + 16 * u + i];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wm + 16 * t + kq + 4 * v;
                const int64_t p = p0 + wp + 16 * u + i;
                if (m < N && p < P) C[(int64_t)m * P + p] = acc[t][u][v];
            }
}

// out[p][m] = in[m][p] for an R x Q row-major input (R = N rows, Q = N^2 columns).
__global__ __launch_bounds__(kTr * 8) void transpose_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                            int64_t R, int64_t Q) {
    __shared__ double t[kTr][kTr + 1];
    const int64_t q0 = (int64_t)blockIdx.x * kTr, r0 = (int64_t)blockIdx.y * kTr;
    const int tx = threadIdx.x % kTr, ty = threadIdx.x / kTr;
    for (int y = ty; y < kTr; y += 8) {
        const int64_t r = r0 + y, q = q0 + tx;
        t[y][tx] = (r < R && q < Q) ? in[r * Q + q] : 0.0;
    }
    __syncthreads();
    for (int y = ty; y < kTr; y += 8) {
        const int64_t q = q0 + y, r = r0 + tx;
        if (q < Q && r < R) out[q * R + r] = t[tx][y];
    }
}

// x[k1][k2][k3] *= scale / lambda(k)  (the three axes in any order: lambda is symmetric)
__global__ void eigen_scale_kernel(double* __restrict__ x, int N, double s, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n3 = (int64_t)N * N * N;
    if (i >= n3) return;
    const int k1 = (int)(i / ((int64_t)N * N)), k2 = (int)((i / N) % N), k3 = (int)(i % N);
    const double w = M_PI / (double)(N + 1);
    const double lam = (6.0 + s) - 2.0 * (cos(w * (k1 + 1)) + cos(w * (k2 + 1)) + cos(w * (k3 + 1)));
    x[i] *= scale / lam;
}

// dst[r][idx[i]] = src[r][i]: the source values at M+ into the zeroed interior grid
__global__ void scatter_kernel(const double* __restrict__ src, int64_t lds, const int32_t* __restrict__ idx,
                               int64_t n, double* __restrict__ dst, int64_t ldd) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i < n) dst[r * ldd + idx[i]] = src[r * lds + i];
}

// the three axis passes: x <- S along every axis (x and tmp: N^3 each; result in x)
void dst3(const double* S, double* x, double* tmp, int N, hipStream_t st) {
    const int64_t P = (int64_t)N * N;
    const dim3 gg((unsigned)((P + kTile - 1) / kTile), (unsigned)((N + kTile - 1) / kTile));
    const dim3 tg((unsigned)((P + kTr - 1) / kTr), (unsigned)((N + kTr - 1) / kTr));
    for (int pass = 0; pass < 3; ++pass) {
        gemm_s_kernel<<<gg, 256, 0, st>>>(S, x, tmp, N, P);
        transpose_kernel<<<tg, kTr * 8, 0, st>>>(tmp, x, N, P);
    }
    BAE_HIP_CHECK(hipGetLastError());
}

}  // namespace

// u = G_h q on the N^3 interior nodes, in place in x (one RHS); S: the N x N DST-I matrix
// (box_dst_matrix); tmp: N^3 scratch.
void box_solve(const double* S, double* x, double* tmp, int N, double s, hipStream_t st) {
    if (N <= 0) return;
    dst3(S, x, tmp, N, st);
    const int64_t n3 = (int64_t)N * N * N;
    const double c = 2.0 / (double)(N + 1);
    eigen_scale_kernel<<<(unsigned)((n3 + 255) / 256), 256, 0, st>>>(x, N, s, c * c * c);
    BAE_HIP_CHECK(hipGetLastError());
    dst3(S, x, tmp, N, st);
}

void box_scatter(const double* src, int64_t lds, const int32_t* idx, int64_t n, double* dst, int64_t ldd, int nrhs,
                 hipStream_t st) {
    if (n <= 0) return;
    scatter_kernel<<<dim3((unsigned)((n + 255) / 256), nrhs), 256, 0, st>>>(src, lds, idx, n, dst, ldd);
    BAE_HIP_CHECK(hipGetLastError());
}

void box_dst_matrix(int N, double* S, hipStream_t st) {
    if (N <= 0) return;
    dst_matrix_kernel<<<(unsigned)(((int64_t)N * N + 255) / 256), 256, 0, st>>>(N, S);
    BAE_HIP_CHECK(hipGetLastError());
}

}  // namespace bae
