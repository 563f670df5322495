// Fast summation of the LGF sum by FFT convolution (the paper's stated future work, Sec. 3.5
// and Sec. 5): every source and target of one context lies in the box of N+ u E, so the sum
// v(t) = sum_s w(s) G(t - s) is a convolution on that box.  Zero padding to M_d >= 2 e_d - 1
// per axis makes the cyclic convolution on the padded grid exact on the box (Hockney), with
// the kernel sampled at the wrapped offsets: g(i) = G(i) for i < e, G(M - i) for i > M - e.
// G is even in every coordinate, so its transform is real and even: one octant is stored.
//
// Per right-hand side the transform is pruned to where data are: the z transforms run on the
// e0 x e1 rows that hold weights (two real rows per complex FFT) and keep the half spectrum
// k <= M2/2 of each real row (the rest is its conjugate mirror), the y transforms run on
// e0 x (M2/2 + 1) lines, the x transforms on all M1 x (M2/2 + 1) lines fused with the product by
// the kernel's transform and the inverse x transform, which keeps only the e0 planes of the
// box; the inverse y and z transforms keep only the box again.  All passes are FP64 in LDS.
#include <cmath>

#include "conv.hpp"
#include "fft_device.hpp"
#include "lgf_device.hpp"

namespace bae {

namespace {

using namespace fftdev;

constexpr int kConvThreads = kFftThreads;
constexpr int kMaxLinesPerBlock = 32;   // lines_for's cap (packed real rows included)
constexpr int kIt = kFftPoints / kConvThreads;   // elements per thread of a block's lines, at most

__device__ __forceinline__ int64_t idx3(int i, int j, int k, int n1, int n2) { return ((int64_t)i * n1 + j) * n2 + k; }

// Pass 1: forward z transforms of the real rows (i < e0, j < e1) of R [e0][e1][e2], zero-padded
// to M2, two rows per complex FFT (Z = F(a + i b): F a = (Z_k + conj Z_{-k}) / 2,
// F b = (Z_k - conj Z_{-k}) / 2i); the half spectrum k < H2 = M2/2 + 1 into C [e0][M1][H2].
template <int THREADS>
__global__ __launch_bounds__(THREADS, 4) void conv_z_fwd(const double* __restrict__ R, int e0, int e1, int e2,
                                                          int M1, double2* __restrict__ C, const FftDev p, int P,
                                                          const int32_t* __restrict__ skip) {
    extern __shared__ double2 lds[];
    __shared__ int64_t cbase[kMaxLinesPerBlock];   // start of row l0 + pl's half spectrum in C (-1: none)
    if (skip && *skip) return;
    const int M = p.M, nfft = P / 2;
    double2* A = lds;
    double2* tw = A + (int64_t)nfft * M;
    load_roots(p, tw);
    double* Ad = (double*)A;
    const int64_t l0 = (int64_t)xcd_group(blockIdx.x, gridDim.x) * P, nl = (int64_t)e0 * e1;
    const int H = M / 2 + 1;
    if ((int)threadIdx.x < P) {
        const int64_t l = l0 + threadIdx.x;
        cbase[threadIdx.x] = l < nl ? idx3((int)(l / e1), (int)(l % e1), 0, M1, H) : -1;
    }
    for (int e = threadIdx.x; e < nfft * M; e += blockDim.x) A[e] = make_double2(0.0, 0.0);
    __syncthreads();
    const float re2 = rcp_up(e2), rH = rcp_up(H);
    // every load of the thread issued before the first LDS write (one memory latency, not eight)
    {
        double v[kIt];
        int at[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * THREADS;
            at[it] = -1;
            if (e >= P * e2) continue;
            const int pl = fdiv_up(e, re2), k = e - pl * e2;
            if (cbase[pl] < 0) continue;
            v[it] = R[(l0 + pl) * e2 + k];
            at[it] = 2 * ((pl >> 1) * M + k) + (pl & 1);
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it)
            if (at[it] >= 0) Ad[at[it]] = v[it];
        // P e2 can pass kFftPoints by up to P / 2 (e2 <= (M + 1) / 2)
        for (int e = threadIdx.x + kIt * THREADS; e < P * e2; e += THREADS) {
            const int pl = fdiv_up(e, re2), k = e - pl * e2;
            if (cbase[pl] >= 0) Ad[2 * ((pl >> 1) * M + k) + (pl & 1)] = R[(l0 + pl) * e2 + k];
        }
    }
    __syncthreads();
    fft_lds<THREADS, false>(A, nfft, p, tw);
    const double2* Z = A;
    for (int e = threadIdx.x; e < P * H; e += blockDim.x) {
        const int pl = fdiv_up(e, rH), k = e - pl * H;
        const int64_t cb = cbase[pl];
        if (cb < 0) continue;
        const double2* z = Z + (int64_t)(pl >> 1) * M;
        const double2 a = z[k], b = z[k == 0 ? 0 : M - k];
        // b is conjugated: conj(b) = (b.x, -b.y)
        const double2 X = (pl & 1) ? make_double2(0.5 * (a.y + b.y), -0.5 * (a.x - b.x))
                                   : make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
        C[cb + k] = X;
    }
}

// Transforms of complex lines along a strided axis of C: line l, element n at
// (l / lin) sout + (l % lin) + n sline.  mode 0: forward, elements n < nload loaded (zero
// beyond), n < nstore stored; mode 1: forward, times the kernel's transform, inverse (the x
// pass; n < nload loaded and stored); mode 2: inverse, all M loaded, n < nstore stored.
// P consecutive lines (consecutive in memory) per block.
// MODE is a template parameter so that each kernel holds only the transforms it runs.
template <int THREADS, int MODE>
__global__ __launch_bounds__(THREADS, 4) void conv_lines(double2* __restrict__ C, int64_t nlines, int64_t lin,
                                                          int64_t sout, int64_t sline, int nload, int nstore,
                                                          const FftDev p, int P, const double* __restrict__ ghat,
                                                          int M1, int L2, int H1, int H2,
                                                          const int32_t* __restrict__ skip) {
    extern __shared__ double2 lds[];
    // per line of the block: its first element in C (-1: past the last line) and, in the x
    // pass, its row of the kernel's transform; element n is then lbase + n sline
    __shared__ int64_t lbase[kMaxLinesPerBlock];
    __shared__ int32_t grow[kMaxLinesPerBlock];
    if (skip && *skip) return;
    const int M = p.M;
    double2* A = lds;
    double2* tw = A + (int64_t)P * M;
    load_roots(p, tw);
    const int64_t l0 = (int64_t)xcd_group(blockIdx.x, gridDim.x) * P;
    if ((int)threadIdx.x < P) {
        const int64_t l = l0 + threadIdx.x;
        lbase[threadIdx.x] = l < nlines ? (l / lin) * sout + (l % lin) : -1;
        if constexpr (MODE == 1) {
            // line l = j L2 + k of the x pass on half spectra (L2 = M2/2 + 1, k <= M2/2); the
            // transform is even in every index
            const int j = (int)(l / L2), k = (int)(l % L2);
            grow[threadIdx.x] = min(j, M1 - j) * H2 + k;
        }
    }
    __syncthreads();
    const float rP = rcp_up(P);
    const int nl = MODE == 2 ? M : nload;
    // every load of the thread issued before the first LDS write (one memory latency, not eight)
    {
        double2 v[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * THREADS;
            v[it] = make_double2(0.0, 0.0);
            if (e >= P * M) continue;
            const int n = fdiv_up(e, rP), pl = e - n * P;
            const int64_t lb = lbase[pl];
            if (n < nl && lb >= 0) v[it] = C[lb + n * sline];
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * THREADS;
            if (e >= P * M) continue;
            const int n = fdiv_up(e, rP), pl = e - n * P;
            A[pl * M + n] = v[it];
        }
    }
    __syncthreads();
    double2* Z = A;
    if constexpr (MODE == 2) fft_lds<THREADS, true>(Z, P, p, tw);
    else fft_lds<THREADS, false>(Z, P, p, tw);
    if constexpr (MODE == 1) {   // the product by the kernel's transform, then the inverse
        const int64_t gplane = (int64_t)H1 * H2;
        // the block's lines are consecutive rows of the kernel's transform: the line index
        // fastest, so that a wavefront reads runs of consecutive values of it; all of a
        // thread's loads issued before the first product (P M <= kIt THREADS)
        double g[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * THREADS;
            g[it] = 0.0;
            if (e >= P * M) continue;
            const int n = fdiv_up(e, rP), pl = e - n * P;
            if (lbase[pl] >= 0) g[it] = ghat[min(n, M - n) * gplane + grow[pl]];
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * THREADS;
            if (e >= P * M) continue;
            const int n = fdiv_up(e, rP), pl = e - n * P;
            const double2 z = Z[(int64_t)pl * M + n];
            Z[(int64_t)pl * M + n] = make_double2(g[it] * z.x, g[it] * z.y);
        }
        __syncthreads();
        fft_lds<THREADS, true>(Z, P, p, tw);
    }
    for (int e = threadIdx.x; e < P * nstore; e += blockDim.x) {
        const int n = fdiv_up(e, rP), pl = e - n * P;
        const int64_t lb = lbase[pl];
        if (lb >= 0) C[lb + n * sline] = Z[(int64_t)pl * M + n];
    }
}

// Last pass: inverse z transforms of the rows (i < e0, j < e1) of C (half spectra, the rest the
// conjugate mirror X_k = conj X_{M-k}), two rows per complex FFT (the results are real:
// F^-1(X_a + i X_b) = a + i b), n < e2 kept, times scale, into R.
template <int THREADS>
__global__ __launch_bounds__(THREADS, 4) void conv_z_inv(const double2* __restrict__ C, int e0, int e1, int e2,
                                                          int M1, double* __restrict__ R, const FftDev p, int P,
                                                          double scale, const int32_t* __restrict__ skip) {
    extern __shared__ double2 lds[];
    __shared__ int64_t cbase[kMaxLinesPerBlock];   // start of row l0 + pl's half spectrum in C (-1: none)
    if (skip && *skip) return;
    const int M = p.M, nfft = P / 2;
    double2* A = lds;
    double2* tw = A + (int64_t)nfft * M;
    load_roots(p, tw);
    const int64_t l0 = (int64_t)xcd_group(blockIdx.x, gridDim.x) * P, nl = (int64_t)e0 * e1;
    const int H = M / 2 + 1;
    if ((int)threadIdx.x < P) {
        const int64_t l = l0 + threadIdx.x;
        cbase[threadIdx.x] = l < nl ? idx3((int)(l / e1), (int)(l % e1), 0, M1, H) : -1;
    }
    __syncthreads();
    const float rM = rcp_up(M), re2 = rcp_up(e2);
    // every load of the thread issued before the first LDS write (one memory latency, not four)
    {
        double2 xa[kIt], xb[kIt];   // nfft M <= kFftPoints
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * THREADS;
            xa[it] = xb[it] = make_double2(0.0, 0.0);
            if (e >= nfft * M) continue;
            const int c = fdiv_up(e, rM), k = e - c * M;
            const int kk = k >= H ? M - k : k;
            const int64_t ba = cbase[2 * c], bb = cbase[2 * c + 1];
            if (ba >= 0) xa[it] = C[ba + kk];
            if (bb >= 0) xb[it] = C[bb + kk];
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * THREADS;
            if (e >= nfft * M) continue;
            const int c = fdiv_up(e, rM), k = e - c * M;
            double2 a = xa[it], b = xb[it];
            if (k >= H) {   // the conjugate mirror
                a.y = -a.y;
                b.y = -b.y;
            }
            A[e] = make_double2(a.x - b.y, a.y + b.x);
        }
    }
    __syncthreads();
    fft_lds<THREADS, true>(A, nfft, p, tw);
    const double2* Z = A;
    for (int e = threadIdx.x; e < P * e2; e += blockDim.x) {
        const int pl = fdiv_up(e, re2), k = e - pl * e2;
        if (cbase[pl] < 0) continue;
        const double2 z = Z[(int64_t)(pl >> 1) * M + k];
        R[(l0 + pl) * e2 + k] = scale * ((pl & 1) ? z.y : z.x);
    }
}

// The kernel sampled at the wrapped offsets of the padded grid (full M0 x M1 x M2, complex with
// zero imaginary part), G exactly as the FP64 sum evaluates it.
__global__ void conv_kernel_grid(double2* __restrict__ g, int M0, int M1, int M2, int e0, int e1, int e2,
                                 const double* __restrict__ tab, int tab_r, int full_r, int far_ok) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)M0 * M1 * M2) return;
    const int i = (int)(q / ((int64_t)M1 * M2)), j = (int)((q / M2) % M1), k = (int)(q % M2);
    auto wrap = [](int x, int M, int e) { return x < e ? x : (x > M - e ? M - x : -1); };
    const int a = wrap(i, M0, e0), b = wrap(j, M1, e1), c = wrap(k, M2, e2);
    double v = 0.0;
    if (a >= 0 && b >= 0 && c >= 0) {
        const int hi = max(a, max(b, c)), lo = min(a, min(b, c)), mid = a + b + c - hi - lo;
        if (hi > tab_r && far_ok) {
            const double X = (double)(kQuant * a), Y = (double)(kQuant * b), Z = (double)(kQuant * c);
            v = lgfdev::far_field<double>(X * X, Y * Y, Z * Z);
        } else if (hi <= full_r) {
            v = tab[(int64_t)hi * (hi + 1) * (hi + 2) / 6 + (int64_t)mid * (mid + 1) / 2 + lo];
        } else {
            v = __builtin_nan("");
        }
    }
    g[q] = make_double2(v, 0.0);
}

// The real part of the transformed kernel on the octant [H0][H1][H2].
__global__ void conv_octant(const double2* __restrict__ g, int M1, int M2, int H0, int H1, int H2,
                            double* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)H0 * H1 * H2) return;
    const int a = (int)(q / ((int64_t)H1 * H2)), b = (int)((q / H2) % H1), c = (int)(q % H2);
    out[q] = g[idx3(a, b, c, M1, M2)].x;
}

__global__ void conv_scatter(const double* __restrict__ w, const int32_t* __restrict__ sidx, int64_t ns,
                             double* __restrict__ R) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) R[sidx[s]] = w[s];
}

__global__ void conv_gather(const double* __restrict__ R, const int32_t* __restrict__ tidx, int64_t nt,
                            double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nt) out[t] = R[tidx[t]];
}

__global__ void conv_fill(double* __restrict__ x, int64_t n, const int32_t* __restrict__ skip) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (skip && *skip) return;
    if (i < n) x[i] = 0.0;
}

// Lines per block of a pass (fft_lines_per_block); packed real rows go two to a complex line.
int lines_for(int M, bool packed) {
    const int P = packed ? 2 * fft_lines_per_block(M, 16) : fft_lines_per_block(M, 32);
    if (P > kMaxLinesPerBlock) throw Error{BAE_ERR_ARG, "LGF convolution: too many lines per block"};
    return P;
}

// The passes run 256-thread blocks of a quarter of the points and LDS, four to a compute unit,
// so that some blocks' loads and stores overlap the others' LDS stages (a 1024-thread block at
// 128 VGPRs holds a compute unit alone and runs its phases in series: two blocks of 512 took
// the 257^3 convolution from 1.41 to 1.21 ms, four of 256 to 1.18 ms, eight of 128 took 1.35 ms);
// lines longer than such a block holds (2048)
// keep the 1024-thread blocks.
constexpr int kSplit = 4;
constexpr int kSplitThreads = kConvThreads / kSplit;
constexpr size_t kSplitLdsBytes = kFftLdsBytes / kSplit;
bool split_blocks(int M) { return M <= kFftPointsPerThread * kSplitThreads; }   // one line fits a block
int split_lines(int M, bool packed = false) {
    const int by_points = kFftPointsPerThread * kSplitThreads / M;
    const int by_lds = (int)(kSplitLdsBytes / (16 * (size_t)M)) - 1;
    const int c = std::max(1, std::min(packed ? kMaxLinesPerBlock / 2 : kMaxLinesPerBlock, std::min(by_points, by_lds)));
    return packed ? 2 * c : c;
}

void set_lds_attr() {
    static bool done = false;
    if (done) return;
    for (const void* f : {(const void*)conv_z_fwd<kConvThreads>, (const void*)conv_z_fwd<kSplitThreads>,
                          (const void*)conv_lines<kConvThreads, 0>, (const void*)conv_lines<kSplitThreads, 0>,
                          (const void*)conv_lines<kConvThreads, 1>, (const void*)conv_lines<kSplitThreads, 1>,
                          (const void*)conv_lines<kConvThreads, 2>, (const void*)conv_lines<kSplitThreads, 2>,
                          (const void*)conv_z_inv<kConvThreads>, (const void*)conv_z_inv<kSplitThreads>})
        BAE_HIP_CHECK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFftLdsBytes));
    done = true;
}

// conv_lines for a mode known at run time
template <int THREADS, typename... A>
void launch_lines(int mode, unsigned grid, size_t lds, hipStream_t st, A... args) {
    if (mode == 0) conv_lines<THREADS, 0><<<grid, THREADS, lds, st>>>(args...);
    else if (mode == 1) conv_lines<THREADS, 1><<<grid, THREADS, lds, st>>>(args...);
    else if (mode == 2) conv_lines<THREADS, 2><<<grid, THREADS, lds, st>>>(args...);
    else throw Error{BAE_ERR_ARG, "LGF convolution: unknown line-pass mode"};
}

// C lines along y (i < e0, k < M2; j the element) or x (j < M1, k < M2; i the element)
void run_lines(const ConvPlan& cp, double2* C, int axis, int nload, int nstore, int mode, const int32_t* skip,
               hipStream_t st) {
    const int M1 = cp.M[1], M2 = cp.M[2];
    const FftDev& p = axis == 1 ? cp.fy : cp.fx;
    int64_t nlines, lin, sout, sline;
    const int H2 = cp.H[2];   // the half spectrum along z
    if (axis == 1) {
        nlines = (int64_t)cp.e[0] * H2;
        lin = H2;
        sout = (int64_t)M1 * H2;
        sline = H2;
    } else {
        nlines = (int64_t)M1 * H2;
        lin = nlines;
        sout = 0;
        sline = (int64_t)M1 * H2;
    }
    const bool split = split_blocks(p.M);
    const int P = split ? split_lines(p.M) : lines_for(p.M, false);
    const size_t lds = sizeof(double2) * ((size_t)P + 1) * p.M;
    const unsigned grid = (unsigned)((nlines + P - 1) / P);
    if (split)
        launch_lines<kSplitThreads>(mode, grid, lds, st, C, nlines, lin, sout, sline, nload, nstore, p, P, cp.ghat, M1,
                                    H2, cp.H[1], cp.H[2], skip);
    else
        launch_lines<kConvThreads>(mode, grid, lds, st, C, nlines, lin, sout, sline, nload, nstore, p, P, cp.ghat, M1,
                                   H2, cp.H[1], cp.H[2], skip);
    BAE_HIP_CHECK(hipGetLastError());
}

}  // namespace

int fft_smooth_length(int n) {
    for (int m = std::max(1, n);; ++m) {
        int r = m;
        for (int q : {2, 3, 5})
            while (r % q == 0) r /= q;
        if (r == 1) return m;
    }
}

ConvPlan::~ConvPlan() {
    (void)hipFree(ghat);
    (void)hipFree(R);
    (void)hipFree(C);
}

void ConvPlan::build(const int lo_[3], const int hi_[3], const SumTables& tabs, hipStream_t st) {
    for (int a = 0; a < 3; ++a) {
        lo[a] = lo_[a];
        e[a] = hi_[a] - lo_[a] + 1;
        M[a] = fft_smooth_length(2 * e[a] - 1);
        if (M[a] > kFftMaxLen) throw Error{BAE_ERR_ARG, "LGF convolution: box too long for the LDS FFT"};
        H[a] = M[a] / 2 + 1;
    }
    set_lds_attr();
    fx = fft_plan(M[0], st);
    fy = fft_plan(M[1], st);
    fz = fft_plan(M[2], st);
    const int64_t full = (int64_t)M[0] * M[1] * M[2], oct = (int64_t)H[0] * H[1] * H[2];
    const int64_t box = (int64_t)e[0] * e[1] * e[2], cbytes = (int64_t)e[0] * M[1] * H[2];
    auto dmalloc = [](void** p, size_t n) {
        if (hipMalloc(p, n) != hipSuccess) throw Error{BAE_ERR_OOM, "LGF convolution: device allocation failed"};
    };
    dmalloc((void**)&ghat, sizeof(double) * oct);
    dmalloc((void**)&R, sizeof(double) * box);
    dmalloc((void**)&C, sizeof(double2) * cbytes);
    bytes = sizeof(double) * (oct + box) + sizeof(double2) * cbytes;
    // the kernel's transform: sample, three full passes (z, y, x), keep one octant
    double2* g = nullptr;
    dmalloc((void**)&g, sizeof(double2) * full);
    conv_kernel_grid<<<(unsigned)((full + 255) / 256), 256, 0, st>>>(g, M[0], M[1], M[2], e[0], e[1], e[2],
                                                                      tabs.full64, tabs.tab_r64, tabs.full_r,
                                                                      tabs.far64() ? 1 : 0);
    BAE_HIP_CHECK(hipGetLastError());
    {   // z: rows of the full grid (complex, contiguous)
        const int P = lines_for(M[2], false);
        const int64_t nl = (int64_t)M[0] * M[1];
        conv_lines<kConvThreads, 0><<<(unsigned)((nl + P - 1) / P), kConvThreads, sizeof(double2) * ((size_t)P + 1) * M[2], st>>>(
            g, nl, 1, M[2], 1, M[2], M[2], fz, P, nullptr, M[1], M[2], H[1], H[2], nullptr);
        BAE_HIP_CHECK(hipGetLastError());
    }
    {   // y over every plane, x over every line
        const int P = lines_for(M[1], false);
        const int64_t nl = (int64_t)M[0] * M[2];
        conv_lines<kConvThreads, 0><<<(unsigned)((nl + P - 1) / P), kConvThreads, sizeof(double2) * ((size_t)P + 1) * M[1], st>>>(
            g, nl, M[2], (int64_t)M[1] * M[2], M[2], M[1], M[1], fy, P, nullptr, M[1], M[2], H[1], H[2], nullptr);
        BAE_HIP_CHECK(hipGetLastError());
        const int Px = lines_for(M[0], false);
        const int64_t nlx = (int64_t)M[1] * M[2];
        conv_lines<kConvThreads, 0><<<(unsigned)((nlx + Px - 1) / Px), kConvThreads, sizeof(double2) * ((size_t)Px + 1) * M[0], st>>>(
            g, nlx, nlx, 0, nlx, M[0], M[0], fx, Px, nullptr, M[1], M[2], H[1], H[2], nullptr);
        BAE_HIP_CHECK(hipGetLastError());
    }
    conv_octant<<<(unsigned)((oct + 255) / 256), 256, 0, st>>>(g, M[1], M[2], H[0], H[1], H[2], ghat);
    BAE_HIP_CHECK(hipGetLastError());
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    (void)hipFree(g);
}

void ConvPlan::apply(const double* w, const int32_t* sidx, int64_t ns, const int32_t* tidx, int64_t nt, double* out,
                     double scale, const int32_t* skip, hipStream_t st) {
    const int64_t box = (int64_t)e[0] * e[1] * e[2];
    conv_fill<<<(unsigned)((box + 255) / 256), 256, 0, st>>>(R, box, skip);
    if (ns > 0) conv_scatter<<<(unsigned)((ns + 255) / 256), 256, 0, st>>>(w, sidx, ns, R);
    BAE_HIP_CHECK(hipGetLastError());
    const bool splitz = split_blocks(M[2]);
    const int Pz = splitz ? split_lines(M[2], true) : lines_for(M[2], true);
    const int64_t nrow = (int64_t)e[0] * e[1];
    const size_t ldsz = sizeof(double2) * (size_t)(Pz / 2 + 1) * M[2];   // Pz / 2 complex lines, the roots
    const unsigned gz = (unsigned)((nrow + Pz - 1) / Pz);
    if (splitz) conv_z_fwd<kSplitThreads><<<gz, kSplitThreads, ldsz, st>>>(R, e[0], e[1], e[2], M[1], C, fz, Pz, skip);
    else conv_z_fwd<kConvThreads><<<gz, kConvThreads, ldsz, st>>>(R, e[0], e[1], e[2], M[1], C, fz, Pz, skip);
    BAE_HIP_CHECK(hipGetLastError());
    run_lines(*this, C, 1, e[1], M[1], 0, skip, st);   // y forward: rows j < e1 hold data
    run_lines(*this, C, 0, e[0], e[0], 1, skip, st);   // x forward, product, x inverse
    run_lines(*this, C, 1, M[1], e[1], 2, skip, st);   // y inverse: keep j < e1
    const double norm = scale / ((double)M[0] * M[1] * M[2]);
    if (splitz) conv_z_inv<kSplitThreads><<<gz, kSplitThreads, ldsz, st>>>(C, e[0], e[1], e[2], M[1], R, fz, Pz, norm, skip);
    else conv_z_inv<kConvThreads><<<gz, kConvThreads, ldsz, st>>>(C, e[0], e[1], e[2], M[1], R, fz, Pz, norm, skip);
    BAE_HIP_CHECK(hipGetLastError());
    if (nt > 0) conv_gather<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(R, tidx, nt, out);
    BAE_HIP_CHECK(hipGetLastError());
}

}  // namespace bae
