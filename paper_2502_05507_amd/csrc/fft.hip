// Mixed-radix FFTs in LDS and the sine transforms built on them.
//
// Algorithm 1 solves the finite auxiliary problem G_h (Sec. 2.1: L_h on the interior nodes of
// the box, zero on its boundary) "via FFT".  The sine vectors diagonalise L_h on the box:
// along an axis of N interior nodes the DST-I X_k = sum_{n=1..N} x_n sin(pi n k / (N + 1)).
// Here every DST-I is one complex FFT of length M = 2(N + 1) of the odd extension
// y = (0, x_1..x_N, 0, -x_N..-x_1), whose transform is -2i X; two real lines ride in one
// complex FFT (a in the real part, b in the imaginary part: FFT = -2i X_a + 2 X_b).
//
// The FFT itself is a Stockham autosort transform in LDS (no bit reversal): M factors into
// radices 4, 2, 3, 5 and any remaining primes; stage s with radix R and stride Ns maps input
// j + r M/R (r < R), twiddled by w^(r (j mod Ns) M/(Ns R)), to output
// (j div Ns) Ns R + (j mod Ns) + k Ns after an R-point DFT (w = e^(-2 pi i / M); every root
// comes from one table of M entries).  Radices up to 8 run their DFT in registers; larger
// primes evaluate each output as an R-term sum straight from LDS (O(M R) per stage: such
// lengths are rare, and correct).
//
// Lines along any axis of a row-major [n0][n1][n2] array are gathered by one workgroup each
// group of P lines: along the contiguous axis whole rows, along the others P consecutive
// columns, so every load and store is a run of P (or n2) consecutive doubles.
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "fft.hpp"
#include "fft_device.hpp"

namespace bae {

namespace {

using namespace fftdev;

// Position of element n of line l along `axis` of an [n0][n1][n2] array.
__device__ __forceinline__ int64_t line_at(int axis, int64_t l, int64_t n, int n0, int n1, int n2) {
    (void)n0;
    if (axis == 2) return l * n2 + n;                                       // l = i n1 + j
    if (axis == 1) return (l / n2) * (int64_t)n1 * n2 + (l % n2) + n * n2;  // l = i n2 + k
    return l + n * (int64_t)n1 * n2;                                        // l = j n2 + k
}

// DST-I of every line along `axis` (length N = its extent), in place, times `scale`.  A block
// takes P lines (P even: line pairs share a complex FFT of length p.M = 2(N + 1)).
// With eig.c0 set (the last forward pass, axis 2), each output is also divided by the
// eigenvalue of L_h at its frequency (i, j, k): lambda = (6 + s) - c0[i] - c1[j] - c2[k] with
// c_d[k] = 2 cos(pi (k + 1) / (n_d + 1)) -- the division of the box solve, fused into the pass
// that produces the last frequency index.
struct BoxEigen {
    const double* c0 = nullptr;
    const double* c1 = nullptr;
    const double* c2 = nullptr;
    double shift = 0.0;   // 6 + s
};

constexpr int kMaxDstLines = 32;   // lines_per_block's cap

template <int THREADS>
__global__ __launch_bounds__(THREADS, 4) void dst_axis_kernel(double* __restrict__ x, int axis, int n0, int n1,
                                                                int n2, int64_t nlines, int P, const FftDev p,
                                                                double scale, const BoxEigen eig) {
    extern __shared__ double2 lds[];
    // per line of the block: the position of its element 0 (-1: past the last line) and, in
    // the pass that divides by the eigenvalues, the line's part of them (c0[i] + c1[j]);
    // element n of the line is then at lbase + n stride
    __shared__ int64_t lbase[kMaxDstLines];
    __shared__ double esum[kMaxDstLines];
    const int N = axis == 0 ? n0 : axis == 1 ? n1 : n2;
    const int64_t stride = axis == 2 ? 1 : axis == 1 ? (int64_t)n2 : (int64_t)n1 * n2;
    const int M = p.M;
    const int nfft = P / 2;
    double2* A = lds;
    double2* tw = A + (int64_t)nfft * M;
    load_roots(p, tw);
    const int64_t l0 = (int64_t)xcd_group(blockIdx.x, gridDim.x) * P;
    if ((int)threadIdx.x < P) {
        const int64_t l = l0 + threadIdx.x;
        lbase[threadIdx.x] = l >= nlines ? -1 : line_at(axis, l, 0, n0, n1, n2);
        if (eig.c0 && l < nlines) {   // axis 2: line l = i n1 + j
            const int i = (int)(l / n1), j = (int)(l - (int64_t)i * n1);
            esum[threadIdx.x] = eig.c0[i] + eig.c1[j];
        }
    }
    double* Ad = (double*)A;
    // the two end points of every odd extension are zero
    for (int e = threadIdx.x; e < nfft; e += blockDim.x) {
        A[(int64_t)e * M] = make_double2(0.0, 0.0);
        A[(int64_t)e * M + N + 1] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    const float rN = rcp_up(N), rP = rcp_up(P);
    // element e of the block: line pl, position n (lines consecutive along the contiguous
    // axis, interleaved along the others)
    auto split = [=](int e) -> int2 {
        if (axis == 2) {
            const int pl = fdiv_up(e, rN);
            return make_int2(pl, e - pl * N);
        }
        const int n = fdiv_up(e, rP);
        return make_int2(e - n * P, n);
    };
    // every load of the thread issued before the first LDS write (P N < (P / 2) M <= kFftPoints:
    // at most kIt per thread)
    {
        constexpr int kIt = kFftPointsPerThread;
        double v[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * THREADS;
            v[it] = 0.0;
            if (e >= P * N) continue;
            const int2 q = split(e);
            const int64_t lb = lbase[q.x];
            if (lb >= 0) v[it] = x[lb + q.y * stride];
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * THREADS;
            if (e >= P * N) continue;
            const int2 q = split(e);
            const int c = q.x >> 1, comp = q.x & 1;
            Ad[2 * (c * M + q.y + 1) + comp] = v[it];
            Ad[2 * (c * M + M - q.y - 1) + comp] = -v[it];
        }
    }
    __syncthreads();
    fft_lds<THREADS, false>(A, nfft, p, tw);
    const double2* Z = A;
    const double h = 0.5 * scale;
    for (int e = threadIdx.x; e < P * N; e += blockDim.x) {
        const int2 q = split(e);
        const int pl = q.x, n = q.y;
        const int64_t lb = lbase[pl];
        if (lb < 0) continue;
        const double2 z = Z[(int64_t)(pl >> 1) * M + n + 1];
        double v = (pl & 1) ? h * z.x : -h * z.y;
        if (eig.c0) v /= eig.shift - (esum[pl] + eig.c2[n]);   // axis 2: element n = k
        x[lb + n * stride] = v;
    }
}

// W = chi_{M-} L_h H on the interior nodes (N0 x N1 x N2, offset one node from the full grid
// [n0][n1][n2]): the source of the difference potential G_h[chi_{M-} L_h u_gamma] (Sec. 2.1),
// H the density extended by zero; nodes of the box boundary count as zero.
__global__ void difference_source_kernel(const double* __restrict__ H, const uint8_t* __restrict__ inside, int n1,
                                         int n2, int N0, int N1, int N2, double s, double* __restrict__ W) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N0 * N1 * N2) return;
    const int a = (int)(i / ((int64_t)N1 * N2)), b = (int)((i / N2) % N1), c = (int)(i % N2);
    if (inside[((int64_t)(a + 1) * n1 + (b + 1)) * n2 + (c + 1)]) {
        W[i] = 0.0;
        return;
    }
    const int64_t sa = (int64_t)N1 * N2, sb = N2;
    double v = (6.0 + s) * H[i];
    if (a > 0) v -= H[i - sa];
    if (a + 1 < N0) v -= H[i + sa];
    if (b > 0) v -= H[i - sb];
    if (b + 1 < N1) v -= H[i + sb];
    if (c > 0) v -= H[i - 1];
    if (c + 1 < N2) v -= H[i + 1];
    W[i] = v;
}

struct PlanHolder {
    FftDev dev{};
    double2* tw = nullptr;
    ~PlanHolder() {}   // the table lives until the process ends (plans are shared)
};

std::mutex g_plan_mu;
auto* g_plans = new std::map<std::pair<int, int>, std::unique_ptr<PlanHolder>>();
// c[k] = 2 cos(pi (k + 1) / (N + 1)), k < N, per (device, N): the axis terms of the box
// eigenvalues (kept until the process ends, like the plans)
auto* g_cos = new std::map<std::pair<int, int>, double*>();

const double* eigen_cos(int N, hipStream_t st) {
    int device = 0;
    BAE_HIP_CHECK(hipGetDevice(&device));
    std::lock_guard<std::mutex> lk(g_plan_mu);
    double*& slot = (*g_cos)[{device, N}];
    if (!slot) {
        std::vector<double> c(N);
        for (int k = 0; k < N; ++k)
            c[k] = (double)(2.0L * cosl(3.14159265358979323846264338327950288L * (long double)(k + 1) /
                                        (long double)(N + 1)));
        double* d = nullptr;
        BAE_HIP_CHECK(hipMalloc((void**)&d, sizeof(double) * N));
        BAE_HIP_CHECK(hipMemcpyAsync(d, c.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
        BAE_HIP_CHECK(hipStreamSynchronize(st));
        slot = d;
    }
    return slot;
}

}  // namespace

std::vector<int> fft_factors(int M) {
    std::vector<int> f;
    int r = M;
    while (r % 4 == 0) {
        f.push_back(4);
        r /= 4;
    }
    for (int q : {2, 3, 5})
        while (r % q == 0) {
            f.push_back(q);
            r /= q;
        }
    for (int q = 7; (int64_t)q * q <= r; q += 2)
        while (r % q == 0) {
            f.push_back(q);
            r /= q;
        }
    if (r > 1) f.push_back(r);
    return f;
}

FftDev fft_plan(int M, hipStream_t st) {
    if (M < 1 || M > kFftMaxLen) throw Error{BAE_ERR_ARG, "FFT length out of range"};
    int device = 0;
    BAE_HIP_CHECK(hipGetDevice(&device));
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto& slot = (*g_plans)[{device, M}];
    if (!slot) {
        auto h = std::make_unique<PlanHolder>();
        const std::vector<int> f = fft_factors(M);
        if ((int)f.size() > kFftMaxFactors) throw Error{BAE_ERR_ARG, "FFT length has too many factors"};
        h->dev.M = M;
        h->dev.nf = (int)f.size();
        for (size_t i = 0; i < f.size(); ++i) h->dev.f[i] = f[i];
        std::vector<double2> tw(M);
        for (int t = 0; t < M; ++t) {
            // extended precision keeps every root correct to FP64 rounding
            const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)M;
            tw[t] = make_double2((double)cosl(a), (double)(-sinl(a)));
        }
        BAE_HIP_CHECK(hipMalloc((void**)&h->tw, sizeof(double2) * M));
        BAE_HIP_CHECK(hipMemcpyAsync(h->tw, tw.data(), sizeof(double2) * M, hipMemcpyHostToDevice, st));
        BAE_HIP_CHECK(hipStreamSynchronize(st));
        h->dev.tw = h->tw;
        slot = std::move(h);
    }
    return slot->dev;
}

static int lines_per_block(int M) {
    const int P = 2 * fft_lines_per_block(M, 16);   // two real lines per complex FFT, at most 32
    if (P > kMaxDstLines) throw Error{BAE_ERR_ARG, "sine transform: too many lines per block"};
    return P;
}

// Transforms up to 2048 long run 256-thread blocks of a quarter of the points and LDS, four to
// a compute unit, so that some blocks' loads and stores overlap the others' LDS stages.
constexpr int kDstSplit = 4;
constexpr int kDstSplitThreads = fftdev::kFftThreads / kDstSplit;
static bool dst_split(int M) { return M <= fftdev::kFftPointsPerThread * kDstSplitThreads; }   // one line pair fits a block
static int dst_split_lines(int M) {
    const int by_points = fftdev::kFftPointsPerThread * kDstSplitThreads / M;
    const int by_lds = (int)(kFftLdsBytes / kDstSplit / (16 * (size_t)M)) - 1;
    return 2 * std::max(1, std::min(kMaxDstLines / 2, std::min(by_points, by_lds)));
}

static void dst_axis_eig(double* x, int n0, int n1, int n2, int axis, double scale, const BoxEigen& eig,
                         hipStream_t st) {
    const int N = axis == 0 ? n0 : axis == 1 ? n1 : n2;
    if (N <= 0) return;
    const FftDev p = fft_plan(2 * (N + 1), st);
    const bool split = dst_split(p.M);
    const int P = split ? dst_split_lines(p.M) : lines_per_block(p.M);
    const int64_t nlines = (int64_t)n0 * n1 * n2 / N;
    const size_t lds = sizeof(double2) * (size_t)(P / 2 + 1) * p.M;   // P / 2 complex lines, the roots
    static bool attr = false;
    if (!attr) {
        for (const void* f : {(const void*)dst_axis_kernel<fftdev::kFftThreads>, (const void*)dst_axis_kernel<kDstSplitThreads>})
            BAE_HIP_CHECK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFftLdsBytes));
        attr = true;
    }
    const unsigned blocks = (unsigned)((nlines + P - 1) / P);
    if (split)
        dst_axis_kernel<kDstSplitThreads><<<blocks, kDstSplitThreads, lds, st>>>(x, axis, n0, n1, n2, nlines, P, p, scale, eig);
    else
        dst_axis_kernel<fftdev::kFftThreads><<<blocks, fftdev::kFftThreads, lds, st>>>(x, axis, n0, n1, n2, nlines, P, p,
                                                                                    scale, eig);
    BAE_HIP_CHECK(hipGetLastError());
}

void dst_axis(double* x, int n0, int n1, int n2, int axis, double scale, hipStream_t st) {
    dst_axis_eig(x, n0, n1, n2, axis, scale, BoxEigen{}, st);
}

void difference_source(const double* H, const uint8_t* inside, const int* n, double s, double* W, hipStream_t st) {
    const int N0 = n[0] - 2, N1 = n[1] - 2, N2 = n[2] - 2;
    const int64_t nn = (int64_t)N0 * N1 * N2;
    if (nn <= 0) return;
    difference_source_kernel<<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(H, inside, n[1], n[2], N0, N1, N2, s, W);
    BAE_HIP_CHECK(hipGetLastError());
}

void box_solve_fft(double* x, int n0, int n1, int n2, double s, hipStream_t st) {
    if ((int64_t)n0 * n1 * n2 <= 0) return;
    const double scale = (2.0 / (n0 + 1)) * (2.0 / (n1 + 1)) * (2.0 / (n2 + 1));
    BoxEigen eig;
    eig.c0 = eigen_cos(n0, st);
    eig.c1 = eigen_cos(n1, st);
    eig.c2 = eigen_cos(n2, st);
    eig.shift = 6.0 + s;
    dst_axis(x, n0, n1, n2, 0, 1.0, st);
    dst_axis(x, n0, n1, n2, 1, 1.0, st);
    dst_axis_eig(x, n0, n1, n2, 2, scale, eig, st);   // with the eigenvalue division
    for (int a = 0; a < 3; ++a) dst_axis(x, n0, n1, n2, a, 1.0, st);
}

}  // namespace bae
