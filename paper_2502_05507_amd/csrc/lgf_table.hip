// FP64 generation of the free-space lattice Green's function table on the GPU.
//
// Paper Sec. 2.2: with L = (6+s) I - sum of the 6 shifts (s = sigma h^2), the LGF is
//   G_s(a,b,c) = int_0^inf exp(-(6+s) t) I_a(2t) I_b(2t) I_c(2t) dt
//              = int_0^inf exp(-s t) It_a(2t) It_b(2t) It_c(2t) dt,  It_n(x) = exp(-x) I_n(x),
// (Watson's transformation of eq. "lgf"; the sigma factor enters as exp(-s t)).  As in the
// paper the integral is split at T*: a quadrature rule on [0, T*] and the large-argument
// series of I_n (Abramowitz-Stegun 9.7.1) integrated term by term beyond T*.
//
// Design for the GPU (not from the paper):
//   * quadrature in u = ln t, composite 20-point Gauss-Legendre (width-4 panels on
//     [-40,-8], width-1.5 panels on [-8, ln T*]), T* = 8 R^2 + 64 so that every factor's
//     asymptotic series has ratio <= 1/32 beyond T*;
//   * one thread per quadrature node computes It_n(2 t_q), n = 0..R, by the backward
//     recurrence of the ratios r_n = I_n / I_{n-1} = x / (2n + x r_{n+1}) (Miller's method in
//     ratio form, no overflow), normalised by It_0 + 2 sum_{n>=1} It_n = 1;
//   * one thread per table entry forms the separable sum sum_q W_q B_q[a] B_q[b] B_q[c]
//     (B stored node-major so consecutive a are coalesced) plus the tail series.
// Table layout: sorted triple a <= b <= c at index c(c+1)(c+2)/6 + b(b+1)/2 + a (the
// 1/48 symmetry of Sec. 4).
#include <array>
#include <cmath>
#include <mutex>

#include "internal.hpp"

namespace bae {

namespace {

constexpr int kGL = 20;          // Gauss-Legendre points per panel
constexpr int kTail = 10;        // asymptotic terms per Bessel factor
constexpr double kULo = -40.0;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // final derivative at the converged node
                p0 = 1.0;
                p1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                const double d = n * (z * p1 - p0) / (z * z - 1.0);
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * d * d);
                break;
            }
        }
    }
}

struct TailParams {
    double J[3 * kTail + 1];   // (4 pi)^-3/2 2^-k int_T^inf e^{-st} t^{-3/2-k} dt
};

// The composite rule in u = ln t: kGL-point panels of width 4 on [kULo, -8] (n_lo of them),
// then of width 1.5 from -8, the last one ending at u_hi = ln T* (n_hi of them).
struct Rule {
    double gx[kGL], gw[kGL];   // Gauss-Legendre on [-1, 1]
    double s, u_hi;
    int n_lo, n_hi;
};

// Node q of the rule: t_q = e^u and the weight of dt = t du with the factor e^{-s t}.
__global__ void nodes_kernel(const Rule rule, int Q, double* __restrict__ t, double* __restrict__ w) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const int p = q / kGL, i = q % kGL;
    double lo, hi;
    if (p < rule.n_lo) {
        lo = kULo + 4.0 * p;
        hi = p + 1 < rule.n_lo ? lo + 4.0 : -8.0;
    } else {
        const int k = p - rule.n_lo;
        lo = -8.0 + 1.5 * k;
        hi = k + 1 < rule.n_hi ? lo + 1.5 : rule.u_hi;
    }
    const double u = 0.5 * (hi - lo) * rule.gx[i] + 0.5 * (hi + lo);
    const double tq = exp(u);
    t[q] = tq;
    w[q] = 0.5 * (hi - lo) * rule.gw[i] * tq * exp(-rule.s * tq);
}

// int_T^inf exp(-s t) t^{-3/2-k} dt for k = 0..kmax (host).
void tail_moments(double s, double T, int kmax, double* J) {
    if (s == 0.0) {
        for (int k = 0; k <= kmax; ++k) J[k] = std::pow(T, -(k + 0.5)) / (k + 0.5);
        return;
    }
    // s^{k+1/2} Gamma(-k-1/2, sT); Gamma(a-1,x) = (Gamma(a,x) - x^{a-1} e^{-x})/(a-1)
    const double x = s * T;
    double g = std::sqrt(M_PI) * std::erfc(std::sqrt(x));  // Gamma(1/2, x)
    double a = 0.5;
    for (int k = 0; k <= kmax; ++k) {
        g = (g - std::pow(x, a - 1.0) * std::exp(-x)) / (a - 1.0);
        a -= 1.0;
        J[k] = std::pow(s, k + 0.5) * g;
    }
}

__global__ void bessel_kernel(const double* __restrict__ t, int Q, int R, double* __restrict__ B) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const double x = 2.0 * t[q];
    double* row = B + (int64_t)q * (R + 1);
    const int nstart = R + 60 + (int)(10.0 * sqrt(x));
    double r = 0.0, S = 0.0;
    for (int n = nstart; n >= 1; --n) {
        r = x / (2.0 * n + x * r);
        S = r * (1.0 + S);
        if (n <= R) row[n] = r;
    }
    double In = 1.0 / (1.0 + 2.0 * S);
    row[0] = In;
    for (int n = 1; n <= R; ++n) {
        In *= row[n];
        row[n] = In;
    }
}

__device__ inline int64_t tetra(int64_t c) { return c * (c + 1) * (c + 2) / 6; }

// alpha_k(n): It_n(x) ~ (2 pi x)^{-1/2} sum_k alpha_k x^{-k}; evaluated at x = 2t the
// factor 2^-k is folded into J.
__device__ inline void hankel(int n, double* a) {
    const double mu = 4.0 * n * (double)n;
    a[0] = 1.0;
    for (int k = 1; k <= kTail; ++k) a[k] = a[k - 1] * (-(mu - (2.0 * k - 1.0) * (2.0 * k - 1.0))) / (8.0 * k);
}

__global__ void table_kernel(const double* __restrict__ B, const double* __restrict__ W, int Q, int R,
                             int64_t E, TailParams tp, double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int64_t c = (int64_t)cbrt(6.0 * (double)e);
    while (c > 0 && tetra(c) > e) --c;
    while (tetra(c + 1) <= e) ++c;
    const int64_t rem = e - tetra(c);
    int64_t b = (int64_t)((sqrt(8.0 * (double)rem + 1.0) - 1.0) * 0.5);
    while (b > 0 && b * (b + 1) / 2 > rem) --b;
    while ((b + 1) * (b + 2) / 2 <= rem) ++b;
    const int64_t a = rem - b * (b + 1) / 2;

    double acc = 0.0;
    const int ld = R + 1;
    for (int q = 0; q < Q; ++q) {
        const double* row = B + (int64_t)q * ld;
        acc = fma(W[q] * row[a], row[b] * row[c], acc);
    }
    double ha[kTail + 1], hb[kTail + 1], hc[kTail + 1];
    hankel((int)a, ha);
    hankel((int)b, hb);
    hankel((int)c, hc);
    double tail = 0.0;
    for (int i = 0; i <= kTail; ++i)
        for (int j = 0; j <= kTail; ++j) {
            const double aij = ha[i] * hb[j];
            double s = 0.0;
            for (int l = 0; l <= kTail; ++l) s = fma(hc[l], tp.J[i + j + l], s);
            tail = fma(aij, s, tail);
        }
    out[e] = acc + tail;
}

}  // namespace

int64_t table_size(int R) { return (int64_t)(R + 1) * (R + 2) * (R + 3) / 6; }

// Host part of the rule for radius R (no heap allocation): T* = 8 R^2 + 64.
static void make_rule(double s, int R, Rule& rule, TailParams& tp, int& Q) {
    const double T = 8.0 * R * (double)R + 64.0;
    rule.s = s;
    rule.u_hi = std::log(T);
    gauss_legendre(kGL, rule.gx, rule.gw);
    rule.n_lo = 0;
    for (double u = kULo; u < -8.0 - 1e-12; u += 4.0) rule.n_lo++;
    rule.n_hi = 0;
    for (double u = -8.0; u < rule.u_hi - 1e-9; u += 1.5) rule.n_hi++;
    Q = (rule.n_lo + rule.n_hi) * kGL;
    double J[3 * kTail + 1];
    tail_moments(s, T, 3 * kTail, J);
    const double c0 = std::pow(4.0 * M_PI, -1.5);
    for (int k = 0; k <= 3 * kTail; ++k) tp.J[k] = c0 * std::ldexp(J[k], -k);
}

// The three launches on `stream`; scratch: 2 Q + Q (R + 1) doubles (nodes, weights, the
// scaled Bessel values B[q][n]).
static void launch_table(const Rule& rule, const TailParams& tp, int Q, int R, double* scratch, double* out,
                         hipStream_t stream) {
    double* dt = scratch;
    double* dw = scratch + Q;
    double* dB = scratch + 2 * (int64_t)Q;
    nodes_kernel<<<(Q + 63) / 64, 64, 0, stream>>>(rule, Q, dt, dw);
    BAE_HIP_CHECK(hipGetLastError());
    bessel_kernel<<<(Q + 63) / 64, 64, 0, stream>>>(dt, Q, R, dB);
    BAE_HIP_CHECK(hipGetLastError());
    const int64_t E = table_size(R);
    table_kernel<<<(unsigned)((E + 255) / 256), 256, 0, stream>>>(dB, dw, Q, R, E, tp, out);
    BAE_HIP_CHECK(hipGetLastError());
}

void lgf_table_generate(double s, int R, double* out, hipStream_t stream) {
    Rule rule;
    TailParams tp;
    int Q = 0;
    make_rule(s, R, rule, tp, Q);
    double* scratch = nullptr;
    if (hipMalloc((void**)&scratch, sizeof(double) * (2 * (int64_t)Q + (int64_t)Q * (R + 1))) != hipSuccess)
        throw Error{BAE_ERR_OOM, "LGF table scratch allocation failed"};
    try {
        launch_table(rule, tp, Q, R, scratch, out, stream);
    } catch (...) {
        (void)hipStreamSynchronize(stream);
        (void)hipFree(scratch);
        throw;
    }
    BAE_HIP_CHECK(hipStreamSynchronize(stream));   // the scratch must outlive the kernels
    BAE_HIP_CHECK(hipFree(scratch));
}

// ------------------------------------------------------------------ allocation-free form
// For callers that cannot allocate (graph capture, serving loops): the same kernels with
// their scratch in a file-scope device array that each GPU holds until the process ends.
// Host code reaches it only through the address hipGetSymbolAddress returns on that
// device; the array's own name is a host-side stand-in there.
constexpr int kNoAllocQMax = 540;   // nodes of the rule for any R <= 4096 (at most 520)
constexpr int64_t kNoAllocDoubles = 2 * (int64_t)kNoAllocQMax + (int64_t)kNoAllocQMax * (kNoAllocMaxR + 1);
static __device__ __align__(256) double scratch[kNoAllocDoubles];   // 8.9 MB

static std::mutex g_scratch_mu;
static std::array<double*, 64> g_scratch_ptr{};   // per device ordinal

static double* scratch_on(int device) {
    if (device < 0 || device >= (int)g_scratch_ptr.size()) throw Error{BAE_ERR_ARG, "device ordinal out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // this device's copy
        if (e != hipSuccess || !p)
            throw Error{BAE_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(e)};
        g_scratch_ptr[device] = (double*)p;
    }
    return g_scratch_ptr[device];
}

void lgf_table_generate_noalloc(double s, int R, double* out, hipStream_t stream) {
    if (R > kNoAllocMaxR)
        throw Error{BAE_ERR_ARG, "bae_lgf_table_noalloc: R = " + std::to_string(R) + " exceeds its scratch (R <= " +
                                     std::to_string(kNoAllocMaxR) + ")"};
    Rule rule;
    TailParams tp;
    int Q = 0;
    make_rule(s, R, rule, tp, Q);
    if (Q > kNoAllocQMax) throw Error{BAE_ERR_ARG, "bae_lgf_table_noalloc: quadrature rule exceeds its scratch"};
    int device = 0;
    BAE_HIP_CHECK(hipGetDevice(&device));
    launch_table(rule, tp, Q, R, scratch_on(device), out, stream);
}

}  // namespace bae
