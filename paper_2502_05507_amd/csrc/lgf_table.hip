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
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace bae {

namespace {

constexpr int kGL = 20;          // Gauss-Legendre points per panel
constexpr int kTail = 10;        // asymptotic terms per Bessel factor
constexpr double kULo = -40.0;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
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

void lgf_table_generate(double s, int R, double* out, hipStream_t stream) {
    const double T = 8.0 * R * (double)R + 64.0;
    const double uhi = std::log(T);
    std::vector<double> gx, gw;
    gauss_legendre(kGL, gx, gw);
    std::vector<double> edges;
    for (double u = kULo; u < -8.0 - 1e-12; u += 4.0) edges.push_back(u);
    for (double u = -8.0; u < uhi - 1e-9; u += 1.5) edges.push_back(u);
    edges.push_back(uhi);
    std::vector<double> tq, wq;
    for (size_t p = 0; p + 1 < edges.size(); ++p) {
        const double lo = edges[p], hi = edges[p + 1];
        for (int i = 0; i < kGL; ++i) {
            const double u = 0.5 * (hi - lo) * gx[i] + 0.5 * (hi + lo);
            const double t = std::exp(u);
            tq.push_back(t);
            wq.push_back(0.5 * (hi - lo) * gw[i] * t * std::exp(-s * t));  // dt = t du, e^{-st}
        }
    }
    const int Q = (int)tq.size();
    TailParams tp;
    double J[3 * kTail + 1];
    tail_moments(s, T, 3 * kTail, J);
    const double c0 = std::pow(4.0 * M_PI, -1.5);
    for (int k = 0; k <= 3 * kTail; ++k) tp.J[k] = c0 * std::ldexp(J[k], -k);

    double *dt = nullptr, *dw = nullptr, *dB = nullptr;
    if (hipMalloc((void**)&dt, sizeof(double) * Q) != hipSuccess ||
        hipMalloc((void**)&dw, sizeof(double) * Q) != hipSuccess ||
        hipMalloc((void**)&dB, sizeof(double) * (int64_t)Q * (R + 1)) != hipSuccess) {
        (void)hipFree(dt);
        (void)hipFree(dw);
        throw Error{BAE_ERR_OOM, "LGF table scratch allocation failed"};
    }
    BAE_HIP_CHECK(hipMemcpyAsync(dt, tq.data(), sizeof(double) * Q, hipMemcpyHostToDevice, stream));
    BAE_HIP_CHECK(hipMemcpyAsync(dw, wq.data(), sizeof(double) * Q, hipMemcpyHostToDevice, stream));
    bessel_kernel<<<(Q + 63) / 64, 64, 0, stream>>>(dt, Q, R, dB);
    BAE_HIP_CHECK(hipGetLastError());
    const int64_t E = table_size(R);
    table_kernel<<<(unsigned)((E + 255) / 256), 256, 0, stream>>>(dB, dw, Q, R, E, tp, out);
    BAE_HIP_CHECK(hipGetLastError());
    // scratch and the pageable host vectors must outlive the kernels
    BAE_HIP_CHECK(hipStreamSynchronize(stream));
    BAE_HIP_CHECK(hipFree(dB));
    BAE_HIP_CHECK(hipFree(dw));
    BAE_HIP_CHECK(hipFree(dt));
}

}  // namespace bae
