// Device side of the LDS FFT (shared by the sine transforms and the LGF convolution).
#pragma once

#include "fft.hpp"

namespace bae {
namespace fftdev {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// the table root w^t = e^(-2 pi i t / M), conjugated for the inverse transform
__device__ __forceinline__ double2 root(const FftDev& p, int t, bool inv) {
    const double2 w = p.tw[t];
    return inv ? make_double2(w.x, -w.y) : w;
}
// multiplication by -i (forward) or +i (inverse)
__device__ __forceinline__ double2 rot(double2 a, bool inv) {
    return inv ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

constexpr int kRegRadix = 8;   // radices up to this run their DFT in registers

// `count` FFTs of length p.M stored one after another at src (LDS); ping-pong with dst.
// Returns the buffer that holds the result.  Every thread of the block must call it.
static __device__ __noinline__ double2* fft_lds(double2* src, double2* dst, int count, const FftDev& p, bool inv) {
    const int M = p.M;
    int Ns = 1;
    for (int s = 0; s < p.nf; ++s) {
        const int R = p.f[s];
        const int m = M / R;              // butterflies per line
        const int tstep = M / (Ns * R);   // root index of the twiddle step
        if (R <= kRegRadix) {
            for (int e = threadIdx.x; e < count * m; e += blockDim.x) {
                const int c = e / m, j = e - c * m;
                const double2* in = src + (int64_t)c * M;
                double2* out = dst + (int64_t)c * M;
                const int jm = j % Ns;
                double2 v[kRegRadix];
                for (int r = 0; r < R; ++r) {
                    v[r] = in[j + r * m];
                    if (r > 0 && jm > 0) v[r] = cmul(v[r], root(p, (r * jm * tstep) % M, inv));
                }
                const int o = (j / Ns) * Ns * R + jm;
                if (R == 2) {
                    out[o] = cadd(v[0], v[1]);
                    out[o + Ns] = csub(v[0], v[1]);
                } else if (R == 4) {
                    const double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
                    const double2 c2 = cadd(v[1], v[3]), d = rot(csub(v[1], v[3]), inv);
                    out[o] = cadd(a, c2);
                    out[o + Ns] = cadd(b, d);
                    out[o + 2 * Ns] = csub(a, c2);
                    out[o + 3 * Ns] = csub(b, d);
                } else {
                    // R-point DFT with the table: X_k = sum_r v_r w^(r k M / R)
                    const int rs = M / R;
                    for (int k = 0; k < R; ++k) {
                        double2 acc = v[0];
                        for (int r = 1; r < R; ++r) acc = cadd(acc, cmul(v[r], root(p, ((r * k) % R) * rs, inv)));
                        out[o + k * Ns] = acc;
                    }
                }
            }
        } else {
            // large prime radix: each output directly, X = sum_r in[j + r m] w^(r base)
            for (int e = threadIdx.x; e < count * M; e += blockDim.x) {
                const int c = e / M, q = e - c * M;
                const int k = q / m, j = q - k * m;
                const double2* in = src + (int64_t)c * M;
                double2* out = dst + (int64_t)c * M;
                const int jm = j % Ns;
                const int base = (jm * tstep + k * (M / R)) % M;
                double2 acc = in[j];
                int t = 0;
                for (int r = 1; r < R; ++r) {
                    t += base;
                    if (t >= M) t -= M;
                    acc = cadd(acc, cmul(in[j + r * m], root(p, t, inv)));
                }
                out[(j / Ns) * Ns * R + jm + k * Ns] = acc;
            }
        }
        __syncthreads();
        double2* x = src;
        src = dst;
        dst = x;
        Ns *= R;
    }
    return src;
}

}  // namespace fftdev
}  // namespace bae
