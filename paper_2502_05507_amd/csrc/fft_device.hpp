// Device side of the LDS FFT (shared by the sine transforms and the LGF convolution).
//
// Stockham autosort stages in LDS: stage s with radix R and stride Ns maps input j + r M/R
// (r < R), twiddled by w^(r (j mod Ns) M/(Ns R)), to output (j div Ns) Ns R + (j mod Ns) + k Ns
// after an R-point DFT (w = e^(-2 pi i / M)); all inputs of a stage are read into registers
// before any output is written, so one LDS buffer serves.  Radices 2, 3, 4 and 5 have their butterflies
// written out, in registers; any other prime evaluates each output as an R-term sum straight
// from LDS.  The root table is staged in LDS by the caller.  The direction is a template
// parameter, so conjugated roots and the rotations by -i or +i fold into sign modifiers.
// Index divisions by stage constants go through a float reciprocal rounded up (below).
#pragma once

#include "fft.hpp"

namespace bae {
namespace fftdev {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(s * a.x, s * a.y); }
// the root w^t, conjugated for the inverse transform
template <bool INV>
__device__ __forceinline__ double2 root(const double2* tw, int t) {
    const double2 w = tw[t];
    return INV ? make_double2(w.x, -w.y) : w;
}
// multiplication by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ double2 rot(double2 a) {
    return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}
// 1/d rounded up: the hardware reciprocal (within one ulp) times 1 + 2^-16.  For 1 <= d <= 8192
// and 0 <= e < 2^14 the product e rcp_up(d), rounded to float, lies in [e/d, floor(e/d) + 1),
// so its truncation is e div d with no correction step: the excess over e/d, below
// (e/d) 2^-15, is less than 1/d, the least distance from e/d up to the next integer.  Checked
// exhaustively over that range with reciprocals up to two ulps either side of 1/d.
__device__ __forceinline__ float rcp_up(int d) { return __builtin_amdgcn_rcpf((float)d) * (1.0f + 0x1p-16f); }
__device__ __forceinline__ int fdiv_up(int e, float rd) { return (int)((float)e * rd); }

template <int R, bool INV>
__device__ __forceinline__ void butterfly(double2 (&v)[R]) {
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
        const double2 c = cadd(v[1], v[3]), d = rot<INV>(csub(v[1], v[3]));
        v[0] = cadd(a, c);
        v[1] = cadd(b, d);
        v[2] = csub(a, c);
        v[3] = csub(b, d);
    } else if constexpr (R == 3) {
        constexpr double s3 = 0.86602540378443864676;   // sin(2 pi / 3)
        const double2 a = cadd(v[1], v[2]);
        const double2 t = make_double2(v[0].x - 0.5 * a.x, v[0].y - 0.5 * a.y);
        const double2 d = rot<INV>(cscale(csub(v[1], v[2]), s3));
        v[0] = cadd(v[0], a);
        v[1] = cadd(t, d);
        v[2] = csub(t, d);
    } else if constexpr (R == 5) {
        constexpr double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;   // cos(2pi/5), cos(4pi/5)
        constexpr double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;    // sin(2pi/5), sin(4pi/5)
        const double2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
        const double2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        const double2 x0 = v[0];
        const double2 p1 = make_double2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
        const double2 p2 = make_double2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
        const double2 q1 = rot<INV>(make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
        const double2 q2 = rot<INV>(make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
        v[0] = cadd(x0, cadd(a1, a2));
        v[1] = cadd(p1, q1);
        v[4] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[3] = csub(p2, q2);
    }
}

// In-place stages: a block of kFftThreads threads holds `count` lines of length M (count M <=
// kFftPoints) in one LDS buffer; every thread reads its butterflies' inputs into registers,
// the block synchronises, and the outputs overwrite the buffer.
constexpr int kFftThreads = 1024;
constexpr int kFftPoints = 8192;                         // count * M per block at most

// THREADS: the block size; a block holds at most kFftPointsPerThread * THREADS points.
constexpr int kFftPointsPerThread = kFftPoints / kFftThreads;

// tstep = M / (Ns R), passed by the caller, which forms it without a division.
template <int R, int THREADS, bool INV>
__device__ __forceinline__ void stage(double2* __restrict__ buf, int count, int M, int Ns, int tstep,
                                      const double2* __restrict__ tw) {
    const int m = M / R, total = count * m;
    const float rm = rcp_up(m), rns = rcp_up(Ns);
    constexpr int I = (kFftPointsPerThread * THREADS / R + THREADS - 1) / THREADS;
    double2 v[I][R];
    int o[I];
#pragma unroll
    for (int it = 0; it < I; ++it) {
        int e = threadIdx.x + it * THREADS;
        // opaque, so that its quotients are formed here and not kept live across every stage
        // of the transform (they are invariant per radix; held, they spill)
        asm volatile("" : "+v"(e));
        o[it] = -1;
        if (e >= total) continue;
        const int c = fdiv_up(e, rm), j = e - c * m;
        const int jq = fdiv_up(j, rns), jm = j - jq * Ns;
        const double2* in = buf + c * M;
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = in[j + r * m];
        if (jm > 0) {
            const int t1 = jm * tstep;   // the roots w^(r t1), r t1 < M
            int t = 0;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                t += t1;
                v[it][r] = cmul(v[it][r], root<INV>(tw, t));
            }
        }
        butterfly<R, INV>(v[it]);
        o[it] = c * M + jq * Ns * R + jm;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < I; ++it) {
        if (o[it] < 0) continue;
#pragma unroll
        for (int k = 0; k < R; ++k) buf[o[it] + k * Ns] = v[it][k];
    }
}

// any radix R: every output an R-term sum, X = sum_r in[j + r m] w^(r base)
template <int THREADS, bool INV>
__device__ __forceinline__ void stage_any(double2* __restrict__ buf, int count, int M, int Ns, int R, int tstep,
                                          const double2* __restrict__ tw) {
    const int m = M / R, total = count * M;
    const float rM = rcp_up(M), rm = rcp_up(m), rns = rcp_up(Ns);
    constexpr int I = kFftPointsPerThread;
    double2 acc[I];
    int o[I];
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int e = threadIdx.x + it * THREADS;
        o[it] = -1;
        if (e >= total) continue;
        const int c = fdiv_up(e, rM), q = e - c * M;
        const int k = fdiv_up(q, rm), j = q - k * m;
        const int jq = fdiv_up(j, rns), jm = j - jq * Ns;
        const double2* in = buf + c * M;
        const int base = jm * tstep + k * m;   // < M
        double2 a = in[j];
        int t = 0;
        for (int r = 1; r < R; ++r) {
            t += base;
            if (t >= M) t -= M;
            a = cadd(a, cmul(in[j + r * m], root<INV>(tw, t)));
        }
        acc[it] = a;
        o[it] = c * M + jq * Ns * R + jm + k * Ns;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < I; ++it)
        if (o[it] >= 0) buf[o[it]] = acc[it];
}

// Workgroups are dispatched to the 8 XCDs of an MI355X round-robin (workgroup b to XCD b mod 8).
// The group of lines a workgroup takes is chosen so that each XCD walks a contiguous range of
// groups: neighbouring groups share cache lines at their edges, which that XCD's L2 then fetches
// once.  A bijection of [0, n).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_group(int b, int n) {
    const int x = b % kXcds, k = b / kXcds, q = n / kXcds, r = n % kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Copies the root table (M entries) into LDS; the caller synchronises before fft_lds.
__device__ __forceinline__ void load_roots(const FftDev& p, double2* tw) {
    for (int t = threadIdx.x; t < p.M; t += blockDim.x) tw[t] = p.tw[t];
}

// `count` FFTs of length p.M (count p.M <= kFftPointsPerThread THREADS <= 8192) stored one
// after another in buf (LDS), in place, by a block of THREADS threads; tw: the root table in
// LDS; INV: the inverse (unnormalised) transform.  Every thread of the block must call it; the
// result is in buf when it returns.
template <int THREADS, bool INV>
__device__ __forceinline__ void fft_lds(double2* buf, int count, const FftDev& p, const double2* tw) {
    const int M = p.M;
    int Ns = 1, rest = M;   // rest = M / Ns: the product of the radices still to apply
    for (int s = 0; s < p.nf; ++s) {
        const int R = p.f[s];
        switch (R) {
            case 2: rest /= 2; stage<2, THREADS, INV>(buf, count, M, Ns, rest, tw); break;
            case 3: rest /= 3; stage<3, THREADS, INV>(buf, count, M, Ns, rest, tw); break;
            case 4: rest /= 4; stage<4, THREADS, INV>(buf, count, M, Ns, rest, tw); break;
            case 5: rest /= 5; stage<5, THREADS, INV>(buf, count, M, Ns, rest, tw); break;
            default: rest /= R; stage_any<THREADS, INV>(buf, count, M, Ns, R, rest, tw); break;
        }
        __syncthreads();
        Ns *= R;
    }
}

}  // namespace fftdev
}  // namespace bae
