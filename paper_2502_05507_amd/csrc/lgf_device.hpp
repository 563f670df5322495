// Device-side pieces of the LGF sum shared by the per-context kernels (lgf_sum.hip) and
// the batched engine (batch.hip): kernel evaluation (LDS table, far field, global table),
// wavefront reductions, compensated accumulators and the tile loop.
#pragma once

#include "internal.hpp"

namespace bae {
namespace lgfdev {

constexpr int kBlock = 256;
constexpr int kUnroll = 8;                           // sources per unrolled step (batched scalar loads)
constexpr int kFar2R = 64;                           // FP32: q = 2 far field beyond this gap
constexpr int kNearR = 32;                           // LDS table radius (both precisions)
constexpr int kNearE = (kNearR + 1) * (kNearR + 2) * (kNearR + 3) / 6;

constexpr double kPi = 3.14159265358979323846;
constexpr double C0 = 1.0 / (4.0 * kPi);
constexpr double C1 = 1.0 / (16.0 * kPi), C2 = -5.0 / (16.0 * kPi);
constexpr double D0 = 23.0 / (128.0 * kPi), D1 = -336.0 / (128.0 * kPi), D2 = 1155.0 / (128.0 * kPi),
                 D3 = -1134.0 / (128.0 * kPi);
constexpr double F0 = 647.0 / (512.0 * kPi), F1 = -20301.0 / (512.0 * kPi), F2 = 178035.0 / (512.0 * kPi),
                 F3 = -425425.0 / (512.0 * kPi), F4 = -208494.0 / (512.0 * kPi), F5 = 810810.0 / (512.0 * kPi);

template <typename Real>
__device__ __forceinline__ Real rsqrt_t(Real x);
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) { return rsqrt(x); }
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// q = 2 only (FP32 beyond kFar2R, where the q = 3 term is below 4.3e-8 relative).
__device__ __forceinline__ float far_field_q2(float X, float Y, float Z) {
    const float r2 = X + Y + Z;
    const float e2 = fmaf(X, Y + Z, Y * Z);
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rho = rinv * rinv;
    const float x = e2 * rho * rho;
    return rinv * fmaf(rho, fmaf(float(C2), x, float(C1)), float(C0));
}

// Far field from the squared offset components (all >= 0, not all 0).  FP64 keeps the
// q = 4 term (|error| <= 6.6e-11 relative beyond the LDS radius); FP32 stops at q = 3,
// whose error there (<= 4.8e-9) is already below FP32 rounding.
template <typename Real>
__device__ __forceinline__ Real far_field(Real X, Real Y, Real Z) {
    const Real r2 = X + Y + Z;
    const Real yz = Y * Z;
    const Real e2 = fma(X, Y + Z, yz);
    const Real e3 = X * yz;
    const Real rinv = rsqrt_t<Real>(r2);
    const Real rho = rinv * rinv;
    const Real rho2 = rho * rho;
    const Real x = e2 * rho2;
    const Real y = e3 * rho2 * rho;
    Real d = fma(Real(D3), y, fma(x, fma(x, Real(D2), Real(D1)), Real(D0)));
    if constexpr (sizeof(Real) == 8) {
        const Real f = fma(y, fma(Real(F5), x, Real(F4)), fma(x, fma(x, fma(x, Real(F3), Real(F2)), Real(F1)), Real(F0)));
        d = fma(rho, f, d);
    }
    const Real c = fma(Real(C2), x, Real(C1));
    const Real B = fma(rho, fma(rho, d, c), Real(C0));
    return rinv * B;
}

__device__ __forceinline__ uint32_t sorted_index(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t lo = min(a, min(b, c));
    const uint32_t hi = max(a, max(b, c));
    const uint32_t mid = a + b + c - lo - hi;
    return hi * (hi + 1) * (hi + 2) / 6 + ((mid * (mid + 1)) >> 1) + lo;
}

__device__ __forceinline__ uint64_t sorted_index64(uint64_t a, uint64_t b, uint64_t c) {
    const uint64_t lo = min(a, min(b, c));
    const uint64_t hi = max(a, max(b, c));
    const uint64_t mid = a + b + c - lo - hi;
    return hi * (hi + 1) * (hi + 2) / 6 + ((mid * (mid + 1)) >> 1) + lo;
}

// Offsets reaching here satisfy max|d_i| <= the resident table radius whenever the far
// field is off (the sum only pairs points of one bounding box; lgf_eval checks it).
template <typename Real>
__device__ __forceinline__ Real eval_pair(int dx, int dy, int dz, const Real* __restrict__ lds_tab,
                                          const Real* __restrict__ full_tab, bool far_field_ok) {
    const uint32_t a = (uint32_t)abs(dx), b = (uint32_t)abs(dy), c = (uint32_t)abs(dz);
    const uint32_t m = max(a, max(b, c));
    if (m <= (uint32_t)kNearR) return lds_tab[sorted_index(a, b, c)];
    if (far_field_ok) return far_field<Real>(Real(a * a), Real(b * b), Real(c * c));
    return full_tab[sorted_index64(a, b, c)];
}

__device__ __forceinline__ int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

template <typename Real>
struct Acc;
template <>
struct Acc<double> {
    double s = 0.0;
    __device__ __forceinline__ void add(double v) { s += v; }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ double value() const { return s; }
};
template <>
struct Acc<float> {
    float run = 0.f, sum = 0.f, comp = 0.f;
    __device__ __forceinline__ void add(float v) { run += v; }
    __device__ __forceinline__ void flush() {
        const float t = sum + run;
        comp += fabsf(sum) >= fabsf(run) ? (sum - t) + run : (run - t) + sum;
        sum = t;
        run = 0.f;
    }
    __device__ __forceinline__ double value() const { return (double)sum + (double)comp + (double)run; }
};

template <typename Real>
struct SumArgs {
    const int32_t *tx, *ty, *tz;
    int nt;
    const int32_t *sx, *sy, *sz;
    const Real *sxr, *syr, *szr;      // source coordinates in the kernel's precision
    const int32_t* sbox;              // [nblk][6] source block bounding boxes
    int ns, nblk, blk_per_chunk;
    const Real* w;
    int64_t ldw;
    const Real* near_tab;
    const Real* full_tab;
    int far_ok;
    double* part;
    int64_t ldp;
};

// One thread per target.  Each wavefront walks the source blocks of its chunk and, from
// the bounding boxes of its 64 targets and of the block, picks one of four loops
// (a wavefront-uniform branch):
//   far     every pair beyond the LDS radius, sigma = 0: far field in registers
//   gather  every pair beyond the LDS radius, sigma > 0: the global table
//   near    every pair within the LDS radius: LDS table
//   mixed   per-pair choice
template <typename Real, int NR>
__device__ __forceinline__ void sum_tile(const SumArgs<Real>& a, const Real* __restrict__ tab, int tile, int chunk) {
    const int t = tile * kBlock + threadIdx.x;
    const int tc = min(t, a.nt - 1);
    const int ix = a.tx[tc], iy = a.ty[tc], iz = a.tz[tc];
    const Real fx = (Real)ix, fy = (Real)iy, fz = (Real)iz;
    const int lx = wave_min(ix), ly = wave_min(iy), lz = wave_min(iz);
    const int hx = wave_max(ix), hy = wave_max(iy), hz = wave_max(iz);

    const int b0 = chunk * a.blk_per_chunk;
    const int b1 = min(a.nblk, b0 + a.blk_per_chunk);
    Acc<Real> acc[NR];
    for (int b = b0; b < b1; ++b) {
        const int32_t* bb = a.sbox + 6 * b;
        const int gap = max(max(max(bb[0] - hx, lx - bb[3]), max(bb[1] - hy, ly - bb[4])),
                            max(max(bb[2] - hz, lz - bb[5]), 0));
        const int span = max(max(max(bb[3] - lx, hx - bb[0]), max(bb[4] - ly, hy - bb[1])),
                             max(bb[5] - lz, hz - bb[2]));
        const int sb = b * kSourceBlock;        // blocks are full: the source arrays are padded
        if (sizeof(Real) == 4 && gap > kFar2R && a.far_ok) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += kUnroll) {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int s = s0 + u;
                    const float dx = (float)fx - (float)a.sxr[s], dy = (float)fy - (float)a.syr[s],
                                dz = (float)fz - (float)a.szr[s];
                    const Real G = (Real)far_field_q2(dx * dx, dy * dy, dz * dz);
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * a.w[r * a.ldw + s]);
                }
            }
        } else if (gap > kNearR && a.far_ok) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += kUnroll) {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int s = s0 + u;
                    const Real dx = fx - a.sxr[s], dy = fy - a.syr[s], dz = fz - a.szr[s];
                    const Real G = far_field<Real>(dx * dx, dy * dy, dz * dz);
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * a.w[r * a.ldw + s]);
                }
            }
        } else if (gap > kNearR) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += kUnroll) {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int s = s0 + u;
                    const uint32_t da = (uint32_t)abs(ix - a.sx[s]), db = (uint32_t)abs(iy - a.sy[s]),
                                   dc = (uint32_t)abs(iz - a.sz[s]);
                    const Real G = a.full_tab[sorted_index64(da, db, dc)];
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * a.w[r * a.ldw + s]);
                }
            }
        } else if (span <= kNearR) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += kUnroll) {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int s = s0 + u;
                    const uint32_t da = (uint32_t)abs(ix - a.sx[s]), db = (uint32_t)abs(iy - a.sy[s]),
                                   dc = (uint32_t)abs(iz - a.sz[s]);
                    const Real G = tab[sorted_index(da, db, dc)];
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * a.w[r * a.ldw + s]);
                }
            }
        } else {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += kUnroll) {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int s = s0 + u;
                    const Real G = eval_pair<Real>(ix - a.sx[s], iy - a.sy[s], iz - a.sz[s], tab, a.full_tab,
                                                   a.far_ok != 0);
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * a.w[r * a.ldw + s]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r].flush();
    }
    if (t < a.nt) {
#pragma unroll
        for (int r = 0; r < NR; ++r) a.part[(int64_t)r * a.ldp + (int64_t)chunk * a.nt + t] = acc[r].value();
    }
}

}  // namespace lgfdev
}  // namespace bae
