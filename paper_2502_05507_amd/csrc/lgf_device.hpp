// Device-side pieces of the LGF sum shared by the per-context kernels (lgf_sum.hip) and
// the batched engine (batch.hip): kernel evaluation (LDS table, far field, global table),
// wavefront reductions, compensated accumulators and the tile loop.
//
// Coordinates on the device are 4 x the lattice index (kQuant), as int32, float and double.
// Then |t - s| of two points is directly the byte offset of |d| into a uint32 array, which
// is how the 1/48-symmetric table index is formed without a multiply:
//   index(d) = tet(hi) + tri(mid) + lo,  (lo <= mid <= hi) = sorted |d_i|,
//   tet(h) = h(h+1)(h+2)/6, tri(m) = m(m+1)/2   (the triples with max <= h-1, then mid)
// with tet and tri read from two small LDS arrays that hold sizeof(Real) x their values:
// per pair three absolute differences (v_sad_u32), min3 / med3 / max3, two LDS reads and
// one add give the byte address of G in the LDS (or global) table.
#pragma once

#include "internal.hpp"

namespace bae {
namespace lgfdev {

constexpr int kWave = 64;
template <typename Real>
constexpr int unroll() { return 4; }   // sources per unrolled step
// Sources per step of the one-RHS table loop: 32-byte scalar loads, twice as many LDS reads in
// flight.  Every other loop takes 4, so that its double-buffered sources leave the block loop
// enough scalar registers (with 8 everywhere the FP32 sum spilled 69 of them to VGPR lanes and
// restored them in every block; far-dominated sums ran 7% slower).
template <typename Real, int NR>
constexpr int table_unroll() { return NR == 1 ? 32 / (int)sizeof(Real) : 4; }
constexpr int kMaxR = kMaxTableRadius;               // largest table radius (tet / tri arrays)

// LDS layouts.  FAR (sigma = 0, far field beyond the table): the index arrays only need the
// table radius, leaving room for a larger table.  Otherwise (sigma > 0) they span every
// offset of the global table.
template <typename Real, bool FAR>
constexpr int tab_radius() {
    return sizeof(Real) == 4 ? (FAR ? kLdsRadiusFar32 : kLdsRadius32) : (FAR ? kLdsRadiusFar64 : kLdsRadius64);
}
template <typename Real, bool FAR>
constexpr int tab_entries() {
    return (tab_radius<Real, FAR>() + 1) * (tab_radius<Real, FAR>() + 2) * (tab_radius<Real, FAR>() + 3) / 6;
}

constexpr double kPi = 3.14159265358979323846;
// Far-field coefficients for the quantised offset D = kQuant d (so |D| = 4|n|): with
// rinv = 1/|D| and rho = 1/|D|^2 the expansion keeps its form, each power of rho and the
// leading 1/|n| picking up a power of kQuant (exact: powers of two).
constexpr double Q1 = kQuant, Q3 = Q1 * Q1 * Q1, Q5 = Q3 * Q1 * Q1, Q7 = Q5 * Q1 * Q1;
constexpr double C0 = Q1 / (4.0 * kPi);
constexpr double C1 = Q3 / (16.0 * kPi), C2 = -5.0 * Q3 / (16.0 * kPi);
constexpr double D0 = 23.0 * Q5 / (128.0 * kPi), D1 = -336.0 * Q5 / (128.0 * kPi), D2 = 1155.0 * Q5 / (128.0 * kPi),
                 D3 = -1134.0 * Q5 / (128.0 * kPi);
constexpr double F0 = 647.0 * Q7 / (512.0 * kPi), F1 = -20301.0 * Q7 / (512.0 * kPi),
                 F2 = 178035.0 * Q7 / (512.0 * kPi), F3 = -425425.0 * Q7 / (512.0 * kPi),
                 F4 = -208494.0 * Q7 / (512.0 * kPi), F5 = 810810.0 * Q7 / (512.0 * kPi);

// FP32: q = 2.  Beyond the far-field gap (|n| >= 33) the dropped q = 3 term is at most
// 0.72 |n|^-4 = 6.1e-7 of G (on the axes), below the rounding error the FP32 sum carries
// anyway: the FP32 double-layer operator differs from the FP64 one by 3.3e-7 (relative L2,
// 129^3 ellipsoid) with q = 2 or q = 3 alike.  X, Y, Z: squared quantised offset components.
__device__ __forceinline__ float far_field_q2(float X, float Y, float Z) {
    const float r2 = X + Y + Z;
    const float e2 = fmaf(X, Y + Z, Y * Z);
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rho = rinv * rinv;
    const float x = e2 * rho * rho;
    return rinv * fmaf(rho, fmaf(float(C2), x, float(C1)), float(C0));
}

// FP32, sigma = 0, q = 2 again, from the lattice offset n (not quantised) through
//   r2 = |n|^2,  Z = n_z^2,  m = n_y^2 - n_x^2,
// which the sum loop gets from packed binary16 differences with two dot products.  With
// zeta = Z / r2 and mu = m / r2 the second symmetric polynomial of the squared components is
// e2 = r2^2 (1 + 2 zeta - 3 zeta^2 - mu^2) / 4, which turns the q = 2 expansion into
//   G = kFarScale32 rinv [16/5 + rho (mu^2 + 3 zeta^2 - 2 zeta - 1/5)],  rinv = 1/|n|, rho = rinv^2.
// Returned without the factor kFarScale32, which the caller applies once per source block.
constexpr float kFarScale32 = float(5.0 / (64.0 * kPi));
__device__ __forceinline__ float far_field_q2_lattice(float r2, float Z, float m) {
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rho = rinv * rinv;
    const float zeta = Z * rho, mu = m * rho;
    const float c = fmaf(mu, mu, fmaf(zeta, fmaf(zeta, 3.0f, -2.0f), -0.2f));
    return rinv * fmaf(rho, c, 3.2f);
}

// Four far-field pairs of one target: the binary16 differences d_k = t - s_k (s_k
// wavefront-uniform, in scalar registers) and from them
//   r2_k = d_k.x^2 + d_k.y^2 + Z_k,   m_k = d_k.y^2 - d_k.x^2
// (inputs: integers of magnitude <= 2048, exact in binary16; every product and sum is an
// integer below 2^24, exact in FP32).  A VALU instruction may read the result of a DOT
// instruction only three wait states after it, which the compiler cannot see inside an asm
// statement: hence one statement per four pairs, ending in those wait states.
__device__ __forceinline__ void far_pairs4(uint32_t t, uint32_t s0, uint32_t s1, uint32_t s2, uint32_t s3,
                                           const float (&Z)[4], float (&r2)[4], float (&m)[4]) {
    uint32_t d0, d1, d2, d3;
    asm("v_pk_add_f16 %0, %12, %13 neg_lo:[0,1] neg_hi:[0,1]\n\t"
        "v_pk_add_f16 %1, %12, %14 neg_lo:[0,1] neg_hi:[0,1]\n\t"
        "v_pk_add_f16 %2, %12, %15 neg_lo:[0,1] neg_hi:[0,1]\n\t"
        "v_pk_add_f16 %3, %12, %16 neg_lo:[0,1] neg_hi:[0,1]\n\t"
        "v_dot2_f32_f16 %4, %0, %0, %17\n\t"
        "v_dot2_f32_f16 %5, %0, %0, 0 neg_lo:[0,1,0]\n\t"
        "v_dot2_f32_f16 %6, %1, %1, %18\n\t"
        "v_dot2_f32_f16 %7, %1, %1, 0 neg_lo:[0,1,0]\n\t"
        "v_dot2_f32_f16 %8, %2, %2, %19\n\t"
        "v_dot2_f32_f16 %9, %2, %2, 0 neg_lo:[0,1,0]\n\t"
        "v_dot2_f32_f16 %10, %3, %3, %20\n\t"
        "v_dot2_f32_f16 %11, %3, %3, 0 neg_lo:[0,1,0]\n\t"
        "s_nop 2"
        : "=&v"(d0), "=&v"(d1), "=&v"(d2), "=&v"(d3), "=&v"(r2[0]), "=&v"(m[0]), "=&v"(r2[1]), "=&v"(m[1]),
          "=&v"(r2[2]), "=&v"(m[2]), "=&v"(r2[3]), "=&v"(m[3])
        : "v"(t), "s"(s0), "s"(s1), "s"(s2), "s"(s3), "v"(Z[0]), "v"(Z[1]), "v"(Z[2]), "v"(Z[3]));
}

// 1/sqrt(x) of a positive finite FP64 square sum: the hardware estimate and one Newton
// step, whose relative error is about 1.5 e0^2 for an estimate error e0 (no special
// cases to handle, unlike the library rsqrt).
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// The same for four targets t_k of one lane against one source s (both per lane).
__device__ __forceinline__ void far_pairs4v(const uint32_t (&t)[4], uint32_t s, const float (&Z)[4], float (&r2)[4],
                                            float (&m)[4]) {
    uint32_t d0, d1, d2, d3;
    asm("v_pk_add_f16 %0, %12, %16 neg_lo:[0,1] neg_hi:[0,1]\n\t"
        "v_pk_add_f16 %1, %13, %16 neg_lo:[0,1] neg_hi:[0,1]\n\t"
        "v_pk_add_f16 %2, %14, %16 neg_lo:[0,1] neg_hi:[0,1]\n\t"
        "v_pk_add_f16 %3, %15, %16 neg_lo:[0,1] neg_hi:[0,1]\n\t"
        "v_dot2_f32_f16 %4, %0, %0, %17\n\t"
        "v_dot2_f32_f16 %5, %0, %0, 0 neg_lo:[0,1,0]\n\t"
        "v_dot2_f32_f16 %6, %1, %1, %18\n\t"
        "v_dot2_f32_f16 %7, %1, %1, 0 neg_lo:[0,1,0]\n\t"
        "v_dot2_f32_f16 %8, %2, %2, %19\n\t"
        "v_dot2_f32_f16 %9, %2, %2, 0 neg_lo:[0,1,0]\n\t"
        "v_dot2_f32_f16 %10, %3, %3, %20\n\t"
        "v_dot2_f32_f16 %11, %3, %3, 0 neg_lo:[0,1,0]\n\t"
        "s_nop 2"
        : "=&v"(d0), "=&v"(d1), "=&v"(d2), "=&v"(d3), "=&v"(r2[0]), "=&v"(m[0]), "=&v"(r2[1]), "=&v"(m[1]),
          "=&v"(r2[2]), "=&v"(m[2]), "=&v"(r2[3]), "=&v"(m[3])
        : "v"(t[0]), "v"(t[1]), "v"(t[2]), "v"(t[3]), "v"(s), "v"(Z[0]), "v"(Z[1]), "v"(Z[2]), "v"(Z[3]));
}

// FP64: q = 4 from the squared quantised offset components (all >= 0, not all 0); relative
// error <= 6.6e-11 beyond the far-field gap.
__device__ __forceinline__ double far_field_q4(double X, double Y, double Z) {
    const double r2 = X + Y + Z;
    const double yz = Y * Z;
    const double e2 = fma(X, Y + Z, yz);
    const double e3 = X * yz;
    const double rinv = rsqrt_pos(r2);
    const double rho = rinv * rinv;
    const double rho2 = rho * rho;
    const double x = e2 * rho2;
    const double y = e3 * rho2 * rho;
    double d = fma(D3, y, fma(x, fma(x, D2, D1), D0));
    const double f = fma(y, fma(F5, x, F4), fma(x, fma(x, fma(x, F3, F2), F1), F0));
    d = fma(rho, f, d);
    const double c = fma(C2, x, C1);
    const double B = fma(rho, fma(rho, d, c), C0);
    return rinv * B;
}

// sigma > 0 (s = kappa^2 in lattice units): the same Fourier-symbol expansion with
// 1/(s + |theta|^2)^k in place of 1/|theta|^(2k) gives, with u = kappa |n|,
//   G_s(n) = e^(-u) / (4 pi |n|) [1 + T2 + O(|n|^-4)],
//   T2 = [(1 + u)(1 - 5x)/4 - u^2 x/2 + u^3 (1 - 2x)/24] / |n|^2,
// which at u = 0 is the q = 2 term above.  It is evaluated as e^(-u + T2) / (4 pi |n|): the
// factor 1 + T2 becomes e^T2, which differs from it by T2^2/2 = O(|n|^-4), the order of the
// first dropped term, and puts the correction into the exponent (one instruction fewer per
// value).  The expansion is asymptotic in 1/|n| at fixed u only while kappa is small, so a
// context uses it only after checking this form against its own exact table at every offset
// beyond the LDS radius.  kq = kappa / kQuant and yk = -kappa log2(e) / kQuant (quantised
// offsets: |D| = kQuant |n|).
template <typename Real>
__device__ __forceinline__ Real far_field_yukawa(Real X, Real Y, Real Z, Real kq, Real yk) {
    constexpr double kLog2C = -1.6514961294723187;   // log2(kQuant / (4 pi)) = log2(1 / pi)
    constexpr double kL = 1.4426950408889634;         // log2(e)
    const Real r2 = X + Y + Z;
    const Real e2 = fma(X, Y + Z, Y * Z);
    Real rinv;
    if constexpr (sizeof(Real) == 4) {
        rinv = __builtin_amdgcn_rsqf(r2);
    } else {
        rinv = rsqrt(r2);
    }
    const Real rho = rinv * rinv;
    const Real x = e2 * rho * rho;
    const Real rq = r2 * rinv;
    const Real u = rq * kq;
    // kQuant^2 = 16 folded into the bracket (rho is 1/|D|^2 = 1/(16 |n|^2)), and log2(e)
    const Real A = fma(Real(-20 * kL), x, Real(4 * kL));
    const Real c2 = Real(-8 * kL) * x;
    const Real c3 = fma(Real(-4.0 / 3.0 * kL), x, Real(2.0 / 3.0 * kL));
    const Real br = fma(u, fma(u, fma(u, c3, c2), A), A);
    const Real arg = fma(rho, br, fma(rq, yk, Real(kLog2C)));
    if constexpr (sizeof(Real) == 4) return __builtin_amdgcn_exp2f(arg) * rinv;
    else return exp2(arg) * rinv;
}

// The same sigma > 0 form from the lattice offset (FP32), through r2, Z and m as in
// far_field_q2_lattice: with x4 = 4 e2/|n|^4 = 1 + 2 zeta - 3 zeta^2 - mu^2,
//   T2 |n|^2 = A (1 + u) + B u^2 + C u^3,  A = 1/4 - 5 x4/16, B = -x4/8, C = 1/24 - x4/48.
// Since u^2 / |n|^2 = kappa^2 and u^3 / |n|^2 = kappa^3 |n|, the exponent of
// G = 2^arg / |n| is, with L = log2(e),
//   arg = log2(1/(4 pi)) - L u + L T2 = P + |n| Q + rho L A (1 + u),
//   P = log2(1/(4 pi)) + L kappa^2 B,   Q = -L kappa + L kappa^3 C,
// P and Q linear in x4 with per-launch coefficients (YukawaLattice): two fused
// multiply-adds fewer per value than the cubic in u.  rho r2 = 1 up to the rounding of the
// rsqrt estimate, which touches the two folded terms (at most 1e-3 of the exponent's
// correction) at 1e-7.
struct YukawaLattice {
    float kl = 0.f;           // kappa (lattice units)
    float p0 = 0.f, p1 = 0.f; // P = p0 + p1 x4
    float q0 = 0.f, q1 = 0.f; // Q = q0 + q1 x4
};
inline YukawaLattice yukawa_lattice(double kappa) {
    constexpr double L = 1.4426950408889634;
    const double k2 = kappa * kappa, k3 = k2 * kappa;
    YukawaLattice y;
    y.kl = (float)kappa;
    y.p0 = (float)-3.6514961294723187;   // log2(1 / (4 pi))
    y.p1 = (float)(-L * k2 / 8.0);
    y.q0 = (float)(-L * kappa + L * k3 / 24.0);
    y.q1 = (float)(-L * k3 / 48.0);
    return y;
}
__device__ __forceinline__ float far_field_yukawa_lattice(float r2, float Z, float m, const YukawaLattice& y) {
    constexpr double kL = 1.4426950408889634;   // log2(e)
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rho = rinv * rinv;
    const float zeta = Z * rho, mu = m * rho;
    const float x4 = fmaf(-mu, mu, fmaf(zeta, fmaf(zeta, -3.0f, 2.0f), 1.0f));
    const float rq = r2 * rinv;
    const float P = fmaf(x4, y.p1, y.p0);
    const float Q = fmaf(x4, y.q1, y.q0);
    const float AL = fmaf(x4, float(-0.3125 * kL), float(0.25 * kL));
    // rho (1 + u) = rho + kappa rinv (rho |n| = rinv)
    const float s1 = fmaf(rinv, y.kl, rho);
    const float arg = fmaf(AL, s1, fmaf(rq, Q, P));
    return __builtin_amdgcn_exp2f(arg) * rinv;
}

template <typename Real>
__device__ __forceinline__ Real far_field(Real X, Real Y, Real Z) {
    if constexpr (sizeof(Real) == 4) return far_field_q2(X, Y, Z);
    else return far_field_q4(X, Y, Z);
}

// |a - b| of two non-negative coordinates in one instruction.  The second operand is a
// wavefront-uniform value held in a scalar register (a source point of the unrolled loop).
__device__ __forceinline__ uint32_t absdiff_s(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_sad_u32 %0, %1, %2, 0" : "=v"(r) : "v"(a), "s"(b));
    return r;
}
// ... with both operands per lane.
__device__ __forceinline__ uint32_t absdiff_v(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_sad_u32 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Wavefront-uniform read-only loads through the constant address space: they stay scalar
// loads (s_load) although the kernel also writes memory (partial sums, the work counter).
template <typename T>
__device__ __forceinline__ T ldu(const T* p, int64_t i) {
    return ((const __attribute__((address_space(4))) T*)p)[i];
}

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) { return min(a, min(b, c)); }
__device__ __forceinline__ uint32_t max3u(uint32_t a, uint32_t b, uint32_t c) { return max(a, max(b, c)); }
// The median in one instruction (written out: the compiler would share max(a, b) between
// the median and the maximum and lose both three-operand forms).
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Index tables in LDS: tet[h] = sizeof(Real) tet(h), tri[m] = sizeof(Real) tri(m) (bytes).
template <typename Real>
struct Lds {
    Real* tab;            // table prefix, radius tab_r
    uint32_t* tet;
    uint32_t* tri;
};

// One LDS allocation, index arrays first: every LDS address the lookups form is then a
// register plus a constant below 64 KB, which ds_read takes as its immediate offset.
template <typename Real, bool FAR>
constexpr int idx_len() {   // index array length: > the largest radius indexed, 16-byte multiple
    return ((FAR ? tab_radius<Real, FAR>() : kMaxR) + 4) / 4 * 4;
}
template <typename Real, bool FAR>
constexpr int lds_bytes() { return 2 * idx_len<Real, FAR>() * 4 + tab_entries<Real, FAR>() * (int)sizeof(Real); }
template <typename Real, bool FAR>
__device__ __forceinline__ Lds<Real> lds_layout(char* base) {
    constexpr int n = idx_len<Real, FAR>();
    static_assert(lds_bytes<Real, FAR>() <= 160 * 1024, "LDS of one gfx950 compute unit");
    return Lds<Real>{(Real*)(base + 2 * n * 4), (uint32_t*)base, (uint32_t*)(base + n * 4)};
}

// Byte offset of G(d) in a sorted table from the quantised |d| components.
template <typename Real>
__device__ __forceinline__ uint32_t table_offset(const Lds<Real>& L, uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t lo = min3u(a, b, c), mid = med3u(a, b, c), hi = max3u(a, b, c);
    const uint32_t th = *(const uint32_t*)((const char*)L.tet + hi);
    const uint32_t tm = *(const uint32_t*)((const char*)L.tri + mid);
    if constexpr (sizeof(Real) == 4) return th + tm + lo;
    else return th + tm + 2u * lo;
}

template <typename Real>
__device__ __forceinline__ Real lds_value(const Lds<Real>& L, uint32_t off) {
    return *(const Real*)((const char*)L.tab + off);
}
template <typename Real>
__device__ __forceinline__ Real global_value(const Real* __restrict__ full, uint32_t off) {
    return *(const Real*)((const char*)full + off);
}

template <typename Real>
__device__ __forceinline__ void fill_index(const Lds<Real>& L, int idx_r) {
    for (int h = threadIdx.x; h <= idx_r; h += blockDim.x) {
        const uint32_t u = (uint32_t)h;
        L.tet[h] = (uint32_t)sizeof(Real) * (u * (u + 1) * (u + 2) / 6);
        L.tri[h] = (uint32_t)sizeof(Real) * (u * (u + 1) / 2);
    }
}

// Copy the first n table entries into LDS with 16-byte loads, eight per thread in flight
// (one load at a time would pay the memory latency once per 4 KB of table).  Both tables
// start 16-byte aligned: the device table at an allocation's start, the LDS copy after
// index arrays of a 16-byte multiple.
template <typename Real>
__device__ __forceinline__ void stage_table(Real* dst, const Real* __restrict__ src, int n) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    constexpr int K = 8;
    const int nv = (int)(((int64_t)n * (int64_t)sizeof(Real)) / 16);
    const u32x4* __restrict__ s = (const u32x4*)src;
    u32x4* d = (u32x4*)dst;
    for (int base = threadIdx.x; base < nv; base += K * (int)blockDim.x) {
        u32x4 r[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = base + k * (int)blockDim.x;
            if (i < nv) r[k] = s[i];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = base + k * (int)blockDim.x;
            if (i < nv) d[i] = r[k];
        }
    }
    for (int i = nv * (16 / (int)sizeof(Real)) + (int)threadIdx.x; i < n; i += (int)blockDim.x) dst[i] = src[i];
}

// Fill the LDS table prefix (radius tab_r) and the index arrays up to radius idx_r.
template <typename Real>
__device__ __forceinline__ void fill_lds(const Lds<Real>& L, const Real* __restrict__ src, int tab_r, int idx_r) {
    stage_table(L.tab, src, (tab_r + 1) * (tab_r + 2) * (tab_r + 3) / 6);
    fill_index<Real>(L, idx_r);
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
    __device__ __forceinline__ void scale_run(double) {}
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ double value() const { return s; }
};
template <>
struct Acc<float> {
    float run = 0.f, sum = 0.f, comp = 0.f;
    __device__ __forceinline__ void add(float v) { run += v; }
    __device__ __forceinline__ void scale_run(float f) { run *= f; }   // the block's terms times f
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
    const uint32_t *tx, *ty, *tz;     // quantised target coordinates
    int nt;
    const uint32_t *sx, *sy, *sz;     // quantised source coordinates
    const Real *sxr, *syr, *szr;      // the same in the kernel's precision
    const uint32_t *txy, *sxy;        // lattice (x, y) of targets / sources as packed binary16
    const float *tzl, *szl;           // lattice z (FP32 far field, sigma = 0)
    const int32_t* sbox;              // [nblk][6] quantised source block bounding boxes
    int ns, nblk, blk_per_chunk;
    const Real* w;
    int64_t ldw;
    const Real* near_tab;             // table prefix staged in LDS (radius tab_r)
    const Real* full_tab;             // full table (sigma > 0): radius full_r
    int tab_r;                        // LDS table radius used (<= the kernel's tab_radius)
    int full_r;
    int far_ok;                       // a far field is valid beyond far_gap (and beyond tab_r)
    int far_gap;                      // smallest far-block gap (lattice units)
    int yukawa;                       // the far field is the sigma > 0 form (kq, yk)
    Real kq, yk;
    YukawaLattice yl;                 // the same in lattice units (FP32 far-field blocks)
    double* part;
    int64_t ldp;
};

// One wavefront owns 64 consecutive (Morton-ordered) targets and walks the source blocks of
// one chunk.  From the bounding boxes of its targets and of each block it picks one loop
// with a wavefront-uniform branch (block_class):
//   table   every pair within the LDS table radius
//   far     every pair beyond the far-field gap: expansion in registers (sigma = 0: q = 2
//           in FP32 from binary16 lattice differences, q = 4 in FP64; sigma > 0: the
//           Yukawa form in FP32 where the context accepted it)
//   gather  every pair beyond the LDS radius, sigma > 0: the global table
//   mixed   per-pair choice between the LDS table and the far field / global table
// The sources of one unrolled step, as whole scalar-register vectors.  They are loaded
// before any of the step's arithmetic (the scheduling barrier): scalar loads and LDS reads
// share one completion counter and scalar loads complete out of order, so a scalar load
// left among the table reads would make every wait drain all LDS reads in flight.
template <typename T, int N>
using vec_t = T __attribute__((ext_vector_type(N)));
template <typename T, int N>
__device__ __forceinline__ vec_t<T, N> ldu_vec(const T* p, int64_t i) {
    return *((const __attribute__((address_space(4))) vec_t<T, N>*)(p + i));
}

template <typename Real, int NR, int U = unroll<Real>()>
struct Step {
    vec_t<uint32_t, U> x, y, z;     // quantised integer coordinates (table / gather / mixed)
    vec_t<Real, U> xr, yr, zr;      // the same in the kernel's precision (far field / mixed)
    vec_t<uint32_t, U> xy;          // lattice (x, y) as binary16 pairs and z (FP32 far field)
    vec_t<float, U> zl;
    vec_t<Real, U> w[NR];
};

template <typename Real, int NR, bool INT, bool REAL, bool HALF = false, int U = unroll<Real>()>
__device__ __forceinline__ Step<Real, NR, U> load_step(const SumArgs<Real>& a, int s0) {
    Step<Real, NR, U> st;
    if constexpr (HALF) {
        st.xy = ldu_vec<uint32_t, U>(a.sxy, s0);
        st.zl = ldu_vec<float, U>(a.szl, s0);
    }
    if constexpr (INT) {
        st.x = ldu_vec<uint32_t, U>(a.sx, s0);
        st.y = ldu_vec<uint32_t, U>(a.sy, s0);
        st.z = ldu_vec<uint32_t, U>(a.sz, s0);
    }
    if constexpr (REAL) {
        st.xr = ldu_vec<Real, U>(a.sxr, s0);
        st.yr = ldu_vec<Real, U>(a.syr, s0);
        st.zr = ldu_vec<Real, U>(a.szr, s0);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) st.w[r] = ldu_vec<Real, U>(a.w, r * a.ldw + s0);
    __builtin_amdgcn_sched_barrier(0);
    return st;
}

// Table values of one unrolled step, in phases: all index triples, then all index-array
// reads, then all value reads (LDS or, for GLOBAL, the full table), so each phase's reads
// are in flight together instead of one dependent chain per pair.
template <typename Real, int U, bool GLOBAL>
__device__ __forceinline__ void lookup_step(const Lds<Real>& L, const Real* __restrict__ full, uint32_t ix,
                                            uint32_t iy, uint32_t iz, const vec_t<uint32_t, U>& sx,
                                            const vec_t<uint32_t, U>& sy, const vec_t<uint32_t, U>& sz, Real* G) {
    uint32_t lo[U], mid[U], hi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t a = absdiff_s(ix, sx[u]), b = absdiff_s(iy, sy[u]), c = absdiff_s(iz, sz[u]);
        lo[u] = min3u(a, b, c);
        mid[u] = med3u(a, b, c);
        hi[u] = max3u(a, b, c);
    }
    __builtin_amdgcn_sched_barrier(0);
    uint32_t th[U], tm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        th[u] = *(const uint32_t*)((const char*)L.tet + hi[u]);
        tm[u] = *(const uint32_t*)((const char*)L.tri + mid[u]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t off = sizeof(Real) == 4 ? th[u] + tm[u] + lo[u] : th[u] + tm[u] + 2u * lo[u];
        G[u] = GLOBAL ? global_value(full, off) : lds_value(L, off);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// One FP32 far block (every pair beyond the far-field gap) from the binary16 lattice
// differences: q = 2 (sigma = 0, its constant factor applied once at the end) or the
// Yukawa form (sigma > 0).  Each step's sources are loaded one step ahead.
template <typename Real, int NR, bool YUK>
__device__ __forceinline__ void far2_block(const SumArgs<Real>& a, uint32_t txy, float tzl, int sb, Acc<Real> (&acc)[NR]) {
    constexpr int U = unroll<Real>();
    Step<Real, NR> nx = load_step<Real, NR, false, false, true>(a, sb);
    // every counter drained here, so that the loop's only wait is for its own loads
    __builtin_amdgcn_s_waitcnt(0);
    for (int s0 = sb; s0 < sb + kSourceBlock; s0 += U) {
        const Step<Real, NR> st = nx;
        nx = load_step<Real, NR, false, false, true>(a, min(s0 + U, sb + kSourceBlock - U));
#pragma unroll
        for (int u0 = 0; u0 < U; u0 += 4) {
            float Z[4], r2[4], m[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float dz = tzl - st.zl[u0 + k];
                Z[k] = dz * dz;
            }
            far_pairs4(txy, st.xy[u0], st.xy[u0 + 1], st.xy[u0 + 2], st.xy[u0 + 3], Z, r2, m);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const Real G = YUK ? far_field_yukawa_lattice(r2[k], Z[k], m[k], a.yl)
                                   : far_field_q2_lattice(r2[k], Z[k], m[k]);
#pragma unroll
                for (int r = 0; r < NR; ++r) acc[r].add(G * st.w[r][u0 + k]);
            }
        }
    }
    if (!YUK) {
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r].scale_run(Real(kFarScale32));
    }
}

// ROT: start at a block of the chunk that depends on the tile (see below); without it every
// tile walks the chunk from its first block.
template <typename Real, int NR, bool ROT = true>
__device__ __forceinline__ void sum_tile(const SumArgs<Real>& a, const Lds<Real>& L, int tile, int chunk) {
    constexpr int U = unroll<Real>();
    const int lane = threadIdx.x & (kWave - 1);
    const int t = tile * kWave + lane;
    const int tc = min(t, a.nt - 1);
    const uint32_t ix = a.tx[tc], iy = a.ty[tc], iz = a.tz[tc];
    const Real fx = (Real)ix, fy = (Real)iy, fz = (Real)iz;
    uint32_t txy = 0;
    float tzl = 0.f;
    if constexpr (sizeof(Real) == 4) {
        txy = a.txy[tc];
        tzl = a.tzl[tc];
    }
    const int lx = wave_min((int)ix), ly = wave_min((int)iy), lz = wave_min((int)iz);
    const int hx = wave_max((int)ix), hy = wave_max((int)iy), hz = wave_max((int)iz);
    const uint32_t tab_q = (uint32_t)(kQuant * a.tab_r);

    const int b0 = chunk * a.blk_per_chunk;
    const int b1 = min(a.nblk, b0 + a.blk_per_chunk);
    // the tiles of a work item share its chunk; each starts at another block of it, so the
    // wavefronts of a workgroup are spread over the chunk's block classes at any time (the
    // table loop's LDS waits then overlap other wavefronts' far-field arithmetic) while the
    // chunk's sources stay in the scalar cache for all of them
    const int nb = b1 - b0;
    const int rot = ROT ? ((tile % kGroupTiles) * nb) / kGroupTiles : 0;
    Acc<Real> acc[NR];
    for (int jb = 0; jb < nb; ++jb) {
        int b = b0 + jb + rot;
        if (b >= b1) b -= nb;
        const int32_t* bb = a.sbox + 6 * b;
        const int bx0 = ldu(bb, 0), by0 = ldu(bb, 1), bz0 = ldu(bb, 2), bx1 = ldu(bb, 3), by1 = ldu(bb, 4),
                  bz1 = ldu(bb, 5);
        const int gap = max(max(max(bx0 - hx, lx - bx1), max(by0 - hy, ly - by1)), max(max(bz0 - hz, lz - bz1), 0));
        const int span = max(max(max(bx1 - lx, hx - bx0), max(by1 - ly, hy - by0)), max(bz1 - lz, hz - bz0));
        const int cls = block_class(gap, span, a.tab_r, a.far_ok != 0, sizeof(Real) == 4, a.far_gap);
        const int sb = b * kSourceBlock;        // blocks are full: the source arrays are padded
        if (cls == kClassTable) {
            // the next step's sources are loaded while this step's table reads are in
            // flight (the last step reloads its own: the block's end is the array's end)
            constexpr int UT = table_unroll<Real, NR>();
            Step<Real, NR, UT> st = load_step<Real, NR, true, false, false, UT>(a, sb);
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += UT) {
                Real G[UT];
                lookup_step<Real, UT, false>(L, nullptr, ix, iy, iz, st.x, st.y, st.z, G);
                const Step<Real, NR, UT> nx =
                    load_step<Real, NR, true, false, false, UT>(a, min(s0 + UT, sb + kSourceBlock - UT));
#pragma unroll
                for (int u = 0; u < UT; ++u)
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G[u] * st.w[r][u]);
                st = nx;
            }
        } else if (sizeof(Real) == 4 && cls == kClassFar2) {
            if (a.yukawa) far2_block<Real, NR, true>(a, txy, tzl, sb, acc);
            else far2_block<Real, NR, false>(a, txy, tzl, sb, acc);
        } else if ((cls == kClassFar || cls == kClassFar2) && !a.yukawa) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += U) {
                const Step<Real, NR> st = load_step<Real, NR, false, true>(a, s0);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const Real dx = fx - st.xr[u], dy = fy - st.yr[u], dz = fz - st.zr[u];
                    const Real G = far_field<Real>(dx * dx, dy * dy, dz * dz);
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * st.w[r][u]);
                }
            }
        } else if (cls == kClassFar || cls == kClassFar2) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += U) {
                const Step<Real, NR> st = load_step<Real, NR, false, true>(a, s0);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const Real dx = fx - st.xr[u], dy = fy - st.yr[u], dz = fz - st.zr[u];
                    const Real G = far_field_yukawa<Real>(dx * dx, dy * dy, dz * dz, a.kq, a.yk);
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * st.w[r][u]);
                }
            }
        } else if (cls == kClassGather) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += U) {
                const Step<Real, NR> st = load_step<Real, NR, true, false>(a, s0);
                Real G[U];
                lookup_step<Real, U, true>(L, a.full_tab, ix, iy, iz, st.x, st.y, st.z, G);
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G[u] * st.w[r][u]);
            }
        } else {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += U) {
                const Step<Real, NR> st = load_step<Real, NR, true, true>(a, s0);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t da = absdiff_s(ix, st.x[u]), db = absdiff_s(iy, st.y[u]), dc = absdiff_s(iz, st.z[u]);
                    Real G;
                    if (max3u(da, db, dc) <= tab_q) {
                        G = lds_value(L, table_offset(L, da, db, dc));
                    } else if (a.far_ok) {
                        const Real dx = fx - st.xr[u], dy = fy - st.yr[u], dz = fz - st.zr[u];
                        G = a.yukawa ? far_field_yukawa<Real>(dx * dx, dy * dy, dz * dz, a.kq, a.yk)
                                     : far_field<Real>(dx * dx, dy * dy, dz * dz);
                    } else {
                        G = global_value(a.full_tab, table_offset(L, da, db, dc));
                    }
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * st.w[r][u]);
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
