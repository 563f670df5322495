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
constexpr int unroll() { return 32 / (int)sizeof(Real); }   // sources per unrolled step (32-byte scalar loads)
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

template <typename Real>
__device__ __forceinline__ Real rsqrt_t(Real x);
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) { return rsqrt(x); }
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// q = 2 only (FP32 beyond kFar2Gap, where the q = 3 term is below 4.3e-8 relative).
// X, Y, Z: squared quantised offset components.
__device__ __forceinline__ float far_field_q2(float X, float Y, float Z) {
    const float r2 = X + Y + Z;
    const float e2 = fmaf(X, Y + Z, Y * Z);
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rho = rinv * rinv;
    const float x = e2 * rho * rho;
    return rinv * fmaf(rho, fmaf(float(C2), x, float(C1)), float(C0));
}

// Far field from the squared quantised offset components (all >= 0, not all 0).  FP64
// keeps the q = 4 term (|error| <= 6.6e-11 relative beyond the far-field gap); FP32 stops
// at q = 3, whose error there (<= 4.8e-9) is already below FP32 rounding.
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

// Fill the LDS table prefix (radius tab_r) and the index arrays up to radius idx_r.
template <typename Real>
__device__ __forceinline__ void fill_lds(const Lds<Real>& L, const Real* __restrict__ src, int tab_r, int idx_r) {
    const int n = (tab_r + 1) * (tab_r + 2) * (tab_r + 3) / 6;
    for (int i = threadIdx.x; i < n; i += blockDim.x) L.tab[i] = src[i];
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
    const uint32_t *tx, *ty, *tz;     // quantised target coordinates
    int nt;
    const uint32_t *sx, *sy, *sz;     // quantised source coordinates
    const Real *sxr, *syr, *szr;      // the same in the kernel's precision
    const int32_t* sbox;              // [nblk][6] quantised source block bounding boxes
    int ns, nblk, blk_per_chunk;
    const Real* w;
    int64_t ldw;
    const Real* near_tab;             // table prefix staged in LDS (radius tab_r)
    const Real* full_tab;             // full table (sigma > 0): radius full_r
    int tab_r;                        // LDS table radius used (<= the kernel's tab_radius)
    int full_r;
    int far_ok;
    double* part;
    int64_t ldp;
};

// One wavefront owns 64 consecutive (Morton-ordered) targets and walks the source blocks of
// one chunk.  From the bounding boxes of its targets and of each block it picks one loop
// with a wavefront-uniform branch (block_class):
//   table   every pair within the LDS table radius
//   far2    every pair beyond the q = 2 gap (FP32, sigma = 0): q = 2 expansion
//   far     every pair beyond the far-field gap, sigma = 0: expansion in registers
//   gather  every pair beyond the LDS radius, sigma > 0: the global table
//   mixed   per-pair choice between the LDS table and the far field / global table
template <typename Real, int NR>
__device__ __forceinline__ void sum_tile(const SumArgs<Real>& a, const Lds<Real>& L, int tile, int chunk) {
    const int lane = threadIdx.x & (kWave - 1);
    const int t = tile * kWave + lane;
    const int tc = min(t, a.nt - 1);
    const uint32_t ix = a.tx[tc], iy = a.ty[tc], iz = a.tz[tc];
    const Real fx = (Real)ix, fy = (Real)iy, fz = (Real)iz;
    const int lx = wave_min((int)ix), ly = wave_min((int)iy), lz = wave_min((int)iz);
    const int hx = wave_max((int)ix), hy = wave_max((int)iy), hz = wave_max((int)iz);
    const uint32_t tab_q = (uint32_t)(kQuant * a.tab_r);

    const int b0 = chunk * a.blk_per_chunk;
    const int b1 = min(a.nblk, b0 + a.blk_per_chunk);
    Acc<Real> acc[NR];
    for (int b = b0; b < b1; ++b) {
        const int32_t* bb = a.sbox + 6 * b;
        const int bx0 = ldu(bb, 0), by0 = ldu(bb, 1), bz0 = ldu(bb, 2), bx1 = ldu(bb, 3), by1 = ldu(bb, 4),
                  bz1 = ldu(bb, 5);
        const int gap = max(max(max(bx0 - hx, lx - bx1), max(by0 - hy, ly - by1)), max(max(bz0 - hz, lz - bz1), 0));
        const int span = max(max(max(bx1 - lx, hx - bx0), max(by1 - ly, hy - by0)), max(bz1 - lz, hz - bz0));
        const int cls = block_class(gap, span, a.tab_r, a.far_ok != 0, sizeof(Real) == 4);
        const int sb = b * kSourceBlock;        // blocks are full: the source arrays are padded
        if (cls == kClassTable) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += unroll<Real>()) {
#pragma unroll
                for (int u = 0; u < unroll<Real>(); ++u) {
                    const int s = s0 + u;
                    const uint32_t off =
                        table_offset(L, absdiff_s(ix, ldu(a.sx, s)), absdiff_s(iy, ldu(a.sy, s)), absdiff_s(iz, ldu(a.sz, s)));
                    const Real G = lds_value(L, off);
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * ldu(a.w, r * a.ldw + s));
                }
            }
        } else if (cls == kClassFar2) {
            if constexpr (sizeof(Real) == 4) {
                for (int s0 = sb; s0 < sb + kSourceBlock; s0 += unroll<Real>()) {
#pragma unroll
                    for (int u = 0; u < unroll<Real>(); ++u) {
                        const int s = s0 + u;
                        const float dx = fx - ldu(a.sxr, s), dy = fy - ldu(a.syr, s), dz = fz - ldu(a.szr, s);
                        const Real G = far_field_q2(dx * dx, dy * dy, dz * dz);
#pragma unroll
                        for (int r = 0; r < NR; ++r) acc[r].add(G * ldu(a.w, r * a.ldw + s));
                    }
                }
            }
        } else if (cls == kClassFar) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += unroll<Real>()) {
#pragma unroll
                for (int u = 0; u < unroll<Real>(); ++u) {
                    const int s = s0 + u;
                    const Real dx = fx - ldu(a.sxr, s), dy = fy - ldu(a.syr, s), dz = fz - ldu(a.szr, s);
                    const Real G = far_field<Real>(dx * dx, dy * dy, dz * dz);
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * ldu(a.w, r * a.ldw + s));
                }
            }
        } else if (cls == kClassGather) {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += unroll<Real>()) {
#pragma unroll
                for (int u = 0; u < unroll<Real>(); ++u) {
                    const int s = s0 + u;
                    const uint32_t off =
                        table_offset(L, absdiff_s(ix, ldu(a.sx, s)), absdiff_s(iy, ldu(a.sy, s)), absdiff_s(iz, ldu(a.sz, s)));
                    const Real G = global_value(a.full_tab, off);
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * ldu(a.w, r * a.ldw + s));
                }
            }
        } else {
            for (int s0 = sb; s0 < sb + kSourceBlock; s0 += unroll<Real>()) {
#pragma unroll
                for (int u = 0; u < unroll<Real>(); ++u) {
                    const int s = s0 + u;
                    const uint32_t da = absdiff_s(ix, ldu(a.sx, s)), db = absdiff_s(iy, ldu(a.sy, s)),
                                   dc = absdiff_s(iz, ldu(a.sz, s));
                    Real G;
                    if (max3u(da, db, dc) <= tab_q) {
                        G = lds_value(L, table_offset(L, da, db, dc));
                    } else if (a.far_ok) {
                        const Real dx = fx - ldu(a.sxr, s), dy = fy - ldu(a.syr, s), dz = fz - ldu(a.szr, s);
                        G = far_field<Real>(dx * dx, dy * dy, dz * dz);
                    } else {
                        G = global_value(a.full_tab, table_offset(L, da, db, dc));
                    }
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r].add(G * ldu(a.w, r * a.ldw + s));
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
