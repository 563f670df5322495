// The LGF sum: v[r][t] = sum_s w[r][s] G_s(T_t - S_s) over integer lattice points.
//
// Paper Sec. 3.2: the double layer potential sum_{n in gamma-} q_d(n) sum_{k in D_n}
// [G(m-n) - G(m-k)] is, after collecting coefficients per source point, one LGF sum over
// the sources gamma- u E with weights w(n) = |D_n| q_d(n), w(k) = -sum_{n: k in D_n} q_d(n)
// (the weights are formed by bae_weights_kernel; this file evaluates the sum).  The same
// sum with sources M+ and weights h^2 f gives the free-space volume potential u_p.
//
// Kernel evaluation per (target, source) pair, offset d = T - S, c = max |d_i|:
//   c <= RN : LDS-resident 1/48-symmetric table, index of the sorted |d| triple
//   c >  RN : sigma = 0 -> far-field expansion in registers (below);
//             sigma > 0 -> the full FP64/FP32 table in global memory (L2 / MALL resident)
// Far field (sigma = 0): Sec. 2.2 q-term expansion in the positive sign convention,
//   G_0(n) = (1/(4 pi |n|)) [1 + rho (1 - 5x)/4 + rho^2 P8/32 + rho^3 P12/128] + O(|n|^-9),
//   rho = 1/|n|^2, x = e2 rho^2, y = e3 rho^3, e2 = j^2k^2 + k^2l^2 + l^2j^2, e3 = j^2k^2l^2,
//   P8  = 23 - 336x + 1155x^2 - 1134y   (the paper's q = 3 bracket with -228 in place of
//                                        the printed -288; symmetric-polynomial form)
//   P12 = 647 - 20301x + 178035x^2 - 425425x^3 - 208494y + 810810xy
//        (the q = 4 term, derived for this library by the same Fourier-symbol expansion of
//         1/(6 - 2 sum cos) that yields the paper's terms; relative error 6.6e-11 at |n| = 32
//         on the axis, the worst direction, and 2.5e-13 at 64).
//
// Layout and launch: targets and sources are in Morton order (SoA int32 x, y, z), so the
// 64 targets of a wavefront form a compact patch and near/far branches are mostly uniform.
// One thread owns one target; the source loop index is wavefront-uniform, so source
// coordinates and weights come through scalar loads.  The grid is (target tiles) x (source
// chunks); each block writes its partial sums, reduced later in a fixed order
// (deterministic results).  FP32 pairs are summed in FP32 over runs of 32 sources and
// the run sums folded into a Neumaier-compensated FP32 accumulator.
#include <algorithm>

#include "ops.hpp"

namespace bae {

namespace {

constexpr int kBlock = 256;
constexpr int kNearR = 32;                           // LDS table radius (both precisions)
constexpr int kNearE = (kNearR + 1) * (kNearR + 2) * (kNearR + 3) / 6;
constexpr int kRun = 32;                             // FP32 run length before compensation

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

// far field for an integer offset with squares X, Y, Z (all >= 0, not all 0)
template <typename Real>
__device__ __forceinline__ Real far_field(Real X, Real Y, Real Z) {
    const Real r2 = X + Y + Z;
    const Real e2 = fma(X, Y + Z, Y * Z);
    const Real e3 = X * Y * Z;
    const Real rinv = rsqrt_t<Real>(r2);
    const Real rho = rinv * rinv;
    const Real rho2 = rho * rho;
    const Real x = e2 * rho2;
    const Real y = e3 * rho2 * rho;
    const Real f = fma(y, fma(Real(F5), x, Real(F4)), fma(x, fma(x, fma(x, Real(F3), Real(F2)), Real(F1)), Real(F0)));
    const Real d = fma(Real(D3), y, fma(x, fma(x, Real(D2), Real(D1)), Real(D0)));
    const Real c = fma(Real(C2), x, Real(C1));
    const Real B = fma(rho, fma(rho, fma(rho, f, d), c), Real(C0));
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

template <typename Real, int NR>
__global__ __launch_bounds__(kBlock) void lgf_sum_kernel(
    const int32_t* __restrict__ tx, const int32_t* __restrict__ ty, const int32_t* __restrict__ tz, int nt,
    const int32_t* __restrict__ sx, const int32_t* __restrict__ sy, const int32_t* __restrict__ sz,
    const Real* __restrict__ w, int64_t ldw, int ns, int chunk_len, const Real* __restrict__ near_tab,
    int near_entries, const Real* __restrict__ full_tab, int far_ok, double* __restrict__ part, int64_t ldp) {
    __shared__ Real tab[kNearE];
    for (int i = threadIdx.x; i < near_entries; i += kBlock) tab[i] = near_tab[i];
    __syncthreads();

    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int tc = min(t, nt - 1);
    const int x = tx[tc], y = ty[tc], z = tz[tc];
    const int s0 = blockIdx.y * chunk_len;
    const int s1 = min(ns, s0 + chunk_len);
    const bool ff = far_ok != 0;

    Acc<Real> acc[NR];
    for (int sb = s0; sb < s1; sb += kRun) {
        const int se = min(s1, sb + kRun);
        for (int s = sb; s < se; ++s) {
            const Real G = eval_pair<Real>(x - sx[s], y - sy[s], z - sz[s], tab, full_tab, ff);
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r].add(G * w[r * ldw + s]);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r].flush();
    }
    if (t < nt) {
#pragma unroll
        for (int r = 0; r < NR; ++r) part[(int64_t)r * ldp + (int64_t)blockIdx.y * nt + t] = acc[r].value();
    }
}

template <typename Real>
__global__ void lgf_eval_kernel(const int32_t* __restrict__ off, int64_t count, const Real* __restrict__ near_tab,
                                const Real* __restrict__ full_tab, int full_r, int far_ok, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int dx = off[3 * i], dy = off[3 * i + 1], dz = off[3 * i + 2];
    const int m = max(abs(dx), max(abs(dy), abs(dz)));
    if (m > full_r && !far_ok) {
        out[i] = __builtin_nan("");
        return;
    }
    out[i] = (double)eval_pair<Real>(dx, dy, dz, near_tab, full_tab, far_ok != 0);
}

template <typename Real, int NR>
void launch_nr(const PointSet& T, const PointSet& S, const Real* w, int64_t ldw, const Real* near,
               int near_entries, const Real* full, bool far, double* part, int64_t ldp, int chunks,
               int chunk_len, hipStream_t st) {
    dim3 grid((unsigned)((T.count + kBlock - 1) / kBlock), (unsigned)chunks);
    lgf_sum_kernel<Real, NR><<<grid, kBlock, 0, st>>>(T.x, T.y, T.z, (int)T.count, S.x, S.y, S.z, w, ldw,
                                                      (int)S.count, chunk_len, near, near_entries, full,
                                                      far ? 1 : 0, part, ldp);
    BAE_HIP_CHECK(hipGetLastError());
}

template <typename Real>
void launch_all(const PointSet& T, const PointSet& S, const Real* w, int nrhs, const Real* near, int near_entries,
                const Real* full, bool far, double* part, int chunks, int chunk_len, hipStream_t st) {
    const int64_t ldw = S.count;
    const int64_t ldp = (int64_t)chunks * T.count;
    int r = 0;
    while (r < nrhs) {
        const int left = nrhs - r;
        const Real* wr = w + (int64_t)r * ldw;
        double* pr = part + (int64_t)r * ldp;
        if (left >= 16) {
            launch_nr<Real, 16>(T, S, wr, ldw, near, near_entries, full, far, pr, ldp, chunks, chunk_len, st);
            r += 16;
        } else if (left >= 4) {
            launch_nr<Real, 4>(T, S, wr, ldw, near, near_entries, full, far, pr, ldp, chunks, chunk_len, st);
            r += 4;
        } else {
            launch_nr<Real, 1>(T, S, wr, ldw, near, near_entries, full, far, pr, ldp, chunks, chunk_len, st);
            r += 1;
        }
    }
}

}  // namespace

int lgf_near_radius() { return kNearR; }

int lgf_sum_chunks(int64_t nt, int64_t ns) {
    const int64_t tiles = (nt + kBlock - 1) / kBlock;
    int64_t chunks = (2048 + tiles - 1) / tiles;           // aim at >= 2048 blocks
    chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, ns / 512));
    return (int)std::max<int64_t>(1, std::min<int64_t>(chunks, 64));
}

int lgf_sum_launch(const PointSet& T, const PointSet& S, const void* w, int nrhs, int prec, const SumTables& tabs,
                   double* part, int64_t part_capacity, hipStream_t st) {
    if (T.count == 0) return 0;
    int chunks = lgf_sum_chunks(T.count, S.count);
    while (chunks > 1 && (int64_t)chunks * T.count * nrhs > part_capacity) --chunks;
    if ((int64_t)chunks * T.count * nrhs > part_capacity) throw Error{BAE_ERR_ARG, "partial-sum buffer too small"};
    const int chunk_len = (int)((S.count + chunks - 1) / chunks);
    if (tabs.full_r < kNearR) throw Error{BAE_ERR_ARG, "resident table radius below the LDS radius"};
    const int near_entries = kNearE;
    if (S.count == 0) {
        launch_fill(part, (int64_t)chunks * T.count * nrhs, 0.0, st);
        return chunks;
    }
    if (prec == BAE_PREC_FP64)
        launch_all<double>(T, S, (const double*)w, nrhs, tabs.near64, near_entries, tabs.full64, tabs.far_field, part,
                           chunks, chunk_len, st);
    else
        launch_all<float>(T, S, (const float*)w, nrhs, tabs.near32, near_entries, tabs.full32, tabs.far_field, part,
                          chunks, chunk_len, st);
    return chunks;
}

void lgf_eval_launch(const int32_t* off, int64_t count, double* out, int prec, const SumTables& tabs, hipStream_t st) {
    if (count == 0) return;
    const unsigned blocks = (unsigned)((count + 255) / 256);
    if (prec == BAE_PREC_FP64)
        lgf_eval_kernel<double><<<blocks, 256, 0, st>>>(off, count, tabs.near64, tabs.full64, tabs.full_r,
                                                        tabs.far_field ? 1 : 0, out);
    else
        lgf_eval_kernel<float><<<blocks, 256, 0, st>>>(off, count, tabs.near32, tabs.full32, tabs.full_r,
                                                       tabs.far_field ? 1 : 0, out);
    BAE_HIP_CHECK(hipGetLastError());
}

}  // namespace bae
