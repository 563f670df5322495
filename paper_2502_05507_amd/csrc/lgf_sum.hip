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
// coordinates and weights come through scalar loads.  Sources come in Morton blocks of 64
// with bounding boxes, so each wavefront classifies a whole block (all far, all near, or
// mixed) with one uniform branch.  The grid is (target tiles) x (source chunks); each
// block writes its partial sums, reduced later in a fixed order (deterministic results).
// FP32 pairs are summed in FP32 over each source block and the block sums folded into a
// Neumaier-compensated FP32 accumulator.
#include <algorithm>

#include "lgf_device.hpp"
#include "ops.hpp"

namespace bae {

using namespace lgfdev;

namespace {

template <typename Real, int NR>
__global__ __launch_bounds__(kBlock) void lgf_sum_kernel(const SumArgs<Real> a) {
    __shared__ Real tab[kNearE];
    for (int i = threadIdx.x; i < kNearE; i += kBlock) tab[i] = a.near_tab[i];
    __syncthreads();
    sum_tile<Real, NR>(a, tab, blockIdx.x, blockIdx.y);
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


// ------------------------------------------------------------------ 16-RHS blocked form on MFMA
// For 16 right-hand sides the sum is the dense product V(T x 16) = K(T x S) W(S x 16), with
// K(t, s) = G(t - s) never stored: every wavefront generates a 16 x 4 slice of K per step
// (one kernel value per lane, exactly as in the VALU kernel) and contracts it with the
// matching 4 x 16 slice of W on the matrix cores (v_mfma_{f32,f64}_16x16x4).
// Operand layouts (16x16x4, measured on gfx950): A[i][k] in lane 16k + i, B[k][j] in lane
// 16k + j; the result D[i][j] sits in lane 16v' + j, element v, with i = 4v' + v for f32
// and i = v' + 4v for f64.
// A wavefront owns kTiles tiles of 16 targets (64 targets, the same patch as the VALU
// kernel, so the same near/far block classification applies); a workgroup of 4 wavefronts
// stages each source block's 64 x 16 weights in LDS once for all of them.
constexpr int kTiles = 4;

template <typename Real>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
    using V = __attribute__((__vector_size__(4 * sizeof(float)))) float;
    __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct MfmaAcc<double> {
    using V = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

template <typename Real>
__global__ __launch_bounds__(kBlock) void lgf_sum_mfma_kernel(const SumArgs<Real> a) {
    using V = typename MfmaAcc<Real>::V;
    __shared__ Real tab[kNearE];
    __shared__ Real wl[kSourceBlock][16];
    for (int i = threadIdx.x; i < kNearE; i += kBlock) tab[i] = a.near_tab[i];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row = lane & 15;            // A row (target within a tile) / B, D column (RHS)
    const int kq = lane >> 4;             // A column / B row (source within the step of 4)
    const int base = (blockIdx.x * (kBlock / 64) + wave) * (16 * kTiles);
    int ix[kTiles], iy[kTiles], iz[kTiles];
    Real fx[kTiles], fy[kTiles], fz[kTiles];
    int lx = 1 << 30, ly = 1 << 30, lz = 1 << 30, hx = -(1 << 30), hy = -(1 << 30), hz = -(1 << 30);
#pragma unroll
    for (int j = 0; j < kTiles; ++j) {
        const int tc = min(base + 16 * j + row, a.nt - 1);
        ix[j] = a.tx[tc];
        iy[j] = a.ty[tc];
        iz[j] = a.tz[tc];
        fx[j] = (Real)ix[j];
        fy[j] = (Real)iy[j];
        fz[j] = (Real)iz[j];
        lx = min(lx, ix[j]);
        ly = min(ly, iy[j]);
        lz = min(lz, iz[j]);
        hx = max(hx, ix[j]);
        hy = max(hy, iy[j]);
        hz = max(hz, iz[j]);
    }
    lx = wave_min(lx);
    ly = wave_min(ly);
    lz = wave_min(lz);
    hx = wave_max(hx);
    hy = wave_max(hy);
    hz = wave_max(hz);

    V acc[kTiles], comp[kTiles];
#pragma unroll
    for (int j = 0; j < kTiles; ++j)
        for (int v = 0; v < 4; ++v) acc[j][v] = comp[j][v] = Real(0);

    const int b0 = blockIdx.y * a.blk_per_chunk;
    const int b1 = min(a.nblk, b0 + a.blk_per_chunk);
    for (int b = b0; b < b1; ++b) {
        const int sb = b * kSourceBlock;
        __syncthreads();
        for (int i = threadIdx.x; i < kSourceBlock * 16; i += kBlock) {
            const int r = i / kSourceBlock, sl = i % kSourceBlock;
            wl[sl][r] = a.w[r * a.ldw + sb + sl];
        }
        __syncthreads();
        const int32_t* bb = a.sbox + 6 * b;
        const int gap = max(max(max(bb[0] - hx, lx - bb[3]), max(bb[1] - hy, ly - bb[4])),
                            max(max(bb[2] - hz, lz - bb[5]), 0));
        const int span = max(max(max(bb[3] - lx, hx - bb[0]), max(bb[4] - ly, hy - bb[1])),
                             max(bb[5] - lz, hz - bb[2]));
        const int mode = (gap > kNearR) ? (a.far_ok ? 0 : 1) : (span <= kNearR ? 2 : 3);
        V blk[kTiles];
#pragma unroll
        for (int j = 0; j < kTiles; ++j)
            for (int v = 0; v < 4; ++v) blk[j][v] = Real(0);
        for (int st = 0; st < kSourceBlock; st += 4) {
            const int s = sb + st + kq;
            const Real wb = wl[st + kq][row];
            Real G[kTiles];
            if (mode == 0) {
                const Real sx = a.sxr[s], sy = a.syr[s], sz = a.szr[s];
#pragma unroll
                for (int j = 0; j < kTiles; ++j) {
                    const Real dx = fx[j] - sx, dy = fy[j] - sy, dz = fz[j] - sz;
                    G[j] = far_field<Real>(dx * dx, dy * dy, dz * dz);
                }
            } else {
                const int sx = a.sx[s], sy = a.sy[s], sz = a.sz[s];
                if (mode == 1) {
#pragma unroll
                    for (int j = 0; j < kTiles; ++j)
                        G[j] = a.full_tab[sorted_index64((uint32_t)abs(ix[j] - sx), (uint32_t)abs(iy[j] - sy),
                                                         (uint32_t)abs(iz[j] - sz))];
                } else if (mode == 2) {
#pragma unroll
                    for (int j = 0; j < kTiles; ++j)
                        G[j] = tab[sorted_index((uint32_t)abs(ix[j] - sx), (uint32_t)abs(iy[j] - sy),
                                                (uint32_t)abs(iz[j] - sz))];
                } else {
#pragma unroll
                    for (int j = 0; j < kTiles; ++j)
                        G[j] = eval_pair<Real>(ix[j] - sx, iy[j] - sy, iz[j] - sz, tab, a.full_tab, a.far_ok != 0);
                }
            }
#pragma unroll
            for (int j = 0; j < kTiles; ++j) blk[j] = MfmaAcc<Real>::mma(G[j], wb, blk[j]);
        }
        // fold the block's sums into the running (compensated, for FP32) accumulators
#pragma unroll
        for (int j = 0; j < kTiles; ++j)
            for (int v = 0; v < 4; ++v) {
                if constexpr (sizeof(Real) == 4) {
                    const Real x = blk[j][v], sum = acc[j][v];
                    const Real t = sum + x;
                    comp[j][v] += fabs(sum) >= fabs(x) ? (sum - t) + x : (x - t) + sum;
                    acc[j][v] = t;
                } else {
                    acc[j][v] += blk[j][v];
                }
            }
    }
    // element v of lane (kq, row): D[i][row], i = 4 kq + v (f32) or kq + 4 v (f64)
#pragma unroll
    for (int j = 0; j < kTiles; ++j)
        for (int v = 0; v < 4; ++v) {
            const int i = sizeof(Real) == 4 ? 4 * kq + v : kq + 4 * v;
            const int t = base + 16 * j + i;
            if (t < a.nt)
                a.part[(int64_t)row * a.ldp + (int64_t)blockIdx.y * a.nt + t] =
                    (double)acc[j][v] + (double)comp[j][v];
        }
}

template <typename Real>
const Real* coord(const PointSet& P, int axis);
template <>
const float* coord<float>(const PointSet& P, int axis) {
    return axis == 0 ? P.xf : axis == 1 ? P.yf : P.zf;
}
template <>
const double* coord<double>(const PointSet& P, int axis) {
    return axis == 0 ? P.xd : axis == 1 ? P.yd : P.zd;
}

template <typename Real>
void launch_all(const PointSet& T, const PointSet& S, const Real* w, int nrhs, const Real* near, const Real* full,
                bool far, double* part, int chunks, hipStream_t st) {
    SumArgs<Real> a;
    a.tx = T.x;
    a.ty = T.y;
    a.tz = T.z;
    a.nt = (int)T.count;
    a.sx = S.x;
    a.sy = S.y;
    a.sz = S.z;
    a.sxr = coord<Real>(S, 0);
    a.syr = coord<Real>(S, 1);
    a.szr = coord<Real>(S, 2);
    a.sbox = S.bbox;
    a.ns = (int)S.count;
    a.nblk = (int)S.nblk;
    a.blk_per_chunk = (int)((S.nblk + chunks - 1) / chunks);
    a.ldw = S.padded;
    a.near_tab = near;
    a.full_tab = full;
    a.far_ok = far ? 1 : 0;
    a.ldp = (int64_t)chunks * T.count;
    const dim3 grid((unsigned)((T.count + kBlock - 1) / kBlock), (unsigned)chunks);
    const int per_block = (kBlock / 64) * 16 * kTiles;
    const dim3 grid_mfma((unsigned)((T.count + per_block - 1) / per_block), (unsigned)chunks);
    int r = 0;
    while (r < nrhs) {
        const int left = nrhs - r;
        SumArgs<Real> ar = a;
        ar.w = w + (int64_t)r * a.ldw;
        ar.part = part + (int64_t)r * a.ldp;
        if (left >= 16) {
            lgf_sum_mfma_kernel<Real><<<grid_mfma, kBlock, 0, st>>>(ar);
            r += 16;
        } else if (left >= 4) {
            lgf_sum_kernel<Real, 4><<<grid, kBlock, 0, st>>>(ar);
            r += 4;
        } else {
            lgf_sum_kernel<Real, 1><<<grid, kBlock, 0, st>>>(ar);
            r += 1;
        }
        BAE_HIP_CHECK(hipGetLastError());
    }
}

}  // namespace

int lgf_near_radius() { return kNearR; }
int lgf_far2_gap() { return kFar2R; }

int lgf_sum_chunks(int64_t nt, int64_t ns) {
    const int64_t tiles = (nt + kBlock - 1) / kBlock;
    int64_t chunks = (2048 + tiles - 1) / tiles;           // aim at >= 2048 blocks
    chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, ns / (8 * kSourceBlock)));
    return (int)std::max<int64_t>(1, std::min<int64_t>(chunks, 64));
}

int lgf_sum_launch(const PointSet& T, const PointSet& S, const void* w, int nrhs, int prec, const SumTables& tabs,
                   double* part, int64_t part_capacity, hipStream_t st) {
    if (T.count == 0) return 0;
    int chunks = lgf_sum_chunks(T.count, S.count);
    while (chunks > 1 && (int64_t)chunks * T.count * nrhs > part_capacity) --chunks;
    if ((int64_t)chunks * T.count * nrhs > part_capacity) throw Error{BAE_ERR_ARG, "partial-sum buffer too small"};
    if (tabs.full_r < kNearR) throw Error{BAE_ERR_ARG, "resident table radius below the LDS radius"};
    if (S.count == 0) {
        launch_fill(part, (int64_t)chunks * T.count * nrhs, 0.0, st);
        return chunks;
    }
    if (prec == BAE_PREC_FP64)
        launch_all<double>(T, S, (const double*)w, nrhs, tabs.near64, tabs.full64, tabs.far_field, part, chunks, st);
    else
        launch_all<float>(T, S, (const float*)w, nrhs, tabs.near32, tabs.full32, tabs.far_field, part, chunks, st);
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
