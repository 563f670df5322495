// The LGF sum: v[r][t] = sum_s w[r][s] G_s(T_t - S_s) over integer lattice points.
//
// Paper Sec. 3.2: the double layer potential sum_{n in gamma-} q_d(n) sum_{k in D_n}
// [G(m-n) - G(m-k)] is, after collecting coefficients per source point, one LGF sum over
// the sources gamma- u E with weights w(n) = |D_n| q_d(n), w(k) = -sum_{n: k in D_n} q_d(n)
// (the weights are formed by bae_weights_kernel; this file evaluates the sum).  The same
// sum with sources M+ and weights h^2 f gives the free-space volume potential u_p.
//
// Kernel evaluation per (target, source) pair, offset d = T - S, c = max |d_i|:
//   c <= RL : the LDS-resident prefix of the 1/48-symmetric table (sigma = 0: RL = 60 in
//             FP32, 47 in FP64, 159 / 157 KB of the 160 KB LDS of a gfx950 compute unit;
//             sigma > 0: 59 / 46, next to the index arrays that span the global table)
//   c >  RL : sigma = 0 -> far-field expansion in registers (valid beyond 32, below; q = 4
//             in FP64, q = 2 in FP32, where the FP32 rounding of the sum dominates);
//             sigma > 0 -> the full FP64/FP32 table in global memory (L2 / MALL resident)
// A table lookup costs 8 VALU instructions per pair, the FP32 far field 15 and the FP64 one
// 37, so every block pair that fits the LDS table is evaluated from it.
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
// Layout and launch: targets and sources are in Morton order, so the 64 targets of a
// wavefront form a compact patch.  One thread owns one target; the source index is
// wavefront-uniform, so source coordinates and weights come through scalar loads.  Sources
// come in Morton blocks of 64 with bounding boxes, so each wavefront classifies a whole
// block with one uniform branch.  The grid is persistent: one 1024-thread workgroup per
// compute unit stages the LDS table once and takes work items (16 consecutive 64-target
// tiles, source chunk) -- its first in a fixed assignment, the rest from an atomic counter
// -- from a list ordered by decreasing estimated cost, handing the item's tiles to its
// wavefronts (for_each_item).  Each (tile, chunk) writes its own partial sums, reduced
// later in a fixed order, so results do not depend on the schedule.
// FP32 pairs are summed in FP32 over each source block and the block sums folded into a
// Neumaier-compensated FP32 accumulator.
#include <algorithm>
#include <map>
#include <mutex>

#include "lgf_device.hpp"
#include "ops.hpp"

namespace bae {

using namespace lgfdev;

namespace {

struct Sched {
    const int32_t* skip;   // non-null and set: the whole sum is skipped (a converged solve)
    const uint32_t* items; // group | chunk << 20, by decreasing cost
    uint32_t nitems;
    uint32_t ntiles;       // 64-target tiles
    unsigned long long* counter;   // hands out items G.. (a type no input array has: its
                                   // atomics cannot alias the inputs, whose uniform loads
                                   // then stay scalar); 0 between launches
    int32_t* err;          // set to 1 (system scope) when a bounded wait gives up
    uint32_t polls;        // polls of each bounded wait before it gives up (0: at once)
};

// Per-workgroup hand-off of work items in LDS: a ring of the global item indices of the
// workgroup's next local items, each with its local number as tag, and the number of units
// of it whose wavefronts have read it.
constexpr uint32_t kRing = 4;
struct ItemRing {
    uint32_t units;             // (local item, tile) units handed out so far
    uint32_t item[kRing];
    uint32_t tag[kRing];        // local item number held, ~0 when none
    uint32_t readers[kRing];    // units of it that have read the slot (kGroupTiles when free)
};

__device__ __forceinline__ void ring_init(ItemRing* r) {
    if (threadIdx.x == 0) r->units = 0;
    if (threadIdx.x < kRing) {
        r->tag[threadIdx.x] = ~0u;
        r->readers[threadIdx.x] = kGroupTiles;
    }
}

// A bounded wait that gives up ends its wavefront's work loop and reports it: the sum's
// partial results are then incomplete and the work counter is left mid-way, so the host
// (which polls the error word after the launch) fails the call and resets the counter.
__device__ __forceinline__ void give_up(const Sched& q) {
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(q.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The work loop of one wavefront.  Items are (group of kGroupTiles consecutive target
// tiles, source chunk), by decreasing cost.  A workgroup's local item 0 is item b (its
// index among the G workgroups); each further one comes from the global counter (item
// G + value), fetched one item ahead by the wavefront that takes the first unit of the
// item before.  The workgroup hands the (item, tile) units to its wavefronts in order from
// an LDS counter, so its wavefronts walk the same source blocks at about the same time and
// their scalar loads of the sources hit the scalar cache for all but the first (a wavefront
// on a source chunk of its own misses that cache on every other step and leaves the table
// loop waiting on the miss traffic).  The counter hands out exactly nitems values in all;
// the workgroup that draws the last one resets it for the next launch.
template <typename F>
__device__ __forceinline__ void for_each_item(const Sched& q, ItemRing* r, F&& body) {
    if (q.skip && ldu(q.skip, 0)) return;   // uniform: a converged solve skips the sum
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t G = gridDim.x;
    for (;;) {
        uint32_t u = 0;
        if (lane == 0) u = __hip_atomic_fetch_add(&r->units, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        u = __builtin_amdgcn_readfirstlane(u);
        const uint32_t k = u / kGroupTiles, part = u % kGroupTiles;
        uint32_t idx = blockIdx.x;
        if (k > 0) {
            const uint32_t s = k % kRing;
            for (uint32_t polls = 0;; ++polls) {
                if (polls >= q.polls) {
                    give_up(q);
                    return;
                }
                if (__hip_atomic_load(&r->tag[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == k) break;
                __builtin_amdgcn_s_sleep(1);
            }
            idx = __builtin_amdgcn_readfirstlane(r->item[s]);
            if (lane == 0) __hip_atomic_fetch_add(&r->readers[s], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (idx >= q.nitems) return;
        if (part == 0) {
            // fetch the next local item into its slot, once the item three before has left it
            uint32_t v = 0;
            if (lane == 0)
                v = (uint32_t)__hip_atomic_fetch_add(q.counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            v = __builtin_amdgcn_readfirstlane(v);
            if (v == q.nitems - 1 && lane == 0)
                __hip_atomic_store(q.counter, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t s = (k + 1) % kRing;
            for (uint32_t polls = 0;; ++polls) {
                if (polls >= q.polls) {
                    give_up(q);
                    return;
                }
                if (__hip_atomic_load(&r->readers[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == kGroupTiles)
                    break;
                __builtin_amdgcn_s_sleep(1);
            }
            if (lane == 0) {
                r->item[s] = G + v;
                r->readers[s] = 0;
                __hip_atomic_store(&r->tag[s], k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        const uint32_t it = ldu(q.items, idx);
        const uint32_t t = (it & 0xFFFFFu) * (uint32_t)kGroupTiles + part;
        if (t < q.ntiles) body(t, it >> 20);
    }
}

template <typename Real, int NR, int THREADS, bool FAR>
__global__ __launch_bounds__(THREADS) void lgf_sum_kernel(const SumArgs<Real> a, const Sched q) {
    __shared__ __align__(16) char lds[lds_bytes<Real, FAR>()];
    const Lds<Real> L = lds_layout<Real, FAR>(lds);
    __shared__ ItemRing ring;
    ring_init(&ring);
    fill_lds(L, a.near_tab, a.tab_r, FAR ? a.tab_r : a.full_r);
    __syncthreads();
    for_each_item(q, &ring, [&](uint32_t tile, uint32_t chunk) { sum_tile<Real, NR>(a, L, (int)tile, (int)chunk); });
}

template <typename Real>
__global__ void lgf_eval_kernel(const int32_t* __restrict__ off, int64_t count, const Real* __restrict__ tab,
                                int tab_r, int full_r, int far_ok, int yukawa, Real kq, Real yk,
                                const YukawaLattice yl, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t a = abs(off[3 * i]), b = abs(off[3 * i + 1]), c = abs(off[3 * i + 2]);
    const int64_t m = max(a, max(b, c));
    if (m > tab_r && far_ok) {
        const Real X = Real(kQuant * a), Y = Real(kQuant * b), Z = Real(kQuant * c);
        if constexpr (sizeof(Real) == 4) {
            // the forms of the sum's far blocks (lattice units)
            const float x2 = float(a * a), y2 = float(b * b), z2 = float(c * c);
            out[i] = yukawa ? (double)far_field_yukawa_lattice(x2 + y2 + z2, z2, y2 - x2, yl)
                            : (double)(kFarScale32 * far_field_q2_lattice(x2 + y2 + z2, z2, y2 - x2));
        } else if (yukawa) {
            out[i] = (double)far_field_yukawa<Real>(X * X, Y * Y, Z * Z, kq, yk);
        } else {
            out[i] = (double)far_field<Real>(X * X, Y * Y, Z * Z);
        }
        return;
    }
    if (m > full_r) {
        out[i] = __builtin_nan("");
        return;
    }
    const int64_t lo = min(a, min(b, c)), hi = m, mid = a + b + c - lo - hi;
    out[i] = (double)tab[hi * (hi + 1) * (hi + 2) / 6 + mid * (mid + 1) / 2 + lo];
}

// Relative difference of the sigma > 0 far-field form (in FP64) and the table, over every
// entry whose largest index lies in (from_r, R]; one maximum per block.
__global__ void yukawa_check_kernel(const double* __restrict__ tab, int64_t e0, int64_t e1, double kq, double yk,
                                    double* __restrict__ block_max) {
    __shared__ double sh[256];
    double worst = 0.0;
    for (int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += (int64_t)gridDim.x * blockDim.x) {
        // invert the sorted index e = c(c+1)(c+2)/6 + b(b+1)/2 + a
        int64_t c = (int64_t)cbrt(6.0 * (double)e);
        while (c * (c + 1) * (c + 2) / 6 > e) --c;
        while ((c + 1) * (c + 2) * (c + 3) / 6 <= e) ++c;
        const int64_t rem = e - c * (c + 1) * (c + 2) / 6;
        int64_t b = (int64_t)sqrt(2.0 * (double)rem);
        while (b * (b + 1) / 2 > rem) --b;
        while ((b + 1) * (b + 2) / 2 <= rem) ++b;
        const int64_t a = rem - b * (b + 1) / 2;
        const double X = double(kQuant * a), Y = double(kQuant * b), Z = double(kQuant * c);
        const double f = far_field_yukawa<double>(X * X, Y * Y, Z * Z, kq, yk);
        worst = fmax(worst, fabs(f - tab[e]) / fabs(tab[e]));
    }
    sh[threadIdx.x] = worst;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) block_max[blockIdx.x] = sh[0];
}

// ------------------------------------------------------------------ 16-RHS blocked form on MFMA
// For 16 right-hand sides the sum is the dense product V(T x 16) = K(T x S) W(S x 16), with
// K(t, s) = G(t - s) never stored: every wavefront generates a 16 x 4 slice of K per step
// (one kernel value per lane, exactly as in the VALU kernel) and contracts it with the
// matching 4 x 16 slice of W on the matrix cores (v_mfma_{f32,f64}_16x16x4).
// Operand layouts (16x16x4, measured on gfx950): A[i][k] in lane 16k + i, B[k][j] in lane
// 16k + j; the result D[i][j] sits in lane 16v' + j, element v, with i = 4v' + v for f32
// and i = v' + 4v for f64.
// A wavefront owns kTiles tiles of 16 targets (the 64 targets of one work item, so the
// block classification is the VALU kernel's).
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

// FP32 far block (every pair beyond the far-field gap): the lattice-form far field from the
// binary16 differences, with the next step's source and weight loads in flight while this
// step is evaluated.  The 16 steps are unrolled so that every load addresses its block by an
// immediate offset from three per-lane pointers set once per block.  The products add to the
// running block sums blk (several blocks are summed before they are folded).
template <bool YUK>
__device__ __forceinline__ void mfma_far2_block(const SumArgs<float>& a, const uint32_t (&txy)[kTiles],
                                                const float (&tzl)[kTiles], int sb, int row, int kq,
                                                MfmaAcc<float>::V (&blk)[kTiles]) {
    const uint32_t* pxy = a.sxy + (sb + kq);
    const float* pzl = a.szl + (sb + kq);
    const float* pw = a.w + ((int64_t)row * a.ldw + sb + kq);
    // every counter drained here, so that the loop's waits are for its own loads only
    __builtin_amdgcn_s_waitcnt(0);
    uint32_t sxy = pxy[0];
    float szl = pzl[0], wb = pw[0];
#pragma unroll
    for (int st = 0; st < kSourceBlock; st += 4) {
        const int nx = st + 4 < kSourceBlock ? st + 4 : st;
        const uint32_t sxy_n = pxy[nx];
        const float szl_n = pzl[nx], wb_n = pw[nx];
        float Z[kTiles], r2[kTiles], m[kTiles], G[kTiles];
#pragma unroll
        for (int j = 0; j < kTiles; ++j) {
            const float dz = tzl[j] - szl;
            Z[j] = dz * dz;
        }
        far_pairs4v(txy, sxy, Z, r2, m);
#pragma unroll
        for (int j = 0; j < kTiles; ++j)
            G[j] = YUK ? far_field_yukawa_lattice(r2[j], Z[j], m[j], a.yl) : far_field_q2_lattice(r2[j], Z[j], m[j]);
        // sigma = 0: the lattice form's common factor kFarScale32 rides on the weights
        const float ws = YUK ? wb : wb * kFarScale32;
#pragma unroll
        for (int j = 0; j < kTiles; ++j) blk[j] = MfmaAcc<float>::mma(G[j], ws, blk[j]);
        sxy = sxy_n;
        szl = szl_n;
        wb = wb_n;
    }
}

// Table-value blocks of the FP64 kernel: table blocks read the LDS table (GLOBAL = false);
// gather blocks and mixed blocks without a far field (sigma > 0: the global table holds every
// offset, the LDS prefix included) read the global table, which the L2 and the MALL hold.
// Loaded per step, a step would wait on its sources' coordinates and then on the table reads
// they address, with two wavefronts per SIMD to cover that latency (the LDS table allows one
// workgroup per compute unit).  Here the block's 64 sources are loaded once, one per lane,
// and each step takes its four by a lane permutation (an LDS-crossbar operation, outside the
// vector-memory counter); the weights and table reads of the next DEPTH steps are in flight
// while the current step is contracted.
template <typename Real, bool GLOBAL>
__device__ __forceinline__ void mfma_lookup_block(const SumArgs<Real>& a, const Lds<Real>& L,
                                                  const uint32_t (&ix)[kTiles], const uint32_t (&iy)[kTiles],
                                                  const uint32_t (&iz)[kTiles], int sb, int row, int kq,
                                                  typename MfmaAcc<Real>::V (&blk)[kTiles]) {
    constexpr int DEPTH = GLOBAL ? 2 : 1;
    constexpr int kSteps = kSourceBlock / 4;
    const int lane = threadIdx.x & 63;
    const int bx = (int)a.sx[sb + lane], by = (int)a.sy[sb + lane], bz = (int)a.sz[sb + lane];
    const Real* pw = a.w + ((int64_t)row * a.ldw + sb + kq);
    // the step's weight and its four kernel values (source 4 st + kq of the block)
    auto issue = [&](int st, Real& wv, Real (&g)[kTiles]) {
        const int from = (4 * st + kq) << 2;
        const uint32_t sx = (uint32_t)__builtin_amdgcn_ds_bpermute(from, bx);
        const uint32_t sy = (uint32_t)__builtin_amdgcn_ds_bpermute(from, by);
        const uint32_t sz = (uint32_t)__builtin_amdgcn_ds_bpermute(from, bz);
        // in phases (sorted triples, every index-array read, the sums), so that the eight LDS
        // reads are in flight together
        uint32_t lo[kTiles], mid[kTiles], hi[kTiles];
#pragma unroll
        for (int j = 0; j < kTiles; ++j) {
            const uint32_t da = absdiff_v(ix[j], sx), db = absdiff_v(iy[j], sy), dc = absdiff_v(iz[j], sz);
            lo[j] = min3u(da, db, dc);
            mid[j] = med3u(da, db, dc);
            hi[j] = max3u(da, db, dc);
        }
        __builtin_amdgcn_sched_barrier(0);
        uint32_t th[kTiles], tm[kTiles];
#pragma unroll
        for (int j = 0; j < kTiles; ++j) {
            th[j] = *(const uint32_t*)((const char*)L.tet + hi[j]);
            tm[j] = *(const uint32_t*)((const char*)L.tri + mid[j]);
        }
        __builtin_amdgcn_sched_barrier(0);
        wv = pw[4 * st];
#pragma unroll
        for (int j = 0; j < kTiles; ++j) {
            const uint32_t o = th[j] + tm[j] + (uint32_t)(sizeof(Real) / 4) * lo[j];
            g[j] = GLOBAL ? global_value(a.full_tab, o) : lds_value(L, o);
        }
    };
    Real wq[DEPTH + 1];
    Real G[DEPTH + 1][kTiles];
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) issue(d, wq[d], G[d]);
#pragma unroll
    for (int st = 0; st < kSteps; ++st) {
        if (st + DEPTH < kSteps) issue(st + DEPTH, wq[(st + DEPTH) % (DEPTH + 1)], G[(st + DEPTH) % (DEPTH + 1)]);
        // the later steps' reads are issued before this step's contraction waits on its own
        __builtin_amdgcn_sched_barrier(0);
        const int c = st % (DEPTH + 1);
#pragma unroll
        for (int j = 0; j < kTiles; ++j) blk[j] = MfmaAcc<Real>::mma(G[c][j], wq[c], blk[j]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <typename Real>
__device__ __forceinline__ void mfma_tile(const SumArgs<Real>& a, const Lds<Real>& L, int tile, int chunk) {
    using V = typename MfmaAcc<Real>::V;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15;            // A row (target within a tile) / B, D column (RHS)
    const int kq = lane >> 4;             // A column / B row (source within the step of 4)
    const int base = tile * kWave;
    uint32_t ix[kTiles], iy[kTiles], iz[kTiles], txy[kTiles];
    float tzl[kTiles];
    int lx = 1 << 30, ly = 1 << 30, lz = 1 << 30, hx = 0, hy = 0, hz = 0;
#pragma unroll
    for (int j = 0; j < kTiles; ++j) {
        const int tc = min(base + 16 * j + row, a.nt - 1);
        ix[j] = a.tx[tc];
        iy[j] = a.ty[tc];
        iz[j] = a.tz[tc];
        txy[j] = sizeof(Real) == 4 ? a.txy[tc] : 0u;
        tzl[j] = sizeof(Real) == 4 ? a.tzl[tc] : 0.f;
        lx = min(lx, (int)ix[j]);
        ly = min(ly, (int)iy[j]);
        lz = min(lz, (int)iz[j]);
        hx = max(hx, (int)ix[j]);
        hy = max(hy, (int)iy[j]);
        hz = max(hz, (int)iz[j]);
    }
    lx = wave_min(lx);
    ly = wave_min(ly);
    lz = wave_min(lz);
    hx = wave_max(hx);
    hy = wave_max(hy);
    hz = wave_max(hz);
    const uint32_t tab_q = (uint32_t)(kQuant * a.tab_r);

    V acc[kTiles], comp[kTiles];
#pragma unroll
    for (int j = 0; j < kTiles; ++j)
        for (int v = 0; v < 4; ++v) acc[j][v] = comp[j][v] = Real(0);

    const int b0 = chunk * a.blk_per_chunk;
    const int b1 = min(a.nblk, b0 + a.blk_per_chunk);
    // each tile of the item starts at another block of the chunk (as in sum_tile)
    const int nb = b1 - b0;
    const int rot = ((tile % kGroupTiles) * nb) / kGroupTiles;
    for (int jb = 0; jb < nb; ++jb) {
        int b = b0 + jb + rot;
        if (b >= b1) b -= nb;
        const int sb = b * kSourceBlock;
        const int32_t* bb = a.sbox + 6 * b;
        const int gap = max(max(max(bb[0] - hx, lx - bb[3]), max(bb[1] - hy, ly - bb[4])),
                            max(max(bb[2] - hz, lz - bb[5]), 0));
        const int span = max(max(max(bb[3] - lx, hx - bb[0]), max(bb[4] - ly, hy - bb[1])),
                             max(bb[5] - lz, hz - bb[2]));
        const int cls = block_class(gap, span, a.tab_r, a.far_ok != 0, sizeof(Real) == 4, a.far_gap);
        // FP32: the block's own sums, folded below; FP64: the running sums themselves (no
        // compensation to apply, and 32 registers left for table reads in flight)
        V blkz[kTiles];
        if constexpr (sizeof(Real) == 4) {
#pragma unroll
            for (int j = 0; j < kTiles; ++j)
                for (int v = 0; v < 4; ++v) blkz[j][v] = Real(0);
        }
        V (&blk)[kTiles] = *(sizeof(Real) == 8 ? &acc : &blkz);
        if constexpr (sizeof(Real) == 4) {
            if (cls == kClassFar2) {
                if (a.yukawa) mfma_far2_block<true>(a, txy, tzl, sb, row, kq, blk);
                else mfma_far2_block<false>(a, txy, tzl, sb, row, kq, blk);
            }
        }
        // FP64 table-value blocks have loops of their own (the FP32 kernel's registers, at four
        // wavefronts per SIMD, leave no room for them: its table, gather and mixed blocks take
        // the step loop below)
        bool done = false;
        if constexpr (sizeof(Real) == 8) {
            if (cls == kClassTable) {
                mfma_lookup_block<Real, false>(a, L, ix, iy, iz, sb, row, kq, blk);
                done = true;
            } else if (cls == kClassGather || (cls == kClassMixed && !a.far_ok)) {
                mfma_lookup_block<Real, true>(a, L, ix, iy, iz, sb, row, kq, blk);
                done = true;
            }
        } else {
            done = cls == kClassFar2;
        }
        if (!done) {
        // Table, gather and mixed blocks take the block's 64 integer source coordinates once,
        // one per lane, and each step its four by a lane permutation (outside the
        // vector-memory counter).
        const bool by_lane = !(sizeof(Real) == 8 && cls == kClassFar);
        int bxq = 0, byq = 0, bzq = 0;
        if (by_lane) {
            const int lane = threadIdx.x & 63;
            bxq = (int)a.sx[sb + lane];
            byq = (int)a.sy[sb + lane];
            bzq = (int)a.sz[sb + lane];
        }
        for (int st = 0; st < kSourceBlock; st += 4) {
            const int s = sb + st + kq;
            const Real wb = a.w[row * a.ldw + s];
            Real G[kTiles];
            if (sizeof(Real) == 8 && cls == kClassFar) {
                const Real sx = a.sxr[s], sy = a.syr[s], sz = a.szr[s];
                // the targets' coordinates converted here (registers kept for the loops above)
                if (a.yukawa) {
#pragma unroll
                    for (int j = 0; j < kTiles; ++j) {
                        const Real dx = (Real)ix[j] - sx, dy = (Real)iy[j] - sy, dz = (Real)iz[j] - sz;
                        G[j] = far_field_yukawa<Real>(dx * dx, dy * dy, dz * dz, a.kq, a.yk);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < kTiles; ++j) {
                        const Real dx = (Real)ix[j] - sx, dy = (Real)iy[j] - sy, dz = (Real)iz[j] - sz;
                        G[j] = far_field<Real>(dx * dx, dy * dy, dz * dz);
                    }
                }
            } else {
                const int from = (st + kq) << 2;
                const uint32_t sx = (uint32_t)__builtin_amdgcn_ds_bpermute(from, bxq);
                const uint32_t sy = (uint32_t)__builtin_amdgcn_ds_bpermute(from, byq);
                const uint32_t sz = (uint32_t)__builtin_amdgcn_ds_bpermute(from, bzq);
                if (cls == kClassTable) {
#pragma unroll
                    for (int j = 0; j < kTiles; ++j)
                        G[j] = lds_value(L, table_offset(L, absdiff_v(ix[j], sx), absdiff_v(iy[j], sy),
                                                         absdiff_v(iz[j], sz)));
                } else if (cls == kClassGather) {
#pragma unroll
                    for (int j = 0; j < kTiles; ++j)
                        G[j] = global_value(a.full_tab, table_offset(L, absdiff_v(ix[j], sx), absdiff_v(iy[j], sy),
                                                                      absdiff_v(iz[j], sz)));
                } else {
#pragma unroll
                    for (int j = 0; j < kTiles; ++j) {
                        const uint32_t da = absdiff_v(ix[j], sx), db = absdiff_v(iy[j], sy), dc = absdiff_v(iz[j], sz);
                        if (max3u(da, db, dc) <= tab_q) {
                            G[j] = lds_value(L, table_offset(L, da, db, dc));
                        } else if (a.far_ok) {
                            // |d| components of the integer offsets, exact in the kernel's precision
                            const Real dx = (Real)da, dy = (Real)db, dz = (Real)dc;
                            G[j] = a.yukawa ? far_field_yukawa<Real>(dx * dx, dy * dy, dz * dz, a.kq, a.yk)
                                            : far_field<Real>(dx * dx, dy * dy, dz * dz);
                        } else {
                            G[j] = global_value(a.full_tab, table_offset(L, da, db, dc));
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kTiles; ++j) blk[j] = MfmaAcc<Real>::mma(G[j], wb, blk[j]);
        }
        }
        // FP32: fold the block's sums into the running accumulators, compensated (Kahan):
        // 4 VALU instructions per accumulator element (Neumaier's branch-free form takes 8)
        if constexpr (sizeof(Real) == 4) {
#pragma unroll
            for (int j = 0; j < kTiles; ++j)
                for (int v = 0; v < 4; ++v) {
                    const Real y = blk[j][v] - comp[j][v];
                    const Real t = acc[j][v] + y;
                    comp[j][v] = (t - acc[j][v]) - y;
                    acc[j][v] = t;
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
                a.part[(int64_t)row * a.ldp + (int64_t)chunk * a.nt + t] = (double)acc[j][v] - (double)comp[j][v];
        }
}

template <typename Real, int THREADS, bool FAR>
__global__ __launch_bounds__(THREADS) void lgf_sum_mfma_kernel(const SumArgs<Real> a, const Sched q) {
    __shared__ __align__(16) char lds[lds_bytes<Real, FAR>()];
    const Lds<Real> L = lds_layout<Real, FAR>(lds);
    __shared__ ItemRing ring;
    ring_init(&ring);
    fill_lds(L, a.near_tab, a.tab_r, FAR ? a.tab_r : a.full_r);
    __syncthreads();
    for_each_item(q, &ring, [&](uint32_t tile, uint32_t chunk) { mfma_tile<Real>(a, L, (int)tile, (int)chunk); });
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

// Workgroup sizes: 16 wavefronts, except the FP64 4-RHS and matrix-core kernels, whose
// accumulators need the registers of 8.
template <typename Real>
constexpr int mfma_threads() { return sizeof(Real) == 4 ? kSumThreads : kSumThreads / 2; }
template <typename Real>
constexpr int rhs4_threads() { return sizeof(Real) == 4 ? kSumThreads : kSumThreads / 2; }

template <typename Real>
void launch_all(const PointSet& T, const PointSet& S, const Real* w, int nrhs, const Real* near, const Real* full,
                int tab_r, const SumTables& tabs, const SumPlan& plan, double* part, int grid, const int32_t* skip,
                hipStream_t st) {
    const bool fp32 = sizeof(Real) == 4;
    const bool far = fp32 ? tabs.far32() : tabs.far64();
    const bool lds_far = tabs.far_field;   // the sigma = 0 LDS layout (short index arrays)
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
    a.txy = T.xy16;
    a.tzl = T.zl;
    a.sxy = S.xy16;
    a.szl = S.zl;
    a.sbox = S.bbox;
    a.ns = (int)S.count;
    a.nblk = (int)S.nblk;
    a.blk_per_chunk = plan.blk_per_chunk;
    a.ldw = S.padded;
    a.near_tab = near;
    a.full_tab = full;
    a.tab_r = tab_r;
    a.full_r = tabs.full_r;
    a.far_ok = far ? 1 : 0;
    a.far_gap = fp32 ? tabs.far_gap32() : tabs.far_gap64();
    a.yukawa = fp32 && tabs.yukawa32 ? 1 : 0;
    a.kq = (Real)(tabs.kappa / kQuant);
    a.yk = (Real)(-tabs.kappa * 1.4426950408889634 / kQuant);
    a.yl = yukawa_lattice(tabs.kappa);
    a.ldp = (int64_t)plan.chunks * T.count;
    int r = 0;
    while (r < nrhs) {
        const int left = nrhs - r;
        SumArgs<Real> ar = a;
        ar.w = w + (int64_t)r * a.ldw;
        ar.part = part + (int64_t)r * a.ldp;
        const int threads = left >= 16 ? mfma_threads<Real>() : left >= 4 ? rhs4_threads<Real>() : kSumThreads;
        const Sched q{skip, plan.items, (uint32_t)plan.nitems, (uint32_t)((T.count + kWave - 1) / kWave), plan.counter,
                      plan.err, plan.wait_polls};
        if (left >= 16) {
            if (lds_far) lgf_sum_mfma_kernel<Real, mfma_threads<Real>(), true><<<grid, mfma_threads<Real>(), 0, st>>>(ar, q);
            else lgf_sum_mfma_kernel<Real, mfma_threads<Real>(), false><<<grid, mfma_threads<Real>(), 0, st>>>(ar, q);
            r += 16;
        } else if (left >= 4) {
            if (lds_far) lgf_sum_kernel<Real, 4, rhs4_threads<Real>(), true><<<grid, rhs4_threads<Real>(), 0, st>>>(ar, q);
            else lgf_sum_kernel<Real, 4, rhs4_threads<Real>(), false><<<grid, rhs4_threads<Real>(), 0, st>>>(ar, q);
            r += 4;
        } else {
            if (lds_far) lgf_sum_kernel<Real, 1, kSumThreads, true><<<grid, kSumThreads, 0, st>>>(ar, q);
            else lgf_sum_kernel<Real, 1, kSumThreads, false><<<grid, kSumThreads, 0, st>>>(ar, q);
            r += 1;
        }
        BAE_HIP_CHECK(hipGetLastError());
    }
}

// Estimated VALU cost per pair of each block class (FP32 instruction counts; the gather
// and mixed classes are charged for their memory and divergence).
constexpr double kClassCost[5] = {8.0, 26.0, 15.0, 40.0, 45.0};

}  // namespace

int lgf_sum_chunks(int64_t nt, int64_t nblk) {
    const int64_t groups = (nt + kWave * kGroupTiles - 1) / (kWave * kGroupTiles);
    // about 32 items per workgroup of a full MI355X (256 CUs): fine enough that the
    // workgroups finish together (with 8, the 257^3 sums lose 10% to the last items)
    // (a small sum, of fewer items than workgroups, gets one source block per item, so
    // that its few wavefronts each walk as short a chain of steps as possible)
    int64_t chunks = (32 * 256 + groups - 1) / groups;
    chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, nblk));
    return (int)std::max<int64_t>(1, std::min<int64_t>(chunks, kMaxChunks));
}

int lgf_sum_grid(int device) {
    static std::mutex mu;
    static std::map<int, int> cus;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cus.find(device);
    if (it != cus.end()) return it->second;
    int n = 0;
    BAE_HIP_CHECK(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device));
    n = std::max(1, n);
    cus[device] = n;
    return n;
}

void plan_sum(const PointSet& T, const PointSet& S, const SumTables& tabs, SumPlan& plan,
              std::vector<uint32_t>& host_items) {
    const int64_t nt = T.count, tiles = (nt + kWave - 1) / kWave, nblk = S.nblk;
    int chunks = lgf_sum_chunks(nt, nblk);
    const int bpc = (int)((nblk + chunks - 1) / std::max(1, chunks));
    chunks = (int)((nblk + bpc - 1) / std::max(1, bpc));
    plan.chunks = std::max(1, chunks);
    plan.blk_per_chunk = std::max(1, bpc);
    const int64_t groups = (tiles + kGroupTiles - 1) / kGroupTiles;
    plan.nitems = groups * plan.chunks;
    if (groups > (1 << 20) || plan.chunks > 4095) throw Error{BAE_ERR_ARG, "LGF sum too large for the work list"};
    for (auto& r : plan.class_pairs)
        for (auto& v : r) v = 0;
    host_items.resize(plan.nitems);
    std::vector<double> cost(plan.nitems, 0.0);
    const bool classify = tiles * nblk <= (int64_t)60000000;
    if (classify) {
        for (int64_t tl = 0; tl < tiles; ++tl) {
            int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {0, 0, 0};
            for (int64_t i = tl * kWave; i < (tl + 1) * kWave; ++i) {
                const int64_t t = std::min(i, nt - 1);
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], T.hq[3 * t + a]);
                    hi[a] = std::max(hi[a], T.hq[3 * t + a]);
                }
            }
            const int64_t tcount = std::min<int64_t>(kWave, nt - tl * kWave);
            for (int64_t b = 0; b < nblk; ++b) {
                const int32_t* bb = &S.hbox[6 * b];
                int gap = 0, span = 0;
                for (int a = 0; a < 3; ++a) {
                    gap = std::max(gap, std::max(bb[a] - hi[a], lo[a] - bb[3 + a]));
                    span = std::max(span, std::max(bb[3 + a] - lo[a], hi[a] - bb[a]));
                }
                const int64_t pairs = tcount * std::min<int64_t>(kSourceBlock, S.count - b * kSourceBlock);
                const int c32 = block_class(gap, span, tabs.tab_r32, tabs.far32(), true, tabs.far_gap32());
                const int c64 = block_class(gap, span, tabs.tab_r64, tabs.far64(), false, tabs.far_gap64());
                plan.class_pairs[1][c32] += pairs;
                plan.class_pairs[0][c64] += pairs;
                cost[(tl / kGroupTiles) * plan.chunks + b / plan.blk_per_chunk] += kClassCost[c32] * (double)pairs;
            }
        }
    }
    // items (group, chunk) ordered by decreasing cost (stable: natural order when unclassified)
    std::vector<int64_t> order(plan.nitems);
    for (int64_t i = 0; i < plan.nitems; ++i) order[i] = i;
    if (classify) std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
    for (int64_t i = 0; i < plan.nitems; ++i) {
        const int64_t g = order[i] / plan.chunks, ch = order[i] % plan.chunks;
        host_items[i] = (uint32_t)g | ((uint32_t)ch << 20);
    }
}

int lgf_sum_launch(const PointSet& T, const PointSet& S, const void* w, int nrhs, int prec, const SumTables& tabs,
                   const SumPlan& plan, double* part, int64_t part_capacity, int grid, hipStream_t st,
                   const int32_t* skip) {
    if (T.count == 0) return 0;
    const int chunks = plan.chunks;
    if ((int64_t)chunks * T.count * nrhs > part_capacity) throw Error{BAE_ERR_ARG, "partial-sum buffer too small"};
    if (tabs.full_r > kMaxR) throw Error{BAE_ERR_ARG, "table radius beyond the index arrays"};
    if (S.count == 0) {
        launch_fill(part, (int64_t)chunks * T.count * nrhs, 0.0, st);
        return chunks;
    }
    if (prec == BAE_PREC_FP64)
        launch_all<double>(T, S, (const double*)w, nrhs, tabs.near64, tabs.full64, tabs.tab_r64, tabs, plan, part,
                           grid, skip, st);
    else
        launch_all<float>(T, S, (const float*)w, nrhs, tabs.near32, tabs.full32, tabs.tab_r32, tabs, plan, part,
                          grid, skip, st);
    return chunks;
}

void lgf_eval_launch(const int32_t* off, int64_t count, double* out, int prec, const SumTables& tabs, hipStream_t st) {
    if (count == 0) return;
    const unsigned blocks = (unsigned)((count + 255) / 256);
    const double kq = tabs.kappa / kQuant, yk = -tabs.kappa * 1.4426950408889634 / kQuant;
    if (prec == BAE_PREC_FP64)
        lgf_eval_kernel<double><<<blocks, 256, 0, st>>>(off, count, tabs.full64, tabs.tab_r64, tabs.full_r,
                                                        tabs.far64() ? 1 : 0, 0, kq, yk, YukawaLattice{}, out);
    else
        lgf_eval_kernel<float><<<blocks, 256, 0, st>>>(off, count, tabs.full32, tabs.tab_r32, tabs.full_r,
                                                       tabs.far32() ? 1 : 0, tabs.yukawa32 ? 1 : 0, (float)kq,
                                                       (float)yk, yukawa_lattice(tabs.kappa), out);
    BAE_HIP_CHECK(hipGetLastError());
}

double yukawa_check(const double* table, int R, int from_r, double kappa, hipStream_t st) {
    if (R <= from_r) return 0.0;
    const int64_t e0 = table_size(from_r), e1 = table_size(R);
    const int blocks = (int)std::min<int64_t>(1024, (e1 - e0 + 255) / 256);
    double* dmax = nullptr;
    BAE_HIP_CHECK(hipMalloc(&dmax, sizeof(double) * blocks));
    yukawa_check_kernel<<<blocks, 256, 0, st>>>(table, e0, e1, kappa / kQuant, -kappa * 1.4426950408889634 / kQuant,
                                                dmax);
    std::vector<double> h(blocks);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), dmax, sizeof(double) * blocks, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dmax);
    if (e != hipSuccess) throw Error{BAE_ERR_HIP, std::string("far-field check: ") + hipGetErrorString(e)};
    double worst = 0.0;
    for (double v : h) worst = std::max(worst, v);
    return worst;
}

}  // namespace bae
