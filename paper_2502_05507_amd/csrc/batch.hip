// Batched solves: many small BAE problems advanced in lock-step.
//
// Every GMRES phase (double-layer weights, LGF sum, closure, the two classical
// Gram-Schmidt passes, the norm, Givens) is ONE launch for all problems of the batch,
// over flat index spaces (per-problem offsets, binary search for the owning problem) or
// over precomputed work lists.  The LGF sum is a persistent kernel: a fixed grid walks a
// list of (problem, 256-target tile, source chunk) items, keeping the problem's LDS table
// while consecutive items share it.  The iteration counter lives in device memory, so one
// GMRES iteration -- or several -- is captured once as a HIP graph and replayed; problems
// that have converged skip their work items.  The tiling (source blocks per chunk,
// persistent grid size) is chosen by a small autotuner that times candidates on the batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <functional>
#include <sstream>

#include "context.hpp"
#include "lgf_device.hpp"

namespace bae {
using namespace lgfdev;

int guard(const std::function<void()>& fn);

namespace {

constexpr int kT = 256;       // threads per block (all batched kernels)
constexpr int kSlice = 2048;  // elements per dot-product slice

// Device descriptor of one problem of the batch.
struct BProb {
    SumArgs<double> s64;   // LGF sum arguments (targets, sources, tables, w, part) for FP64
    SumArgs<float> s32;    // ... for FP32 (same buffers, other precision)
    const int32_t *rowptr, *col;
    const double* coef;
    const int32_t *tq, *tp, *tpos;
    const double* tw;
    int n, nt, ns_pad, chunks, nslices, m;
    double *V, *H, *cs, *sn, *g, *hist, *beta, *hA, *hB, *nrm, *dpart, *y;
    int32_t *done, *kdone;
    double *b, *x, *r, *tmp, *ug, *upg;
    void* w;
    double* part;
};

struct Item {             // LGF-sum work item
    int p, tile, chunk, pad;
};

template <typename Real>
__device__ __forceinline__ const SumArgs<Real>& sum_args(const BProb& q);
template <>
__device__ __forceinline__ const SumArgs<double>& sum_args<double>(const BProb& q) { return q.s64; }
template <>
__device__ __forceinline__ const SumArgs<float>& sum_args<float>(const BProb& q) { return q.s32; }

__device__ inline int owner(const int64_t* off, int np, int64_t g) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- operator pieces
// src: 0 -> V[k], 1 -> x
template <typename Real>
__global__ void b_weights(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total,
                          int src, const int* __restrict__ kdev, int use_done) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    if (use_done && q.done[0]) return;
    if (src == 0 && kdev[0] >= q.m) return;           // never index past the basis
    const int64_t s = gi - off[p];
    if (s >= q.ns_pad) return;
    const double* v = src == 0 ? q.V + (int64_t)kdev[0] * q.n : q.x;
    double acc = 0.0;
    if (s < q.s64.ns)
        for (int j = q.rowptr[s]; j < q.rowptr[s + 1]; ++j) acc = fma(q.coef[j], v[q.col[j]], acc);
    ((Real*)q.w)[s] = (Real)acc;
}

template <typename Real>
__global__ __launch_bounds__(kT) void b_lgf_sum(const BProb* __restrict__ P, const Item* __restrict__ items,
                                                int nitems, int use_done) {
    __shared__ Real tab[kNearE];
    int cur = -1;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Item w = items[it];
        const BProb& q = P[w.p];
        if (use_done && q.done[0]) continue;            // uniform over the block
        const SumArgs<Real>& a = sum_args<Real>(q);
        if (w.p != cur) {
            __syncthreads();
            for (int i = threadIdx.x; i < kNearE; i += kT) tab[i] = a.near_tab[i];
            __syncthreads();
            cur = w.p;
        }
        sum_tile<Real, 1>(a, tab, w.tile, w.chunk);
    }
}

// dst: 0 -> V[k+1], 1 -> tmp
__global__ void b_closure(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total, int dst,
                          const int* __restrict__ kdev, int use_done) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    if (use_done && q.done[0]) return;
    if (dst == 0 && kdev[0] >= q.m) return;
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    const int64_t a = q.tq[i], b = q.tp[i];
    double va = 0.0, vb = 0.0;
    for (int c = 0; c < q.chunks; ++c) {
        va += q.part[(int64_t)c * q.nt + a];
        vb += q.part[(int64_t)c * q.nt + b];
    }
    const double t = q.tw[i];
    double* out = dst == 0 ? q.V + (int64_t)(kdev[0] + 1) * q.n : q.tmp;
    out[i] = (1.0 - t) * va + t * vb;
}

// u_gamma = sum of the partials (scattered to [gamma+; gamma-] order) + u_p on gamma
__global__ void b_gamma_values(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    const int64_t t = gi - off[p];
    if (t >= q.nt) return;
    double acc = 0.0;
    for (int c = 0; c < q.chunks; ++c) acc += q.part[(int64_t)c * q.nt + t];
    const int pos = q.tpos[t];
    q.ug[pos] = acc + q.upg[pos];
}

// ---------------------------------------------------------------- Krylov pieces
__device__ inline double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kT / 64; ++k) s += sh[k];
    return s;
}

// mode 0: dpart[j][slice] = V[j] . V[k+1], j <= k;  mode 1: dpart[0] = V[k+1] . V[k+1];
// mode 2: dpart[0] = vec . vec with vec = b (sel 0) or r (sel 1)
__global__ __launch_bounds__(kT) void b_dots(const BProb* __restrict__ P, const int2* __restrict__ slices, int nitems,
                                             int mode, int sel, const int* __restrict__ kdev, int use_done) {
    __shared__ double sh[kT / 64];
    const int2 w = slices[blockIdx.x];
    const BProb& q = P[w.x];
    if (use_done && q.done[0]) return;
    const int k = kdev[0];
    if (mode != 2 && k >= q.m) return;
    const int64_t lo = (int64_t)w.y * kSlice, hi = min((int64_t)q.n, lo + kSlice);
    if (mode == 0) {
        const double* y = q.V + (int64_t)(k + 1) * q.n;
        for (int j = 0; j <= k; ++j) {
            const double* x = q.V + (int64_t)j * q.n;
            double acc = 0.0;
            for (int64_t i = lo + threadIdx.x; i < hi; i += kT) acc = fma(x[i], y[i], acc);
            const double s = block_sum(acc, sh);
            if (threadIdx.x == 0) q.dpart[(int64_t)j * q.nslices + w.y] = s;
        }
    } else {
        const double* y = mode == 1 ? q.V + (int64_t)(k + 1) * q.n : (sel == 0 ? q.b : q.r);
        double acc = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += kT) acc = fma(y[i], y[i], acc);
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) q.dpart[w.y] = s;
    }
}

// h[j] = sum over slices; dest 0 -> hA, 1 -> hB, 2 -> nrm (one value)
__global__ void b_dots_finalize(const BProb* __restrict__ P, int np, int dest, int nj_mode,
                                const int* __restrict__ kdev, int use_done) {
    const int p = blockIdx.x;
    const BProb& q = P[p];
    if (use_done && q.done[0]) return;
    if (nj_mode == 0 && kdev[0] >= q.m) return;
    const int nj = nj_mode == 0 ? kdev[0] + 1 : 1;
    double* h = dest == 0 ? q.hA : dest == 1 ? q.hB : q.nrm;
    for (int j = threadIdx.x; j < nj; j += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < q.nslices; ++b) s += q.dpart[(int64_t)j * q.nslices + b];
        h[j] = s;
    }
}

__global__ void b_subtract(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total,
                           int which, const int* __restrict__ kdev) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    const int k = kdev[0];
    if (q.done[0] || k >= q.m) return;
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    const double* h = which == 0 ? q.hA : q.hB;
    double acc = 0.0;
    for (int j = 0; j <= k; ++j) acc = fma(h[j], q.V[(int64_t)j * q.n + i], acc);
    q.V[(int64_t)(k + 1) * q.n + i] -= acc;
}

__global__ void b_normalize(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total,
                            const int* __restrict__ kdev) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    if (q.done[0] || kdev[0] >= q.m) return;
    const double nr = sqrt(q.nrm[0]);
    if (gi - off[p] >= q.n) return;
    if (nr > 0.0) q.V[(int64_t)(kdev[0] + 1) * q.n + gi - off[p]] /= nr;
}

// one thread per problem; tol from device memory; the iteration counter advances in
// b_advance after every problem has used it
__global__ void b_givens(const BProb* __restrict__ P, int np, const int* __restrict__ kdev,
                         const double* __restrict__ tol) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const BProb& q = P[p];
    const int k = kdev[0];
    if (q.done[0] || k >= q.m) {
        q.done[0] = 1;
        return;
    }
    double* h = q.H + (int64_t)k * (q.m + 1);
    for (int i = 0; i <= k; ++i) h[i] = q.hA[i] + q.hB[i];
    const double hk1 = sqrt(q.nrm[0]);
    for (int i = 0; i < k; ++i) {
        const double a = h[i], b = h[i + 1];
        h[i] = q.cs[i] * a + q.sn[i] * b;
        h[i + 1] = -q.sn[i] * a + q.cs[i] * b;
    }
    const double a = h[k], b = hk1;
    const double rr = hypot(a, b);
    if (rr == 0.0) {
        q.done[0] = 1;
        q.kdone[0] = k;
        return;
    }
    q.cs[k] = a / rr;
    q.sn[k] = b / rr;
    h[k] = rr;
    h[k + 1] = 0.0;
    q.g[k + 1] = -q.sn[k] * q.g[k];
    q.g[k] = q.cs[k] * q.g[k];
    const double est = fabs(q.g[k + 1]) / q.beta[0];
    q.hist[k] = est;
    q.kdone[0] = k + 1;
    if (est <= tol[0] || hk1 == 0.0 || k + 1 >= q.m || k + 1 >= (int)tol[1]) q.done[0] = 1;
}

// gather per-problem scalars for one host copy: what 0 -> done, 1 -> kdone, 2 -> nrm
__global__ void b_gather(const BProb* __restrict__ P, int np, int what, int32_t* __restrict__ iout,
                         double* __restrict__ dout) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    if (what == 0) iout[p] = P[p].done[0];
    else if (what == 1) iout[p] = P[p].kdone[0];
    else dout[p] = P[p].nrm[0];
}

__global__ void b_advance(int* kdev) {
    if (threadIdx.x == 0 && blockIdx.x == 0) kdev[0] += 1;
}

__global__ void b_set_int(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

__global__ void b_set_double2(double* p, double v0, double v1) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        p[0] = v0;
        p[1] = v1;
    }
}

// sel 0: r0 = b, sel 1: r0 = r.  skip[p] marks problems left alone (refinement).
__global__ void b_init(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total, int sel,
                       const int32_t* __restrict__ skip) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    const double bnorm = sqrt(q.nrm[0]);
    const double* r0 = sel == 0 ? q.b : q.r;
    if (i == 0) {
        q.beta[0] = bnorm;
        q.g[0] = bnorm;
        q.done[0] = (bnorm == 0.0 || (skip && skip[p])) ? 1 : 0;
        q.kdone[0] = 0;
    }
    q.V[i] = bnorm > 0.0 ? r0[i] / bnorm : 0.0;
}

// thread per problem: y = R^-1 g over the first kdone[p] columns
__global__ void b_backsolve(const BProb* __restrict__ P, int np) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const BProb& q = P[p];
    const int kk = q.kdone[0];
    for (int i = kk - 1; i >= 0; --i) {
        double acc = q.g[i];
        for (int j = i + 1; j < kk; ++j) acc -= q.H[(int64_t)j * (q.m + 1) + i] * q.y[j];
        const double d = q.H[(int64_t)i * (q.m + 1) + i];
        q.y[i] = d != 0.0 ? acc / d : 0.0;
    }
}

// x (+)= V y ; then (optionally) nothing else
__global__ void b_update_x(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total,
                           int accumulate) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    const int kk = q.kdone[0];
    double acc = 0.0;
    for (int j = 0; j < kk; ++j) acc = fma(q.y[j], q.V[(int64_t)j * q.n + i], acc);
    q.x[i] = accumulate ? q.x[i] + acc : acc;
}

// r = b - tmp ; x = 0 (mode 1) ; r = b (mode 2)
__global__ void b_vec(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total, int mode) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    if (mode == 0) q.r[i] = q.b[i] - q.tmp[i];
    else if (mode == 1) q.x[i] = 0.0;
    else q.r[i] = q.b[i];
}

inline unsigned nblocks(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kT - 1) / kT); }

}  // namespace
}  // namespace bae

using namespace bae;

struct bae_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<bae_ctx*> ctx;
    int np = 0;
    DevMem probs, off_src, off_row, off_tgt, slices, items, kdev, tol, skip, arena;
    int64_t tot_src = 0, tot_row = 0, tot_tgt = 0;
    int nslices_total = 0, nitems = 0;
    int blk_per_chunk = 8, grid_mult = 4, n_cu = 256;
    std::vector<BProb> hp;
    DevMem gi, gd;             // gathered per-problem ints / doubles
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int graph_iters = 8;
    int32_t* pinned = nullptr;
};

namespace bae {
namespace {

void release_graphs(bae_batch* b) {
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
        b->exec[i] = nullptr;
        b->graph[i] = nullptr;
    }
}

// (Re)build per-problem chunking, the partial-sum arena and the work lists.
void build_layout(bae_batch* b) {
    release_graphs(b);
    hipStream_t st = b->stream;
    BAE_HIP_CHECK(hipStreamSynchronize(st));   // nothing in flight uses the old layout
    b->tot_src = b->tot_row = b->tot_tgt = 0;
    std::vector<int64_t> osrc(b->np), orow(b->np), otgt(b->np);
    std::vector<int2> sl;
    std::vector<Item> it;
    int64_t arena = 0;
    std::vector<int64_t> part_at(b->np), dpart_at(b->np);
    for (int p = 0; p < b->np; ++p) {
        bae_ctx* c = b->ctx[p];
        BProb& q = b->hp[p];
        osrc[p] = b->tot_src;
        orow[p] = b->tot_row;
        otgt[p] = b->tot_tgt;
        b->tot_src += c->S.ps.padded;
        b->tot_row += c->ngm;
        b->tot_tgt += c->nT;
        q.chunks = (int)((c->S.ps.nblk + b->blk_per_chunk - 1) / b->blk_per_chunk);
        q.nslices = (int)((c->ngm + kSlice - 1) / kSlice);
        for (int s = 0; s < q.nslices; ++s) sl.push_back(make_int2(p, s));
        const int tiles = (int)((c->nT + kT - 1) / kT);
        for (int t = 0; t < tiles; ++t)
            for (int ch = 0; ch < q.chunks; ++ch) it.push_back(Item{p, t, ch, 0});
        part_at[p] = arena;
        arena += (int64_t)q.chunks * c->nT;
        dpart_at[p] = arena;
        arena += (int64_t)(c->K.m + 1) * q.nslices;
    }
    // largest problems' items first keeps the persistent grid busy to the end
    std::stable_sort(it.begin(), it.end(), [&](const Item& x, const Item& y) {
        return b->ctx[x.p]->nT * b->ctx[x.p]->nS > b->ctx[y.p]->nT * b->ctx[y.p]->nS;
    });
    b->arena.alloc(sizeof(double) * arena);
    for (int p = 0; p < b->np; ++p) {
        bae_ctx* c = b->ctx[p];
        BProb& q = b->hp[p];
        q.part = b->arena.as<double>() + part_at[p];
        q.dpart = b->arena.as<double>() + dpart_at[p];
        for (int prec = 0; prec < 2; ++prec) {
            auto fill = [&](auto& a, const auto* near, const auto* full, const auto* sxr, const auto* syr,
                            const auto* szr) {
                a.tx = c->T.ps.x;
                a.ty = c->T.ps.y;
                a.tz = c->T.ps.z;
                a.nt = (int)c->nT;
                a.sx = c->S.ps.x;
                a.sy = c->S.ps.y;
                a.sz = c->S.ps.z;
                a.sxr = sxr;
                a.syr = syr;
                a.szr = szr;
                a.sbox = c->S.ps.bbox;
                a.ns = (int)c->nS;
                a.nblk = (int)c->S.ps.nblk;
                a.blk_per_chunk = b->blk_per_chunk;
                a.ldw = c->S.ps.padded;
                a.near_tab = near;
                a.full_tab = full;
                a.far_ok = c->tabs.far_field ? 1 : 0;
                a.part = q.part;
                a.ldp = (int64_t)q.chunks * c->nT;
            };
            if (prec == 0) {
                fill(q.s64, c->tabs.near64, c->tabs.full64, c->S.ps.xd, c->S.ps.yd, c->S.ps.zd);
                q.s64.w = (const double*)c->w.p;
            } else {
                fill(q.s32, c->tabs.near32, c->tabs.full32, c->S.ps.xf, c->S.ps.yf, c->S.ps.zf);
                q.s32.w = (const float*)c->w.p;
            }
        }
    }
    b->nslices_total = (int)sl.size();
    b->nitems = (int)it.size();
    upload(b->off_src, osrc, st);
    upload(b->off_row, orow, st);
    upload(b->off_tgt, otgt, st);
    upload(b->slices, sl, st);
    upload(b->items, it, st);
    upload(b->probs, b->hp, st);
    BAE_HIP_CHECK(hipStreamSynchronize(st));
}

// one operator application for all problems: out = A q (closure) at precision prec
void apply_all(bae_batch* b, int prec, int src, int dst, int use_done) {
    hipStream_t st = b->stream;
    const BProb* P = b->probs.as<BProb>();
    const int* k = b->kdev.as<int>();
    const unsigned grid = (unsigned)std::min(b->nitems, b->grid_mult * b->n_cu);
    if (prec == BAE_PREC_FP64) {
        b_weights<double><<<nblocks(b->tot_src), kT, 0, st>>>(P, b->off_src.as<int64_t>(), b->np, b->tot_src, src, k,
                                                              use_done);
        b_lgf_sum<double><<<grid, kT, 0, st>>>(P, b->items.as<Item>(), b->nitems, use_done);
    } else {
        b_weights<float><<<nblocks(b->tot_src), kT, 0, st>>>(P, b->off_src.as<int64_t>(), b->np, b->tot_src, src, k,
                                                             use_done);
        b_lgf_sum<float><<<grid, kT, 0, st>>>(P, b->items.as<Item>(), b->nitems, use_done);
    }
    if (dst >= 0)
        b_closure<<<nblocks(b->tot_row), kT, 0, st>>>(P, b->off_row.as<int64_t>(), b->np, b->tot_row, dst, k, use_done);
    BAE_HIP_CHECK(hipGetLastError());
}

void norms(bae_batch* b, int sel) {
    hipStream_t st = b->stream;
    const BProb* P = b->probs.as<BProb>();
    b_dots<<<b->nslices_total, kT, 0, st>>>(P, b->slices.as<int2>(), b->nslices_total, 2, sel, b->kdev.as<int>(), 0);
    b_dots_finalize<<<b->np, 64, 0, st>>>(P, b->np, 2, 1, b->kdev.as<int>(), 0);
    BAE_HIP_CHECK(hipGetLastError());
}

void gmres_iteration(bae_batch* b, int prec) {
    hipStream_t st = b->stream;
    const BProb* P = b->probs.as<BProb>();
    const int* k = b->kdev.as<int>();
    apply_all(b, prec, 0, 0, 1);
    const int64_t* orow = b->off_row.as<int64_t>();
    for (int pass = 0; pass < 2; ++pass) {
        b_dots<<<b->nslices_total, kT, 0, st>>>(P, b->slices.as<int2>(), b->nslices_total, 0, 0, k, 1);
        b_dots_finalize<<<b->np, 64, 0, st>>>(P, b->np, pass, 0, k, 1);
        b_subtract<<<nblocks(b->tot_row), kT, 0, st>>>(P, orow, b->np, b->tot_row, pass, k);
    }
    b_dots<<<b->nslices_total, kT, 0, st>>>(P, b->slices.as<int2>(), b->nslices_total, 1, 0, k, 1);
    b_dots_finalize<<<b->np, 64, 0, st>>>(P, b->np, 2, 1, k, 1);
    b_normalize<<<nblocks(b->tot_row), kT, 0, st>>>(P, orow, b->np, b->tot_row, k);
    b_givens<<<(b->np + 63) / 64, 64, 0, st>>>(P, b->np, k, b->tol.as<double>());
    b_advance<<<1, 64, 0, st>>>(b->kdev.as<int>());
    BAE_HIP_CHECK(hipGetLastError());
}

// Lock-step GMRES on all problems (x0 = 0), then x (+)= V y.  Returns iterations run.
int gmres_all(bae_batch* b, int prec, int sel, double tol, int maxit, const std::vector<int32_t>& skip,
              bool accumulate, bool use_graph) {
    hipStream_t st = b->stream;
    const BProb* P = b->probs.as<BProb>();
    b_set_int<<<1, 64, 0, st>>>(b->kdev.as<int>(), 0);
    b_set_double2<<<1, 64, 0, st>>>(b->tol.as<double>(), tol, (double)maxit);
    BAE_HIP_CHECK(hipMemcpyAsync(b->skip.p, skip.data(), sizeof(int32_t) * b->np, hipMemcpyHostToDevice, st));
    norms(b, sel);
    b_init<<<nblocks(b->tot_row), kT, 0, st>>>(P, b->off_row.as<int64_t>(), b->np, b->tot_row, sel,
                                               b->skip.as<int32_t>());
    BAE_HIP_CHECK(hipGetLastError());
    const int gi = prec == BAE_PREC_FP64 ? 0 : 1;
    if (use_graph && !b->exec[gi]) {
        BAE_HIP_CHECK(hipStreamSynchronize(st));
        BAE_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < b->graph_iters; ++i) gmres_iteration(b, prec);
        BAE_HIP_CHECK(hipStreamEndCapture(st, &b->graph[gi]));
        BAE_HIP_CHECK(hipGraphInstantiate(&b->exec[gi], b->graph[gi], nullptr, nullptr, 0));
    }
    int k = 0;
    const int step = use_graph ? b->graph_iters : 4;
    while (k < maxit) {
        if (use_graph) BAE_HIP_CHECK(hipGraphLaunch(b->exec[gi], st));
        else
            for (int i = 0; i < step; ++i) gmres_iteration(b, prec);
        k += step;
        b_gather<<<(b->np + 63) / 64, 64, 0, st>>>(P, b->np, 0, b->gi.as<int32_t>(), nullptr);
        BAE_HIP_CHECK(hipMemcpyAsync(b->pinned, b->gi.p, sizeof(int32_t) * b->np, hipMemcpyDeviceToHost, st));
        BAE_HIP_CHECK(hipStreamSynchronize(st));
        bool all = true;
        for (int p = 0; p < b->np; ++p) all &= b->pinned[p] != 0;
        if (all) break;
    }
    b_backsolve<<<(b->np + 63) / 64, 64, 0, st>>>(P, b->np);
    b_update_x<<<nblocks(b->tot_row), kT, 0, st>>>(P, b->off_row.as<int64_t>(), b->np, b->tot_row, accumulate ? 1 : 0);
    BAE_HIP_CHECK(hipGetLastError());
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    return std::min(k, maxit);
}

std::vector<double> residuals(bae_batch* b, const std::vector<double>& bn) {
    hipStream_t st = b->stream;
    const BProb* P = b->probs.as<BProb>();
    apply_all(b, BAE_PREC_FP64, 1, 1, 0);
    b_vec<<<nblocks(b->tot_row), kT, 0, st>>>(P, b->off_row.as<int64_t>(), b->np, b->tot_row, 0);
    norms(b, 1);
    std::vector<double> out(b->np);
    b_gather<<<(b->np + 63) / 64, 64, 0, st>>>(P, b->np, 2, nullptr, b->gd.as<double>());
    BAE_HIP_CHECK(hipMemcpyAsync(out.data(), b->gd.p, sizeof(double) * b->np, hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    for (int p = 0; p < b->np; ++p) out[p] = bn[p] > 0 ? std::sqrt(out[p]) / bn[p] : 0.0;
    return out;
}

std::string tune_cache_path() {
    if (const char* e = std::getenv("BAE_AUTOTUNE_CACHE")) return e;
    if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/bae_autotune.txt";
    return "";
}

}  // namespace
}  // namespace bae

extern "C" {

int bae_batch_create(bae_ctx* const* ctxs, int32_t n, bae_batch** out) {
    return guard([&] {
        if (!ctxs || !out || n < 1) throw Error{BAE_ERR_ARG, "bae_batch_create: bad argument"};
        *out = nullptr;
        auto b = std::make_unique<bae_batch>();
        b->np = n;
        for (int i = 0; i < n; ++i) {
            bae_ctx* c = ctxs[i];
            if (!c) throw Error{BAE_ERR_ARG, "null context"};
            if (!c->rhs_ready || c->nrhs != 1) throw Error{BAE_ERR_STATE, "every context needs exactly one RHS set"};
            if (i > 0 && c->device != ctxs[0]->device) throw Error{BAE_ERR_ARG, "contexts on different devices"};
            b->ctx.push_back(c);
        }
        b->device = ctxs[0]->device;
        BAE_HIP_CHECK(hipSetDevice(b->device));
        hipDeviceProp_t prop;
        BAE_HIP_CHECK(hipGetDeviceProperties(&prop, b->device));
        b->n_cu = prop.multiProcessorCount;
        BAE_HIP_CHECK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        b->hp.resize(n);
        for (int p = 0; p < n; ++p) {
            bae_ctx* c = b->ctx[p];
            BProb& q = b->hp[p];
            q.rowptr = c->B.rowptr;
            q.col = c->B.col;
            q.coef = c->B.coef;
            q.tq = c->cl.tq;
            q.tp = c->cl.tp;
            q.tw = c->cl.t;
            q.tpos = c->t_pos.as<int32_t>();
            q.n = (int)c->ngm;
            q.nt = (int)c->nT;
            q.ns_pad = (int)c->S.ps.padded;
            q.m = c->K.m;
            q.V = c->K.V;
            q.H = c->K.H;
            q.cs = c->K.cs;
            q.sn = c->K.sn;
            q.g = c->K.g;
            q.hist = c->K.hist;
            q.beta = c->K.beta;
            q.done = c->K.done;
            q.kdone = c->K.kdone;
            q.hA = c->hA.as<double>();
            q.hB = c->hB.as<double>();
            q.nrm = c->nrm.as<double>();
            q.y = c->ycoef.as<double>();
            q.b = c->b.as<double>();
            q.x = c->x.as<double>();
            q.r = c->r.as<double>();
            q.tmp = c->tmp.as<double>();
            q.ug = c->u_gamma.as<double>();
            q.upg = c->up_gamma.as<double>();
            q.w = c->w.p;
        }
        b->kdev.alloc(sizeof(int32_t) * 4);
        b->gi.alloc(sizeof(int32_t) * n);
        b->gd.alloc(sizeof(double) * n);
        b->tol.alloc(sizeof(double) * 2);
        b->skip.alloc(sizeof(int32_t) * n);
        BAE_HIP_CHECK(hipHostMalloc((void**)&b->pinned, sizeof(int32_t) * (n + 1), hipHostMallocDefault));
        // tiling from the autotuner's cache, if any
        const std::string path = tune_cache_path();
        if (!path.empty()) {
            std::ifstream f(path);
            std::string key, line;
            double pairs = 0;
            for (auto* c : b->ctx) pairs += (double)c->nT * c->nS;
            std::ostringstream k;
            k << prop.gcnArchName << " " << (int)std::lround(std::log2(std::max(pairs, 1.0))) << " "
              << (int)std::lround(std::log2((double)n));
            while (std::getline(f, line)) {
                std::istringstream ls(line);
                std::string a, pb, nb;
                int bpc, gm;
                if ((ls >> a >> pb >> nb >> bpc >> gm) && (a + " " + pb + " " + nb) == k.str()) {
                    b->blk_per_chunk = bpc;
                    b->grid_mult = gm;
                }
            }
        }
        build_layout(b.get());
        *out = b.release();
    });
}

int bae_batch_destroy(bae_batch* b) {
    if (!b) return BAE_OK;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    release_graphs(b);
    if (b->pinned) (void)hipHostFree(b->pinned);
    hipStream_t st = b->stream;
    delete b;
    if (st) (void)hipStreamDestroy(st);
    return BAE_OK;
}

int bae_batch_autotune(bae_batch* b, int32_t precision, int32_t* chosen) {
    return guard([&] {
        if (!b) throw Error{BAE_ERR_ARG, "null batch"};
        if (precision != BAE_PREC_FP64 && precision != BAE_PREC_FP32) throw Error{BAE_ERR_ARG, "unknown precision"};
        BAE_HIP_CHECK(hipSetDevice(b->device));
        hipStream_t st = b->stream;
        hipEvent_t e0, e1;
        BAE_HIP_CHECK(hipEventCreate(&e0));
        BAE_HIP_CHECK(hipEventCreate(&e1));
        float best = 1e30f;
        int best_bpc = b->blk_per_chunk, best_gm = b->grid_mult;
        b_vec<<<nblocks(b->tot_row), kT, 0, st>>>(b->probs.as<BProb>(), b->off_row.as<int64_t>(), b->np, b->tot_row,
                                                  1);   // x = 0: the timed applies read it
        for (int bpc : {2, 4, 8, 16, 32, 64})
            for (int gm : {2, 4, 8}) {
                b->blk_per_chunk = bpc;
                b->grid_mult = gm;
                build_layout(b);
                apply_all(b, precision, 1, -1, 0);   // warm-up
                BAE_HIP_CHECK(hipEventRecord(e0, st));
                for (int r = 0; r < 3; ++r) apply_all(b, precision, 1, -1, 0);
                BAE_HIP_CHECK(hipEventRecord(e1, st));
                BAE_HIP_CHECK(hipEventSynchronize(e1));
                float ms = 0;
                BAE_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    best_bpc = bpc;
                    best_gm = gm;
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->blk_per_chunk = best_bpc;
        b->grid_mult = best_gm;
        build_layout(b);
        if (chosen) {
            chosen[0] = best_bpc;
            chosen[1] = best_gm;
        }
        const std::string path = tune_cache_path();
        if (!path.empty()) {
            hipDeviceProp_t prop;
            BAE_HIP_CHECK(hipGetDeviceProperties(&prop, b->device));
            double pairs = 0;
            for (auto* c : b->ctx) pairs += (double)c->nT * c->nS;
            std::ofstream f(path, std::ios::app);
            if (f)
                f << prop.gcnArchName << " " << (int)std::lround(std::log2(std::max(pairs, 1.0))) << " "
                  << (int)std::lround(std::log2((double)b->np)) << " " << best_bpc << " " << best_gm << "\n";
        }
    });
}

int bae_batch_solve(bae_batch* b, const bae_solve_params* prm, int32_t use_graph, bae_result* res) {
    int status = BAE_OK;
    int rc = guard([&] {
        if (!b || !prm) throw Error{BAE_ERR_ARG, "null argument"};
        if (prm->precision != BAE_SOLVE_FP64 && prm->precision != BAE_SOLVE_FP32_REFINED)
            throw Error{BAE_ERR_ARG, "unknown solve precision"};
        if (!(prm->tol > 0.0)) throw Error{BAE_ERR_ARG, "tol must be > 0"};
        BAE_HIP_CHECK(hipSetDevice(b->device));
        hipStream_t st = b->stream;
        const auto t0 = std::chrono::steady_clock::now();
        const BProb* P = b->probs.as<BProb>();
        int mmin = 1 << 30;
        for (auto* c : b->ctx) mmin = std::min(mmin, c->K.m);
        const int maxit = prm->maxit > 0 ? std::min(prm->maxit, mmin) : mmin;
        // ||b||
        norms(b, 0);
        std::vector<double> bn(b->np);
        b_gather<<<(b->np + 63) / 64, 64, 0, st>>>(P, b->np, 2, nullptr, b->gd.as<double>());
        BAE_HIP_CHECK(hipMemcpyAsync(bn.data(), b->gd.p, sizeof(double) * b->np, hipMemcpyDeviceToHost, st));
        BAE_HIP_CHECK(hipStreamSynchronize(st));
        for (auto& v : bn) v = std::sqrt(v);
        b_vec<<<nblocks(b->tot_row), kT, 0, st>>>(P, b->off_row.as<int64_t>(), b->np, b->tot_row, 1);  // x = 0
        std::vector<int> iters(b->np, 0), outer(b->np, 0);
        std::vector<double> relres;
        int64_t mv64 = 0, mv32 = 0;
        for (auto* c : b->ctx) c->hist.assign(1, {});
        auto collect_hist = [&](const std::vector<int32_t>& skip) {
            std::vector<int32_t> kd(b->np);
            b_gather<<<(b->np + 63) / 64, 64, 0, st>>>(P, b->np, 1, b->gi.as<int32_t>(), nullptr);
            BAE_HIP_CHECK(hipMemcpyAsync(kd.data(), b->gi.p, sizeof(int32_t) * b->np, hipMemcpyDeviceToHost, st));
            BAE_HIP_CHECK(hipStreamSynchronize(st));
            for (int p = 0; p < b->np; ++p) {
                if (skip[p]) continue;
                std::vector<double> h(kd[p]);
                if (kd[p] > 0)
                    BAE_HIP_CHECK(hipMemcpy(h.data(), b->hp[p].hist, sizeof(double) * kd[p], hipMemcpyDeviceToHost));
                b->ctx[p]->hist[0].insert(b->ctx[p]->hist[0].end(), h.begin(), h.end());
                iters[p] += kd[p];
            }
        };
        if (prm->precision == BAE_SOLVE_FP64) {
            std::vector<int32_t> skip(b->np, 0);
            const int k = gmres_all(b, BAE_PREC_FP64, 0, prm->tol, maxit, skip, false, use_graph != 0);
            mv64 += k;
            collect_hist(skip);
            relres = residuals(b, bn);
            mv64 += 1;
        } else {
            const double floor_tol = prm->inner_tol > 0 ? prm->inner_tol : 1e-6;
            const int max_outer = prm->max_outer > 0 ? prm->max_outer : 8;
            b_vec<<<nblocks(b->tot_row), kT, 0, st>>>(P, b->off_row.as<int64_t>(), b->np, b->tot_row, 2);  // r = b
            relres.assign(b->np, 1.0);
            for (int o = 0; o < max_outer; ++o) {
                std::vector<int32_t> skip(b->np, 0);
                bool all = true;
                double worst = 0.0;
                for (int p = 0; p < b->np; ++p) {
                    skip[p] = relres[p] <= prm->tol;
                    all &= skip[p] != 0;
                    if (!skip[p]) worst = std::max(worst, relres[p]);
                }
                if (all) break;
                const double inner = std::min(0.1, std::max(floor_tol, 0.5 * prm->tol / worst));
                const int k = gmres_all(b, BAE_PREC_FP32, 1, inner, maxit, skip, true, use_graph != 0);
                mv32 += k;
                collect_hist(skip);
                for (int p = 0; p < b->np; ++p) outer[p] += skip[p] ? 0 : 1;
                relres = residuals(b, bn);
                mv64 += 1;
            }
        }
        // u_gamma = D x + u_p on gamma
        apply_all(b, BAE_PREC_FP64, 1, -1, 0);
        b_gamma_values<<<nblocks(b->tot_tgt), kT, 0, st>>>(P, b->off_tgt.as<int64_t>(), b->np, b->tot_tgt);
        BAE_HIP_CHECK(hipGetLastError());
        BAE_HIP_CHECK(hipStreamSynchronize(st));
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int p = 0; p < b->np; ++p) {
            bae_ctx* c = b->ctx[p];
            const int conv = relres[p] <= prm->tol;
            if (!conv) status = BAE_NOT_CONVERGED;
            c->solved = true;
            c->ugrid.clear();
            if (res) {
                res[p].status = conv ? BAE_OK : BAE_NOT_CONVERGED;
                res[p].iterations = iters[p];
                res[p].outer_steps = outer[p];
                res[p].converged = conv;
                res[p].rel_residual_est = c->hist[0].empty() ? 0.0 : c->hist[0].back();
                res[p].rel_residual_true = relres[p];
                res[p].seconds = secs;
                res[p].matvecs_fp64 = mv64;
                res[p].matvecs_fp32 = mv32;
            }
        }
    });
    return rc != BAE_OK ? rc : status;
}

}  // extern "C"
