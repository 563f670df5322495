// Batched solves: many small BAE problems advanced in lock-step.
//
// Every GMRES phase (double-layer weights, LGF sum, closure, the classical Gram-Schmidt
// passes -- two in FP64, one in FP32 inner solves --, the norm, Givens) is ONE launch for
// all problems of the batch,
// over flat index spaces (per-problem offsets, binary search for the owning problem) or
// over precomputed work lists.  The LGF sum is a persistent kernel: a fixed grid walks a
// list of (problem, 1024-target tile, source chunk) items, keeping the LDS table while
// consecutive items share it.  The iteration counter lives in device memory, so one
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

#include "batch.hpp"
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
    Ctl* ctl;              // this problem's iteration counter, cap and tolerance (in its context)
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
                          int src, int use_done, const int32_t* __restrict__ sel) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    if (sel && !sel[p]) return;
    const BProb& q = P[p];
    if (use_done && q.done[0]) return;
    const int k = q.ctl->k;
    if (src == 0 && (k < 0 || k >= q.m)) return;      // never index outside the basis
    const int64_t s = gi - off[p];
    if (s >= q.ns_pad) return;
    const double* v = src == 0 ? q.V + (int64_t)k * q.n : q.x;
    double acc = 0.0;
    if (s < q.s64.ns)
        for (int j = q.rowptr[s]; j < q.rowptr[s + 1]; ++j) acc = fma(q.coef[j], v[q.col[j]], acc);
    ((Real*)q.w)[s] = (Real)acc;
}

// Persistent LGF sum over (problem, 1024-target tile, source chunk) items: each of the 16
// wavefronts of a workgroup takes one 64-target tile of the item.  The LDS table is
// restaged only when an item needs another table (sigma > 0 problems each have their own;
// every sigma = 0 problem shares one) or a larger prefix of it.
template <typename Real>
__global__ __launch_bounds__(kSumThreads) void b_lgf_sum(const BProb* __restrict__ P, const Item* __restrict__ items,
                                                         int nitems, int use_done, const int32_t* __restrict__ sel) {
    __shared__ __align__(16) char lds[lds_bytes<Real, false>()];
    const Lds<Real> L = lds_layout<Real, false>(lds);
    fill_index<Real>(L, kMaxR);
    const Real* cur = nullptr;
    int cur_r = -1;
    const int wave = threadIdx.x >> 6;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Item w = items[it];
        const BProb& q = P[w.p];
        if ((use_done && q.done[0]) || (sel && !sel[w.p])) continue;   // uniform over the block
        const SumArgs<Real>& a = sum_args<Real>(q);
        if (a.near_tab != cur || a.tab_r > cur_r) {
            __syncthreads();
            stage_table(L.tab, a.near_tab, (a.tab_r + 1) * (a.tab_r + 2) * (a.tab_r + 3) / 6);
            __syncthreads();
            cur = a.near_tab;
            cur_r = a.tab_r;
        }
        const int tile = w.tile * (kSumThreads / kWave) + wave;
        // every problem here is small: its chunk fits the scalar cache only while the
        // item's wavefronts walk it together, so no rotation
        if (tile * kWave < a.nt) sum_tile<Real, 1, false>(a, L, tile, w.chunk);
    }
}

// dst: 0 -> V[k+1], 1 -> tmp
__global__ void b_closure(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total, int dst,
                          int use_done, const int32_t* __restrict__ sel) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    if (sel && !sel[p]) return;
    const BProb& q = P[p];
    if (use_done && q.done[0]) return;
    const int k = q.ctl->k;
    if (dst == 0 && (k < 0 || k >= q.m)) return;
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    const int64_t a = q.tq[i], b = q.tp[i];
    double va = 0.0, vb = 0.0;
    for (int c = 0; c < q.chunks; ++c) {
        va += q.part[(int64_t)c * q.nt + a];
        vb += q.part[(int64_t)c * q.nt + b];
    }
    const double t = q.tw[i];
    double* out = dst == 0 ? q.V + (int64_t)(k + 1) * q.n : q.tmp;
    out[i] = (1.0 - t) * va + t * vb;
}

// u_gamma = sum of the partials (scattered to [gamma+; gamma-] order) + u_p on gamma
__global__ void b_gamma_values(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total,
                               const int32_t* __restrict__ sel) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    if (sel && !sel[p]) return;
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
                                             int mode, int sel, int use_done) {
    __shared__ double sh[kT / 64];
    const int2 w = slices[blockIdx.x];
    const BProb& q = P[w.x];
    if (use_done && q.done[0]) return;
    const int k = q.ctl->k;
    if (mode != 2 && (k < 0 || k >= q.m)) return;
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
__global__ void b_dots_finalize(const BProb* __restrict__ P, int np, int dest, int nj_mode, int use_done) {
    const int p = blockIdx.x;
    const BProb& q = P[p];
    if (use_done && q.done[0]) return;
    const int k = q.ctl->k;
    if (nj_mode == 0 && (k < 0 || k >= q.m)) return;
    const int nj = nj_mode == 0 ? k + 1 : 1;
    double* h = dest == 0 ? q.hA : dest == 1 ? q.hB : q.nrm;
    for (int j = threadIdx.x; j < nj; j += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < q.nslices; ++b) s += q.dpart[(int64_t)j * q.nslices + b];
        h[j] = s;
    }
}

__global__ void b_subtract(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total,
                           int which) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    const int k = q.ctl->k;
    if (q.done[0] || k < 0 || k >= q.m) return;
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    const double* h = which == 0 ? q.hA : q.hB;
    double acc = 0.0;
    for (int j = 0; j <= k; ++j) acc = fma(h[j], q.V[(int64_t)j * q.n + i], acc);
    q.V[(int64_t)(k + 1) * q.n + i] -= acc;
}

__global__ void b_normalize(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    const BProb& q = P[p];
    const int k = q.ctl->k;
    if (q.done[0] || k < 0 || k >= q.m) return;
    const double nr = sqrt(q.nrm[0]);
    if (gi - off[p] >= q.n) return;
    if (nr > 0.0) q.V[(int64_t)(k + 1) * q.n + gi - off[p]] /= nr;
}

// One thread per problem: Givens update of column k, residual estimate, convergence flag,
// then the problem's own step counter advances (every other kernel of the iteration has
// read it by now).
__global__ void b_givens(const BProb* __restrict__ P, int np, int two_pass) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const BProb& q = P[p];
    const int k = q.ctl->k;
    if (q.done[0]) return;
    if (k < 0 || k >= q.m || k >= q.ctl->maxit) {
        q.done[0] = 1;
        return;
    }
    double* h = q.H + (int64_t)k * (q.m + 1);
    for (int i = 0; i <= k; ++i) h[i] = two_pass ? q.hA[i] + q.hB[i] : q.hA[i];
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
    if (est <= q.ctl->tol || hk1 == 0.0 || k + 1 >= q.m || k + 1 >= q.ctl->maxit) q.done[0] = 1;
    q.ctl->k = k + 1;
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


// Start GMRES for the problems with mask[p] = 1 (r0 = b for sel 0, r for sel 1, x0 = 0), with
// the tolerance and iteration cap in ctl_init[p]; other problems are left untouched.
__global__ void b_init(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total, int sel,
                       const int32_t* __restrict__ mask, const Ctl* __restrict__ ctl_init) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    if (!mask[p]) return;
    const BProb& q = P[p];
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    const double bnorm = sqrt(q.nrm[0]);
    const double* r0 = sel == 0 ? q.b : q.r;
    if (i == 0) {
        q.beta[0] = bnorm;
        q.g[0] = bnorm;
        q.done[0] = bnorm == 0.0 ? 1 : 0;
        q.kdone[0] = 0;
        q.ctl->k = 0;
        q.ctl->maxit = ctl_init[p].maxit;
        q.ctl->tol = ctl_init[p].tol;
    }
    q.V[i] = bnorm > 0.0 ? r0[i] / bnorm : 0.0;
}

// thread per problem (mask[p] = 1): y = R^-1 g over the first kdone[p] columns
__global__ void b_backsolve(const BProb* __restrict__ P, int np, const int32_t* __restrict__ mask) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np || !mask[p]) return;
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
                           int accumulate, const int32_t* __restrict__ mask) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    if (!mask[p]) return;
    const BProb& q = P[p];
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    const int kk = q.kdone[0];
    double acc = 0.0;
    for (int j = 0; j < kk; ++j) acc = fma(q.y[j], q.V[(int64_t)j * q.n + i], acc);
    q.x[i] = accumulate ? q.x[i] + acc : acc;
}

// r = b - tmp (mode 0) ; x = 0 (mode 1) ; r = b (mode 2); masked when mask != null
__global__ void b_vec(const BProb* __restrict__ P, const int64_t* __restrict__ off, int np, int64_t total, int mode,
                      const int32_t* __restrict__ mask) {
    const int64_t gi = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (gi >= total) return;
    const int p = owner(off, np, gi);
    if (mask && !mask[p]) return;
    const BProb& q = P[p];
    const int64_t i = gi - off[p];
    if (i >= q.n) return;
    if (mode == 0) q.r[i] = q.b[i] - q.tmp[i];
    else if (mode == 1) q.x[i] = 0.0;
    else q.r[i] = q.b[i];
}

inline unsigned nblocks(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kT - 1) / kT); }

}  // namespace

// ================================================================== host engine
struct BatchEngine {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<bae_ctx*> ctx;
    int np = 0;
    DevMem probs, off_src, off_row, off_tgt, slices, items, ctl_init, mask, arena, gi, gd;
    int64_t tot_src = 0, tot_row = 0, tot_tgt = 0;
    int nslices_total = 0, nitems = 0;
    int blk_per_chunk = 8, grid_mult = 1, n_cu = 256;
    std::vector<BProb> hp;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int graph_iters = 8;
    int32_t* pinned = nullptr;
    int pinned_cap = 0;

    ~BatchEngine() {
        release_graphs();
        if (pinned) (void)hipHostFree(pinned);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    void release_graphs() {
        for (int i = 0; i < 2; ++i) {
            if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
            exec[i] = nullptr;
            graph[i] = nullptr;
        }
    }
};

namespace {

// (Re)build descriptors, per-problem chunking, the arenas and the work lists for the
// current member list.
void build_layout(BatchEngine* b) {
    b->release_graphs();
    hipStream_t st = b->stream;
    BAE_HIP_CHECK(hipStreamSynchronize(st));   // nothing in flight uses the old layout
    b->np = (int)b->ctx.size();
    b->tot_src = b->tot_row = b->tot_tgt = 0;
    b->hp.assign(b->np, BProb{});
    if (b->np == 0) return;
    if (b->pinned_cap < b->np + 1) {
        if (b->pinned) BAE_HIP_CHECK(hipHostFree(b->pinned));
        b->pinned_cap = std::max(64, 2 * (b->np + 1));
        BAE_HIP_CHECK(hipHostMalloc((void**)&b->pinned, sizeof(int32_t) * b->pinned_cap, hipHostMallocDefault));
    }
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
        const int tiles = (int)((c->nT + kSumThreads - 1) / kSumThreads);
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
    b->ctl_init.alloc(sizeof(Ctl) * b->np);
    b->mask.alloc(sizeof(int32_t) * b->np);
    b->gi.alloc(sizeof(int32_t) * b->np);
    b->gd.alloc(sizeof(double) * b->np);
    for (int p = 0; p < b->np; ++p) {
        bae_ctx* c = b->ctx[p];
        BProb& q = b->hp[p];
        q.part = b->arena.as<double>() + part_at[p];
        q.dpart = b->arena.as<double>() + dpart_at[p];
        q.ctl = c->ctl.as<Ctl>();
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
        auto fill = [&](auto& a, const auto* near, const auto* full, const auto* sxr, const auto* syr, const auto* szr) {
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
            a.txy = c->T.ps.xy16;
            a.tzl = c->T.ps.zl;
            a.sxy = c->S.ps.xy16;
            a.szl = c->S.ps.zl;
            a.sbox = c->S.ps.bbox;
            a.ns = (int)c->nS;
            a.nblk = (int)c->S.ps.nblk;
            a.blk_per_chunk = b->blk_per_chunk;
            a.ldw = c->S.ps.padded;
            a.near_tab = near;
            a.full_tab = full;
            a.full_r = c->tabs.full_r;
            a.part = q.part;
            a.ldp = (int64_t)q.chunks * c->nT;
        };
        fill(q.s64, c->tabs.near64, c->tabs.full64, c->S.ps.xd, c->S.ps.yd, c->S.ps.zd);
        q.s64.w = (const double*)c->w.p;
        q.s64.tab_r = std::min(c->tabs.tab_r64, kLdsRadius64);   // this kernel's LDS holds the general layout
        q.s64.far_ok = c->tabs.far64() ? 1 : 0;
        q.s64.far_gap = c->tabs.far_gap64();
        q.s64.yukawa = 0;
        q.s64.kq = q.s64.yk = 0.0;
        q.s64.yl = YukawaLattice{};
        fill(q.s32, c->tabs.near32, c->tabs.full32, c->S.ps.xf, c->S.ps.yf, c->S.ps.zf);
        q.s32.w = (const float*)c->w.p;
        q.s32.tab_r = std::min(c->tabs.tab_r32, kLdsRadius32);
        q.s32.far_ok = c->tabs.far32() ? 1 : 0;
        q.s32.far_gap = c->tabs.yukawa32 ? q.s32.tab_r : c->tabs.far_gap32();
        q.s32.yukawa = c->tabs.yukawa32 ? 1 : 0;
        q.s32.kq = (float)(c->tabs.kappa / kQuant);
        q.s32.yk = (float)(-c->tabs.kappa * 1.4426950408889634 / kQuant);
        q.s32.yl = yukawa_lattice(c->tabs.kappa);
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

// one operator application for all (or all unfinished) problems, src 0: V[k], 1: x;
// dst 0: V[k+1], 1: tmp, -1: partial sums only
void apply_all(BatchEngine* b, int prec, int src, int dst, int use_done, const int32_t* sel = nullptr) {
    hipStream_t st = b->stream;
    const BProb* P = b->probs.as<BProb>();
    const unsigned grid = (unsigned)std::max(1, std::min(b->nitems, b->grid_mult * b->n_cu));
    if (prec == BAE_PREC_FP64) {
        b_weights<double><<<nblocks(b->tot_src), kT, 0, st>>>(P, b->off_src.as<int64_t>(), b->np, b->tot_src, src,
                                                              use_done, sel);
        b_lgf_sum<double><<<grid, kSumThreads, 0, st>>>(P, b->items.as<Item>(), b->nitems, use_done, sel);
    } else {
        b_weights<float><<<nblocks(b->tot_src), kT, 0, st>>>(P, b->off_src.as<int64_t>(), b->np, b->tot_src, src,
                                                             use_done, sel);
        b_lgf_sum<float><<<grid, kSumThreads, 0, st>>>(P, b->items.as<Item>(), b->nitems, use_done, sel);
    }
    if (dst >= 0)
        b_closure<<<nblocks(b->tot_row), kT, 0, st>>>(P, b->off_row.as<int64_t>(), b->np, b->tot_row, dst, use_done,
                                                      sel);
    BAE_HIP_CHECK(hipGetLastError());
}

// nrm[p] = ||b|| (sel 0) or ||r|| (sel 1) squared, for every problem
void norms(BatchEngine* b, int sel) {
    hipStream_t st = b->stream;
    const BProb* P = b->probs.as<BProb>();
    b_dots<<<b->nslices_total, kT, 0, st>>>(P, b->slices.as<int2>(), b->nslices_total, 2, sel, 0);
    b_dots_finalize<<<b->np, 64, 0, st>>>(P, b->np, 2, 1, 0);
    BAE_HIP_CHECK(hipGetLastError());
}

std::vector<double> gather_nrm(BatchEngine* b) {
    hipStream_t st = b->stream;
    std::vector<double> out(b->np);
    b_gather<<<(b->np + 63) / 64, 64, 0, st>>>(b->probs.as<BProb>(), b->np, 2, nullptr, b->gd.as<double>());
    BAE_HIP_CHECK(hipMemcpyAsync(out.data(), b->gd.p, sizeof(double) * b->np, hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    return out;
}

std::vector<int32_t> gather_int(BatchEngine* b, int what) {
    hipStream_t st = b->stream;
    b_gather<<<(b->np + 63) / 64, 64, 0, st>>>(b->probs.as<BProb>(), b->np, what, b->gi.as<int32_t>(), nullptr);
    BAE_HIP_CHECK(hipMemcpyAsync(b->pinned, b->gi.p, sizeof(int32_t) * b->np, hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    return std::vector<int32_t>(b->pinned, b->pinned + b->np);
}

void upload_mask(BatchEngine* b, const std::vector<int32_t>& mask) {
    BAE_HIP_CHECK(hipMemcpyAsync(b->mask.p, mask.data(), sizeof(int32_t) * b->np, hipMemcpyHostToDevice, b->stream));
    BAE_HIP_CHECK(hipStreamSynchronize(b->stream));
}

void gmres_iteration(BatchEngine* b, int prec) {
    hipStream_t st = b->stream;
    const BProb* P = b->probs.as<BProb>();
    apply_all(b, prec, 0, 0, 1);
    const int64_t* orow = b->off_row.as<int64_t>();
    // CGS2 in FP64; one pass in the FP32 inner solves, whose results an exact FP64 residual
    // checks (as in the single-context solver)
    const int passes = prec == BAE_PREC_FP64 ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
        b_dots<<<b->nslices_total, kT, 0, st>>>(P, b->slices.as<int2>(), b->nslices_total, 0, 0, 1);
        b_dots_finalize<<<b->np, 64, 0, st>>>(P, b->np, pass, 0, 1);
        b_subtract<<<nblocks(b->tot_row), kT, 0, st>>>(P, orow, b->np, b->tot_row, pass);
    }
    b_dots<<<b->nslices_total, kT, 0, st>>>(P, b->slices.as<int2>(), b->nslices_total, 1, 0, 1);
    b_dots_finalize<<<b->np, 64, 0, st>>>(P, b->np, 2, 1, 1);
    b_normalize<<<nblocks(b->tot_row), kT, 0, st>>>(P, orow, b->np, b->tot_row);
    b_givens<<<(b->np + 63) / 64, 64, 0, st>>>(P, b->np, passes == 2);
    BAE_HIP_CHECK(hipGetLastError());
}

}  // namespace

// ---------------------------------------------------------------- engine API (batch + server)
void batch_set_members(BatchEngine* b, const std::vector<bae_ctx*>& members) {
    b->ctx = members;
    build_layout(b);
}

// Start GMRES (x0 = 0 relative to the current x when accumulating later) on the masked
// problems: r0 = b (sel 0) or r (sel 1).
void batch_begin(BatchEngine* b, const std::vector<int32_t>& mask, int sel, const std::vector<double>& tol,
                 const std::vector<int>& maxit) {
    if (b->np == 0) return;
    std::vector<Ctl> init(b->np);
    for (int p = 0; p < b->np; ++p) init[p] = Ctl{0, maxit[p], tol[p]};
    hipStream_t st = b->stream;
    BAE_HIP_CHECK(hipMemcpyAsync(b->ctl_init.p, init.data(), sizeof(Ctl) * b->np, hipMemcpyHostToDevice, st));
    BAE_HIP_CHECK(hipMemcpyAsync(b->mask.p, mask.data(), sizeof(int32_t) * b->np, hipMemcpyHostToDevice, st));
    norms(b, sel);
    b_init<<<nblocks(b->tot_row), kT, 0, st>>>(b->probs.as<BProb>(), b->off_row.as<int64_t>(), b->np, b->tot_row, sel,
                                               b->mask.as<int32_t>(), b->ctl_init.as<Ctl>());
    BAE_HIP_CHECK(hipGetLastError());
    BAE_HIP_CHECK(hipStreamSynchronize(st));   // init / mask host vectors released on return
}

// `iters` GMRES iterations of every unfinished problem (graph replay when use_graph)
void batch_iterate(BatchEngine* b, int prec, int iters, bool use_graph) {
    if (b->np == 0) return;
    hipStream_t st = b->stream;
    const int gi = prec == BAE_PREC_FP64 ? 0 : 1;
    if (use_graph) {
        if (!b->exec[gi]) {
            BAE_HIP_CHECK(hipStreamSynchronize(st));
            BAE_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < b->graph_iters; ++i) gmres_iteration(b, prec);
            BAE_HIP_CHECK(hipStreamEndCapture(st, &b->graph[gi]));
            BAE_HIP_CHECK(hipGraphInstantiate(&b->exec[gi], b->graph[gi], nullptr, nullptr, 0));
        }
        for (int i = 0; i < iters; i += b->graph_iters) BAE_HIP_CHECK(hipGraphLaunch(b->exec[gi], st));
    } else {
        for (int i = 0; i < iters; ++i) gmres_iteration(b, prec);
    }
}

std::vector<int32_t> batch_done(BatchEngine* b) { return b->np ? gather_int(b, 0) : std::vector<int32_t>{}; }
std::vector<int32_t> batch_kdone(BatchEngine* b) { return b->np ? gather_int(b, 1) : std::vector<int32_t>{}; }

// x (+)= V y for the masked problems
void batch_finish(BatchEngine* b, const std::vector<int32_t>& mask, bool accumulate) {
    if (b->np == 0) return;
    hipStream_t st = b->stream;
    BAE_HIP_CHECK(hipMemcpyAsync(b->mask.p, mask.data(), sizeof(int32_t) * b->np, hipMemcpyHostToDevice, st));
    b_backsolve<<<(b->np + 63) / 64, 64, 0, st>>>(b->probs.as<BProb>(), b->np, b->mask.as<int32_t>());
    b_update_x<<<nblocks(b->tot_row), kT, 0, st>>>(b->probs.as<BProb>(), b->off_row.as<int64_t>(), b->np, b->tot_row,
                                                   accumulate ? 1 : 0, b->mask.as<int32_t>());
    BAE_HIP_CHECK(hipGetLastError());
    BAE_HIP_CHECK(hipStreamSynchronize(st));
}

// x = 0 (mode 1) or r = b (mode 2) on the masked problems
void batch_vec(BatchEngine* b, int mode, const std::vector<int32_t>& mask) {
    if (b->np == 0) return;
    upload_mask(b, mask);
    b_vec<<<nblocks(b->tot_row), kT, 0, b->stream>>>(b->probs.as<BProb>(), b->off_row.as<int64_t>(), b->np,
                                                     b->tot_row, mode, b->mask.as<int32_t>());
    BAE_HIP_CHECK(hipGetLastError());
}

std::vector<double> batch_bnorms(BatchEngine* b) {
    if (b->np == 0) return {};
    norms(b, 0);
    std::vector<double> v = gather_nrm(b);
    for (auto& x : v) x = std::sqrt(x);
    return v;
}

// r = b - A64 x for every problem (or the masked ones); returns ||r|| per problem
std::vector<double> batch_residual_norms(BatchEngine* b, const std::vector<int32_t>* mask) {
    if (b->np == 0) return {};
    const int32_t* sel = nullptr;
    if (mask) {
        upload_mask(b, *mask);
        sel = b->mask.as<int32_t>();
    }
    apply_all(b, BAE_PREC_FP64, 1, 1, 0, sel);
    b_vec<<<nblocks(b->tot_row), kT, 0, b->stream>>>(b->probs.as<BProb>(), b->off_row.as<int64_t>(), b->np,
                                                     b->tot_row, 0, sel);
    norms(b, 1);
    std::vector<double> v = gather_nrm(b);
    for (auto& x : v) x = std::sqrt(x);
    return v;
}

// u_gamma = D x + u_p on gamma for every problem (or the masked ones)
void batch_gamma_values(BatchEngine* b, const std::vector<int32_t>* mask) {
    if (b->np == 0) return;
    const int32_t* sel = nullptr;
    if (mask) {
        upload_mask(b, *mask);
        sel = b->mask.as<int32_t>();
    }
    apply_all(b, BAE_PREC_FP64, 1, -1, 0, sel);
    b_gamma_values<<<nblocks(b->tot_tgt), kT, 0, b->stream>>>(b->probs.as<BProb>(), b->off_tgt.as<int64_t>(), b->np,
                                                             b->tot_tgt, sel);
    BAE_HIP_CHECK(hipGetLastError());
    BAE_HIP_CHECK(hipStreamSynchronize(b->stream));
}

std::vector<double> batch_history(BatchEngine* b, int p, int count) {
    std::vector<double> h(count);
    if (count > 0)
        BAE_HIP_CHECK(hipMemcpy(h.data(), b->hp[p].hist, sizeof(double) * count, hipMemcpyDeviceToHost));
    return h;
}

BatchEngine* batch_engine_new(int device, hipStream_t stream) {
    auto* b = new BatchEngine();
    b->device = device;
    hipDeviceProp_t prop;
    BAE_HIP_CHECK(hipGetDeviceProperties(&prop, device));
    b->n_cu = prop.multiProcessorCount;
    if (stream) {
        b->stream = stream;
    } else {
        BAE_HIP_CHECK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        b->own_stream = true;
    }
    return b;
}

void batch_engine_delete(BatchEngine* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
}

namespace {

std::string tune_cache_path() {
    if (const char* e = std::getenv("BAE_AUTOTUNE_CACHE")) return e;
    if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/bae_autotune.txt";
    return "";
}

std::string tune_key(BatchEngine* b) {
    hipDeviceProp_t prop;
    BAE_HIP_CHECK(hipGetDeviceProperties(&prop, b->device));
    double pairs = 0;
    for (auto* c : b->ctx) pairs += (double)c->nT * c->nS;
    std::ostringstream k;
    k << prop.gcnArchName << " " << (int)std::lround(std::log2(std::max(pairs, 1.0))) << " "
      << (int)std::lround(std::log2((double)std::max(b->np, 1)));
    return k.str();
}

// Lock-step solve of every member problem (the batched form of bae_solve).
int solve_all(BatchEngine* b, const bae_solve_params* prm, bool use_graph, bae_result* res) {
    const auto t0 = std::chrono::steady_clock::now();
    const int np = b->np;
    int mmin = 1 << 30;
    for (auto* c : b->ctx) mmin = std::min(mmin, c->K.m);
    const int maxit = prm->maxit > 0 ? std::min(prm->maxit, mmin) : mmin;
    const std::vector<int32_t> all(np, 1);
    std::vector<double> bn = batch_bnorms(b);
    batch_vec(b, 1, all);   // x = 0
    std::vector<int> iters(np, 0), outer(np, 0);
    std::vector<double> relres(np, 1.0);
    int64_t mv64 = 0, mv32 = 0;
    for (auto* c : b->ctx) c->hist.assign(1, {});
    auto run = [&](int prec, int sel, const std::vector<int32_t>& mask, const std::vector<double>& tol, bool acc) {
        std::vector<int> mx(np, maxit);
        batch_begin(b, mask, sel, tol, mx);
        int k = 0;
        while (k < maxit) {
            const int step = use_graph ? b->graph_iters : 4;
            batch_iterate(b, prec, step, use_graph);
            k += step;
            const std::vector<int32_t> d = batch_done(b);
            if (std::all_of(d.begin(), d.end(), [](int32_t v) { return v != 0; })) break;
        }
        (prec == BAE_PREC_FP64 ? mv64 : mv32) += std::min(k, maxit);
        batch_finish(b, mask, acc);
        const std::vector<int32_t> kd = batch_kdone(b);
        for (int p = 0; p < np; ++p)
            if (mask[p]) {
                const std::vector<double> h = batch_history(b, p, kd[p]);
                b->ctx[p]->hist[0].insert(b->ctx[p]->hist[0].end(), h.begin(), h.end());
                iters[p] += kd[p];
            }
    };
    if (prm->precision == BAE_SOLVE_FP64) {
        run(BAE_PREC_FP64, 0, all, std::vector<double>(np, prm->tol), false);
        const std::vector<double> rn = batch_residual_norms(b, nullptr);
        mv64 += 1;
        for (int p = 0; p < np; ++p) relres[p] = bn[p] > 0 ? rn[p] / bn[p] : 0.0;
    } else {
        const double floor_tol = prm->inner_tol > 0 ? prm->inner_tol : 1e-6;
        const int max_outer = prm->max_outer > 0 ? prm->max_outer : 8;
        batch_vec(b, 2, all);   // r = b
        for (int p = 0; p < np; ++p) relres[p] = bn[p] > 0 ? 1.0 : 0.0;
        for (int o = 0; o < max_outer; ++o) {
            std::vector<int32_t> mask(np, 0);
            std::vector<double> tol(np, 0.1);
            bool any = false;
            for (int p = 0; p < np; ++p) {
                mask[p] = relres[p] > prm->tol;
                any |= mask[p] != 0;
                if (mask[p]) tol[p] = std::min(0.1, std::max(floor_tol, 0.5 * prm->tol / relres[p]));
            }
            if (!any) break;
            run(BAE_PREC_FP32, 1, mask, tol, true);
            for (int p = 0; p < np; ++p) outer[p] += mask[p];
            const std::vector<double> rn = batch_residual_norms(b, nullptr);
            mv64 += 1;
            for (int p = 0; p < np; ++p) relres[p] = bn[p] > 0 ? rn[p] / bn[p] : 0.0;
        }
    }
    batch_gamma_values(b, nullptr);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int status = BAE_OK;
    for (int p = 0; p < np; ++p) {
        bae_ctx* c = b->ctx[p];
        const int conv = relres[p] <= prm->tol;
        if (!conv) status = BAE_NOT_CONVERGED;
        c->solved = true;
        c->has_grid = false;
        c->dens_n = c->ngm;
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
    return status;
}

}  // namespace
}  // namespace bae

using namespace bae;

struct bae_batch {
    BatchEngine* e = nullptr;
};

extern "C" {

int bae_batch_create(bae_ctx* const* ctxs, int32_t n, bae_batch** out) {
    return guard([&] {
        if (!ctxs || !out || n < 1) throw Error{BAE_ERR_ARG, "bae_batch_create: bad argument"};
        *out = nullptr;
        std::vector<bae_ctx*> members;
        for (int i = 0; i < n; ++i) {
            bae_ctx* c = ctxs[i];
            if (!c) throw Error{BAE_ERR_ARG, "null context"};
            if (!c->rhs_ready || c->nrhs != 1) throw Error{BAE_ERR_STATE, "every context needs exactly one RHS set"};
            if (i > 0 && c->device != ctxs[0]->device) throw Error{BAE_ERR_ARG, "contexts on different devices"};
            members.push_back(c);
        }
        BAE_HIP_CHECK(hipSetDevice(members[0]->device));
        auto b = std::make_unique<bae_batch>();
        b->e = batch_engine_new(members[0]->device, nullptr);
        b->e->ctx = members;
        // tiling from the autotuner's cache, if any
        const std::string path = tune_cache_path();
        if (!path.empty()) {
            std::ifstream f(path);
            const std::string key = tune_key(b->e);
            std::string line;
            while (std::getline(f, line)) {
                std::istringstream ls(line);
                std::string a, pb, nb;
                int bpc, gm;
                if ((ls >> a >> pb >> nb >> bpc >> gm) && (a + " " + pb + " " + nb) == key && bpc > 0 && gm > 0) {
                    b->e->blk_per_chunk = bpc;
                    b->e->grid_mult = gm;
                }
            }
        }
        build_layout(b->e);
        for (bae_ctx* c : members) c->batch_refs++;
        *out = b.release();
    });
}

int bae_batch_destroy(bae_batch* b) {
    if (!b) return BAE_OK;
    (void)hipSetDevice(b->e->device);
    for (bae_ctx* c : b->e->ctx) c->batch_refs--;
    batch_engine_delete(b->e);
    delete b;
    return BAE_OK;
}

int bae_batch_autotune(bae_batch* bb, int32_t precision, int32_t* chosen) {
    return guard([&] {
        if (!bb) throw Error{BAE_ERR_ARG, "null batch"};
        if (precision != BAE_PREC_FP64 && precision != BAE_PREC_FP32) throw Error{BAE_ERR_ARG, "unknown precision"};
        BatchEngine* b = bb->e;
        BAE_HIP_CHECK(hipSetDevice(b->device));
        hipStream_t st = b->stream;
        hipEvent_t e0, e1;
        BAE_HIP_CHECK(hipEventCreate(&e0));
        BAE_HIP_CHECK(hipEventCreate(&e1));
        float best = 1e30f;
        int best_bpc = b->blk_per_chunk, best_gm = b->grid_mult;
        batch_vec(b, 1, std::vector<int32_t>(b->np, 1));   // x = 0: the timed applies read it
        for (int bpc : {2, 4, 8, 16, 32, 64})
            for (int gm : {1, 2, 4}) {
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
            std::ofstream f(path, std::ios::app);
            if (f) f << tune_key(b) << " " << best_bpc << " " << best_gm << "\n";
        }
    });
}

int bae_batch_sum_stats(const bae_batch* bb, int32_t precision, int64_t* counts) {
    return guard([&] {
        if (!bb || !counts) throw Error{BAE_ERR_ARG, "null argument"};
        if (precision != BAE_PREC_FP64 && precision != BAE_PREC_FP32) throw Error{BAE_ERR_ARG, "unknown precision"};
        const bool fp32 = precision == BAE_PREC_FP32;
        for (int i = 0; i < 5; ++i) counts[i] = 0;
        // the batched sum's own classification: the general LDS layout's radii
        for (const bae_ctx* c : bb->e->ctx) {
            const int tab_r = fp32 ? std::min(c->tabs.tab_r32, kLdsRadius32) : std::min(c->tabs.tab_r64, kLdsRadius64);
            const bool far_ok = fp32 ? c->tabs.far32() : c->tabs.far64();
            const int far_gap = fp32 ? (c->tabs.yukawa32 ? tab_r : c->tabs.far_gap32()) : c->tabs.far_gap64();
            classify_pairs(c, fp32, tab_r, far_ok, far_gap, counts);
        }
    });
}

int bae_batch_solve(bae_batch* bb, const bae_solve_params* prm, int32_t use_graph, bae_result* res) {
    int status = BAE_OK;
    int rc = guard([&] {
        if (!bb || !prm) throw Error{BAE_ERR_ARG, "null argument"};
        if (prm->precision != BAE_SOLVE_FP64 && prm->precision != BAE_SOLVE_FP32_REFINED)
            throw Error{BAE_ERR_ARG, "unknown solve precision"};
        if (!(prm->tol > 0.0)) throw Error{BAE_ERR_ARG, "tol must be > 0"};
        if (prm->formulation != BAE_LAYER_DOUBLE)
            throw Error{BAE_ERR_ARG, "batched solves use the double-layer formulation"};
        if (prm->x0_dev) throw Error{BAE_ERR_ARG, "batched solves start from x0 = 0"};
        BAE_HIP_CHECK(hipSetDevice(bb->e->device));
        status = solve_all(bb->e, prm, use_graph != 0, res);
    });
    return rc != BAE_OK ? rc : status;
}

}  // extern "C"
