// C ABI of the BAE / LGF library: context set-up (Algorithm 1, set-up steps), the
// matrix-free operators, device-resident GMRES, FP64 iterative refinement around FP32
// matvecs, and the outputs.  See include/bae.h for the contract of every call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <unordered_map>

#include "context.hpp"
#include "fft.hpp"

namespace bae {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// Tables are shared by every context on a device with the same s (a larger radius
// replaces a smaller one).  The cache lives until the process ends and is never torn
// down by static destructors (the HIP runtime may already be gone by then).
static std::mutex g_table_mu;
static auto* g_tables = new std::map<std::pair<int, uint64_t>, std::shared_ptr<Table>>();

std::shared_ptr<Table> get_table(int device, double s, int R, hipStream_t st) {
    uint64_t key;
    std::memcpy(&key, &s, sizeof key);
    std::lock_guard<std::mutex> lk(g_table_mu);
    auto it = g_tables->find({device, key});
    if (it != g_tables->end() && it->second->R >= R) return it->second;
    auto t = std::make_shared<Table>();
    t->device = device;
    t->s = s;
    t->R = R;
    const int64_t E = table_size(R);
    t->d64.alloc(sizeof(double) * E);
    t->d32.alloc(sizeof(float) * E);
    lgf_table_generate(s, R, t->d64.as<double>(), st);
    launch_to_float(t->d64.as<double>(), t->d32.as<float>(), E, st);
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    (*g_tables)[{device, key}] = t;
    return t;
}

}  // namespace bae

using namespace bae;

namespace bae {

void PlanBuf::build(const PointSet& T, const PointSet& S, const SumTables& tabs, int32_t* err_dev, uint32_t polls,
                    hipStream_t st) {
    std::vector<uint32_t> host;
    plan_sum(T, S, tabs, plan, host);
    upload(items, host, st);
    counter.alloc(sizeof(unsigned long long));
    launch_fill_int(counter.as<int32_t>(), 2, 0, st);
    plan.items = items.as<uint32_t>();
    plan.counter = counter.as<unsigned long long>();
    plan.err = err_dev;
    plan.wait_polls = polls;
    BAE_HIP_CHECK(hipStreamSynchronize(st));
}

void join_job(bae_ctx* c) {
    if (c->job.th.joinable()) c->job.th.join();
}

void check_sum_error(bae_ctx* c) {
    if (!c->err_host || __atomic_load_n(c->err_host, __ATOMIC_ACQUIRE) == 0) return;
    BAE_HIP_CHECK(hipSetDevice(c->device));
    BAE_HIP_CHECK(hipDeviceSynchronize());   // no sum of this context is still in flight
    launch_fill_int(c->plan.counter.as<int32_t>(), 2, 0, c->stream);
    BAE_HIP_CHECK(hipStreamSynchronize(c->stream));
    __atomic_store_n(c->err_host, 0, __ATOMIC_RELEASE);
    throw Error{BAE_ERR_HIP, "LGF sum: a bounded wait of the work hand-off gave up; the results of the calls "
                             "since the last check are incomplete"};
}

// The source weights are FP32 only for the FP32 sum kernels; the FFT convolution takes FP64.
static int weight_prec(int prec) { return prec == BAE_PREC_FP32 ? BAE_PREC_FP32 : BAE_PREC_FP64; }

// Box indices of a point set's points (internal order) in the convolution box.
static std::vector<int32_t> conv_indices(const ConvPlan& cp, const PointSet& ps) {
    std::vector<int32_t> v(ps.count);
    for (int64_t i = 0; i < ps.count; ++i)
        v[i] = (int32_t)cp.index(ps.hq[3 * i] / kQuant, ps.hq[3 * i + 1] / kQuant, ps.hq[3 * i + 2] / kQuant);
    return v;
}

static void ensure_mplus(bae_ctx* c);

// The FFT convolution of the LGF sum (lazy, once per context): its plan on the box of N+ u E
// and the box index of every source and target.
static void ensure_conv(bae_ctx* c, bool mplus = false) {
    if (!c->conv) {
        const Geometry& G = c->geo;
        int64_t box = 1;
        for (int a = 0; a < 3; ++a) box *= (int64_t)(G.bbox_hi[a] - G.bbox_lo[a] + 1);
        if (box > INT32_MAX) throw Error{BAE_ERR_ARG, "LGF convolution: box beyond 2^31 nodes"};
        auto cp = std::make_unique<ConvPlan>();
        cp->build(G.bbox_lo, G.bbox_hi, c->tabs, c->stream);
        upload(c->conv_sidx, conv_indices(*cp, c->S.ps), c->stream);
        upload(c->conv_tidx, conv_indices(*cp, c->T.ps), c->stream);
        BAE_HIP_CHECK(hipStreamSynchronize(c->stream));
        c->conv = std::move(cp);
    }
    if (mplus && !c->conv_midx.p) {
        ensure_mplus(c);
        upload(c->conv_midx, conv_indices(*c->conv, c->Mp.ps), c->stream);
        BAE_HIP_CHECK(hipStreamSynchronize(c->stream));
    }
}

// The current operator's LGF sum at the gamma targets (its sources, weights, work list), or
// with BAE_PREC_FFT its FFT convolution (one partial per target, FP64).
static void apply_lgf(bae_ctx* c, const void* w, int nrhs, int prec, int* chunks_out, hipStream_t st,
                      const int32_t* skip = nullptr) {
    if (prec == BAE_PREC_FFT) {
        ensure_conv(c);
        const int32_t* sidx = c->op.direct ? c->conv_tidx.as<int32_t>() : c->conv_sidx.as<int32_t>();
        const int64_t ldw = c->op.S->padded;
        for (int r = 0; r < nrhs; ++r)
            c->conv->apply((const double*)w + r * ldw, sidx, c->op.S->count, c->conv_tidx.as<int32_t>(), c->nT,
                           c->part.as<double>() + r * c->nT, 1.0, skip, st);
        *chunks_out = 1;
        return;
    }
    *chunks_out = lgf_sum_launch(c->T.ps, *c->op.S, w, nrhs, prec, c->tabs, c->op.plan->plan, c->part.as<double>(),
                                 c->part_cap, c->sum_grid, st, skip);
}

// v = [D+ q; D- q] (external order) for the layer potential of c->op (double or single
// layer), q [nrhs][ngm] with leading dimension ldq
static void double_layer(bae_ctx* c, const double* q, int64_t ldq, double* v, int64_t ldv, int nrhs, int prec,
                         hipStream_t st) {
    launch_weights(*c->op.B, q, ldq, c->w.p, c->op.S->padded, nrhs, weight_prec(prec), st);
    int chunks = 0;
    apply_lgf(c, c->w.p, nrhs, prec, &chunks, st);
    launch_reduce_scatter(c->part.as<double>(), chunks, c->nT, c->t_pos.as<int32_t>(), v, ldv, nrhs, 1.0, st);
}

// The closing step of the operator from the chunk partials: the Dirichlet rows Phi+ v+ +
// Phi- v- of the layer potential (Sec. 3.4), or for the direct formulation v+ + (the sum) on
// gamma+ and the Dirichlet rows of v itself on gamma- (v: the operator's input).
static void op_closure(bae_ctx* c, int chunks, const double* v, int64_t ldv, double* aq, int64_t lda, int nrhs,
                       hipStream_t st) {
    if (c->op.direct)
        launch_direct_closure(c->part.as<double>(), chunks, c->nT, c->t_inv.as<int32_t>(), c->ngp,
                              c->partner_dev.as<int32_t>(), c->cl_t.as<double>(), v, ldv, aq, lda, nrhs,
                              c->vsum.as<double>(), st);
    else
        launch_closure(c->part.as<double>(), chunks, c->nT, c->cl, aq, lda, nrhs, c->vsum.as<double>(), st);
}

// aq = A q for the current operator: Phi+ D+ q + Phi- D- q (double / single layer) or the
// direct system (the LGF sum skipped while *skip is set, when given)
static void bae_operator(bae_ctx* c, const double* q, int64_t ldq, double* aq, int64_t lda, int nrhs, int prec,
                         hipStream_t st, const int32_t* skip = nullptr) {
    launch_weights(*c->op.B, q, ldq, c->w.p, c->op.S->padded, nrhs, weight_prec(prec), st);
    int chunks = 0;
    apply_lgf(c, c->w.p, nrhs, prec, &chunks, st, skip);
    op_closure(c, chunks, q, ldq, aq, lda, nrhs, st);
}

static void norms2(bae_ctx* c, const double* v, int64_t ldv, int nrhs, double* out_dev, hipStream_t st) {
    launch_dots(v, 0, ldv, 1, v, ldv, c->op.n, nrhs, nullptr, c->dotpart.as<double>(), c->maxj, out_dev, 1, 0, st);
}

struct GmresOut {
    std::vector<int> iters;
    std::vector<int> converged;
    std::vector<double> last_est;
};

// Krylov recycling between the inner solves of a refined solve (GCRO, de Sturler): U and
// C = A32 U with orthonormal columns, from the first inner solve's Arnoldi relation
// A32 V_k = V_{k+1} Hbar: with Hbar = Q R (the solve's own Givens rotations give Q, its
// triangular factor R), U = V_k R^-1 and C = V_{k+1} Q.  A later inner solve first takes
// the part of its right-hand side in the span of C, then runs GMRES on the rest with every
// new Krylov vector orthogonalised against C as well; the coefficients of that step (the
// slices of C'w) are kept for the final update.  A restarted solve would rebuild those
// directions from nothing: its right-hand side, the FP32 operator's error, converges slowly.
struct Recycle {
    int p = 0;                    // recycled vectors per RHS (0: none)
    int64_t ld = 0;               // p * n, per-RHS stride of U and C
    double* U = nullptr;
    double* C = nullptr;
    double* slices = nullptr;     // [step][rhs][p][dot_blocks(n)]
};
constexpr int kRecycleDefault = 64;

// Set-up of the direct formulation (Sec. 3.1), once per context: the boundary edges (p in
// gamma+, q in gamma-, neighbours), the weights map of its gamma+ rows -- a source at q
// carries +v(p), a source at p carries -v(q), summed over the edges, so that the LGF sum at
// p* is sum_edges [G(q - p*) v(p) - G(p - p*) v(q)] -- over the targets' own point set, the
// (gamma, gamma) work list, and vectors of |gamma| unknowns.
static void ensure_direct(bae_ctx* c) {
    if (c->direct_ready) return;
    if (c->vec_cap < c->nT && c->batch_refs > 0)
        throw Error{BAE_ERR_STATE, "a direct solve grows the context's vectors: not while it belongs to a batch"};
    hipStream_t st = c->stream;
    const Geometry& G = c->geo;
    std::unordered_map<int64_t, int32_t> gp_at;
    gp_at.reserve((size_t)c->ngp * 2);
    auto lin = [&](const int32_t* v) { return ((int64_t)v[0] * G.n[1] + v[1]) * G.n[2] + v[2]; };
    for (int64_t i = 0; i < c->ngp; ++i) gp_at[lin(&G.gp[3 * i])] = (int32_t)i;
    static const int dirs[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    std::vector<std::vector<std::pair<int32_t, double>>> rows(c->nT);   // by position in [gamma+; gamma-]
    for (int64_t q = 0; q < c->ngm; ++q) {
        const int32_t* v = &G.gm[3 * q];
        for (const auto& d : dirs) {
            const int32_t m[3] = {v[0] + d[0], v[1] + d[1], v[2] + d[2]};
            if (m[0] < 0 || m[1] < 0 || m[2] < 0 || m[0] >= G.n[0] || m[1] >= G.n[1] || m[2] >= G.n[2]) continue;
            if (!G.inside[lin(m)]) continue;
            const auto it = gp_at.find(lin(m));
            if (it == gp_at.end()) throw Error{BAE_ERR_GEOMETRY, "an M+ neighbour of gamma- is not in gamma+"};
            rows[c->ngp + q].push_back({it->second, 1.0});
            rows[it->second].push_back({(int32_t)(c->ngp + q), -1.0});
        }
    }
    std::vector<int32_t> rowptr(c->nT + 1, 0), col, tinv(c->nT);
    std::vector<double> coef;
    for (int64_t i = 0; i < c->nT; ++i) {   // internal (Morton) target order
        const int32_t j = c->T.perm[i];
        tinv[j] = (int32_t)i;
        for (const auto& e : rows[j]) {
            col.push_back(e.first);
            coef.push_back(e.second);
        }
        rowptr[i + 1] = (int32_t)col.size();
    }
    upload(c->csrd_rowptr, rowptr, st);
    upload(c->csrd_col, col, st);
    upload(c->csrd_coef, coef, st);
    upload(c->t_inv, tinv, st);
    c->Bd = CSR{c->nT, c->T.ps.padded, c->csrd_rowptr.as<int32_t>(), c->csrd_col.as<int32_t>(),
                c->csrd_coef.as<double>()};
    c->plan_dir.build(c->T.ps, c->T.ps, c->tabs, c->err_dev, c->wait_polls, st);
    const int mr = c->max_rhs;
    if (c->w.bytes < sizeof(double) * c->T.ps.padded * mr) c->w.alloc(sizeof(double) * std::max(c->T.ps.padded, c->S.ps.padded) * mr);
    const int64_t pc = (int64_t)c->plan_dir.plan.chunks * c->nT * mr;
    if (pc > c->part_cap) {
        c->part.alloc(sizeof(double) * pc);
        c->part_cap = pc;
    }
    c->bdir.alloc(sizeof(double) * c->nT * mr);
    if (c->vec_cap < c->nT) {
        const int64_t n = c->nT, m = c->K.m;
        for (DevMem* d : {&c->x, &c->r, &c->tmp}) d->alloc(sizeof(double) * n * mr);
        c->kV.alloc(sizeof(double) * (m + 1) * n * mr);
        c->K.V = c->kV.as<double>();
        c->dotpart.alloc(sizeof(double) * mr * (2 * (int64_t)c->maxj * dot_blocks(n) + norm_blocks(n)));
        c->vec_cap = n;
    }
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    c->direct_ready = true;
}

// The double-layer operator (the default outside a solve).
static void use_double_layer(bae_ctx* c) {
    c->op = bae_ctx::OpView{&c->B, &c->S.ps, &c->plan, c->ngm, false};
    c->K.n = c->ngm;
    c->K.ld_rhs = (int64_t)(c->K.m + 1) * c->ngm;
}

// Selects the operator of a formulation for a scope (the double layer outside it): the
// single layer's weights map over the same sources, or the direct formulation's map, sources
// and unknowns; the Krylov vectors take the operator's length.
struct LayerScope {
    bae_ctx* c;
    LayerScope(bae_ctx* ctx, int32_t formulation) : c(ctx) {
        if (formulation == BAE_LAYER_DIRECT) {
            ensure_direct(c);
            c->op = bae_ctx::OpView{&c->Bd, &c->T.ps, &c->plan_dir, c->nT, true};
        } else {
            c->op = bae_ctx::OpView{formulation == BAE_LAYER_SINGLE ? &c->B1 : &c->B, &c->S.ps, &c->plan, c->ngm,
                                    false};
        }
        c->K.n = c->op.n;
        c->K.ld_rhs = (int64_t)(c->K.m + 1) * c->op.n;
    }
    ~LayerScope() { use_double_layer(c); }
};

static void build_recycle(bae_ctx* c, int nrhs, const std::vector<int>& skip, int cap, Recycle& rc, hipStream_t st) {
    KrylovState& K = c->K;
    const int64_t n = c->op.n;
    rc.p = 0;
    std::vector<int32_t> kd(nrhs);
    BAE_HIP_CHECK(hipMemcpyAsync(kd.data(), K.kdone, sizeof(int32_t) * nrhs, hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    int p = 0;
    for (int r = 0; r < nrhs; ++r)
        if (skip.empty() || !skip[r]) p = std::max(p, (int)kd[r]);
    p = std::min(p, cap);
    if (p < 2) return;
    const int64_t hsz = (int64_t)K.m * (K.m + 1);
    std::vector<double> H((size_t)hsz * nrhs), cs((size_t)K.m * nrhs), sn((size_t)K.m * nrhs);
    BAE_HIP_CHECK(hipMemcpyAsync(H.data(), K.H, sizeof(double) * H.size(), hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipMemcpyAsync(cs.data(), K.cs, sizeof(double) * cs.size(), hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipMemcpyAsync(sn.data(), K.sn, sizeof(double) * sn.size(), hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    std::vector<double> MQ((size_t)nrhs * (p + 1) * p, 0.0), MU((size_t)nrhs * p * p, 0.0);
    for (int r = 0; r < nrhs; ++r) {
        if (!skip.empty() && skip[r]) continue;
        const int k = std::min((int)kd[r], p);
        const double* Hr = H.data() + r * hsz;
        auto R = [&](int i, int j) { return Hr[(int64_t)j * (K.m + 1) + i]; };   // R[i][j], i <= j < k
        bool ok = k >= 1;
        for (int j = 0; j < k && ok; ++j) ok = std::isfinite(R(j, j)) && R(j, j) != 0.0;
        if (!ok) continue;   // this RHS recycles nothing (its columns stay zero)
        // Q = G_0' G_1' ... G_{k-1}' [I_k; 0]; rotation j mixes rows j, j + 1 as (c s; -s c)
        double* q = MQ.data() + (size_t)r * (p + 1) * p;
        for (int l = 0; l < k; ++l) q[l * p + l] = 1.0;
        for (int j = k - 1; j >= 0; --j) {
            const double cj = cs[(size_t)r * K.m + j], sj = sn[(size_t)r * K.m + j];
            for (int l = 0; l < k; ++l) {
                const double a = q[j * p + l], b = q[(j + 1) * p + l];
                q[j * p + l] = cj * a - sj * b;
                q[(j + 1) * p + l] = sj * a + cj * b;
            }
        }
        // R^-1 (upper triangular), column by column
        double* u = MU.data() + (size_t)r * p * p;
        for (int l = 0; l < k; ++l) {
            u[l * p + l] = 1.0 / R(l, l);
            for (int i = l - 1; i >= 0; --i) {
                double acc = 0.0;
                for (int j = i + 1; j <= l; ++j) acc += R(i, j) * u[j * p + l];
                u[i * p + l] = -acc / R(i, i);
            }
        }
    }
    const int64_t per = (int64_t)nrhs * p * n;
    if (c->rcU.bytes < sizeof(double) * per) c->rcU.alloc(sizeof(double) * per);
    if (c->rcC.bytes < sizeof(double) * per) c->rcC.alloc(sizeof(double) * per);
    const int64_t sl = (int64_t)K.m * nrhs * p * dot_blocks(n);
    if (c->rcS.bytes < sizeof(double) * sl) c->rcS.alloc(sizeof(double) * sl);
    DevMem mq, mu;
    upload(mq, MQ, st);
    upload(mu, MU, st);
    rc.p = p;
    rc.ld = (int64_t)p * n;
    rc.U = c->rcU.as<double>();
    rc.C = c->rcC.as<double>();
    rc.slices = c->rcS.as<double>();
    launch_basis_transform(K.V, n, K.ld_rhs, p + 1, mq.as<double>(), p, n, nrhs, rc.C, n, rc.ld, st);
    launch_basis_transform(K.V, n, K.ld_rhs, p, mu.as<double>(), p, n, nrhs, rc.U, n, rc.ld, st);
    BAE_HIP_CHECK(hipStreamSynchronize(st));   // mq, mu are released on return
}

// x += U C'r and r -= C C'r (the part of r in the span of C), skipped RHS left alone.
static void recycle_project(bae_ctx* c, const Recycle& rc, int nrhs, const std::vector<int>& skip, double* x,
                            double* r, hipStream_t st) {
    const int64_t n = c->op.n;
    DevMem c0, pn;
    c0.alloc(sizeof(double) * 2 * nrhs * rc.p);
    launch_dots(rc.C, n, rc.ld, rc.p, r, n, n, nrhs, nullptr, c->dotpart.as<double>(), c->maxj, c0.as<double>(),
                rc.p, 0, st);
    std::vector<double> h((size_t)2 * nrhs * rc.p);
    BAE_HIP_CHECK(hipMemcpyAsync(h.data(), c0.p, sizeof(double) * nrhs * rc.p, hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    for (int q = 0; q < nrhs; ++q)
        for (int l = 0; l < rc.p; ++l) {
            double& v = h[(size_t)q * rc.p + l];
            if (!skip.empty() && skip[q]) v = 0.0;
            h[(size_t)nrhs * rc.p + (size_t)q * rc.p + l] = -v;
        }
    BAE_HIP_CHECK(hipMemcpyAsync(c0.p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st));
    std::vector<int32_t> pv(nrhs, rc.p);
    upload(pn, pv, st);
    launch_combination(rc.U, n, rc.ld, c0.as<double>(), rc.p, pn.as<int32_t>(), n, nrhs, x, n, 1, st);
    launch_combination(rc.C, n, rc.ld, c0.as<double>() + (int64_t)nrhs * rc.p, rc.p, pn.as<int32_t>(), n, nrhs, r, n,
                       1, st);
    BAE_HIP_CHECK(hipStreamSynchronize(st));
}

// GMRES on A d = r0 for nrhs RHS (x0 = 0), then x (+)= d.  skip[r] marks RHS left alone.
// With rc, every Krylov vector is first orthogonalised against rc.C and x gets the matching
// U correction (GCRO).
static GmresOut gmres(bae_ctx* c, const double* r0, int nrhs, int prec, double tol, int maxit,
                      const std::vector<int>& skip, double* xout, bool accumulate, hipStream_t st,
                      int64_t* matvecs, const Recycle* rc = nullptr) {
    KrylovState& K = c->K;
    const int64_t n = c->op.n;
    const int m = std::min(maxit, K.m);
    norms2(c, r0, n, nrhs, c->nrm.as<double>(), st);
    launch_gmres_init(r0, n, K, n, c->nrm.as<double>(), nrhs, st);
    if (!skip.empty()) {
        std::vector<int32_t> d(nrhs);
        for (int r = 0; r < nrhs; ++r) d[r] = skip[r] ? 1 : 0;
        for (int r = 0; r < nrhs; ++r)
            if (skip[r]) BAE_HIP_CHECK(hipMemcpyAsync(K.done + r, &d[r], sizeof(int32_t), hipMemcpyHostToDevice, st));
        BAE_HIP_CHECK(hipStreamSynchronize(st));
    }
    // Convergence is read back from the device.  With one RHS the host keeps one iteration
    // queued ahead and reads the flags of the previous one, so the device never waits for
    // the host; the queued iteration after convergence skips its LGF sum (the GMRES kernels
    // skip converged RHS anyway).  With several RHS every `check`-th iteration is synchronous.
    const bool lagged = nrhs == 1;
    const double pairs = (double)c->nT * (double)c->nS * nrhs;
    const int check = pairs > 2e7 ? 1 : (pairs > 2e6 ? 2 : 6);
    struct Events {   // released on every exit, errors included
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
            for (auto& x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } evs;
    hipEvent_t* ev = evs.e;
    if (lagged)
        for (int i = 0; i < 2; ++i) BAE_HIP_CHECK(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    // Step k: LGF sum of the weights of V[k] (formed by step k-1's closing launch, or here
    // for k = 0), closure into the work vector, classical Gram-Schmidt, then one closing
    // launch that scales the work vector into V[k+1], forms the next weights from it and
    // updates Givens.  FP64 solves orthogonalise twice (CGS2).  The FP32 inner solves of a
    // refined solve stop near 1e-6 and every result they feed is checked by an exact FP64
    // residual, so one pass is enough there: the two launches of the second pass cost 14% of
    // a 33^3 refined solve and change no iteration count on the test problems.
    const bool two_pass = prec != BAE_PREC_FP32;
    double* wv = c->tmp.as<double>();
    double* pA = c->dotpart.as<double>();
    double* pB = pA + (int64_t)nrhs * c->maxj * dot_blocks(n);
    double* pN = pB + (int64_t)nrhs * c->maxj * dot_blocks(n);
    launch_weights(*c->op.B, K.V, K.ld_rhs, c->w.p, c->op.S->padded, nrhs, weight_prec(prec), st);
    int k = 0;
    for (; k < m; ++k) {
        int chunks = 0;
        apply_lgf(c, c->w.p, nrhs, prec, &chunks, st, lagged ? K.done : nullptr);
        op_closure(c, chunks, K.V + (int64_t)k * n, K.ld_rhs, wv, n, nrhs, st);
        (*matvecs)++;
        if (rc) {   // w -= C (C'w), the coefficients kept for the final update
            double* sl = rc->slices + (int64_t)k * nrhs * rc->p * dot_blocks(n);
            launch_dot_slices(rc->C, n, rc->ld, rc->p, wv, n, n, nrhs, K.done, sl, rc->p, st);
            launch_subtract_combination(rc->C, n, rc->ld, sl, rc->p, rc->p, n, nrhs, K.done, wv, n, nullptr, st);
        }
        // classical Gram-Schmidt (dot-product slices in pA, and in pB for the second pass);
        // the last pass also forms the slices of ||w||^2 (pN), which the closing launch sums
        launch_dot_slices(K.V, n, K.ld_rhs, k + 1, wv, n, n, nrhs, K.done, pA, c->maxj, st);
        launch_subtract_combination(K.V, n, K.ld_rhs, pA, c->maxj, k + 1, n, nrhs, K.done, wv, n,
                                    two_pass ? nullptr : pN, st);
        if (two_pass) {
            launch_dot_slices(K.V, n, K.ld_rhs, k + 1, wv, n, n, nrhs, K.done, pB, c->maxj, st);
            launch_subtract_combination(K.V, n, K.ld_rhs, pB, c->maxj, k + 1, n, nrhs, K.done, wv, n, pN, st);
        }
        launch_finish(K, wv, n, pA, two_pass ? pB : nullptr, c->maxj, pN, k, tol, *c->op.B, c->w.p, c->op.S->padded,
                      weight_prec(prec), nrhs, lagged ? c->flags_dev + (k & 1) : nullptr, st);
        if (lagged) {
            BAE_HIP_CHECK(hipEventRecord(ev[k & 1], st));
            if (k >= 1) {
                BAE_HIP_CHECK(hipEventSynchronize(ev[(k - 1) & 1]));
                check_sum_error(c);
                if (c->pinned_flags[(k - 1) & 1]) {
                    (*matvecs)--;   // the LGF sum of iteration k was skipped
                    break;
                }
            }
            if (k + 1 == m) BAE_HIP_CHECK(hipEventSynchronize(ev[k & 1]));
        } else if ((k + 1) % check == 0 || k + 1 == m) {
            BAE_HIP_CHECK(hipMemcpyAsync(c->pinned_flags, K.done, sizeof(int32_t) * nrhs, hipMemcpyDeviceToHost, st));
            BAE_HIP_CHECK(hipStreamSynchronize(st));
            check_sum_error(c);
            bool all = true;
            for (int r = 0; r < nrhs; ++r) all &= c->pinned_flags[r] != 0;
            if (all) {
                ++k;
                break;
            }
        }
    }
    // host back substitution R y = g for each RHS
    std::vector<int32_t> kd(nrhs), dn(nrhs);
    BAE_HIP_CHECK(hipMemcpyAsync(kd.data(), K.kdone, sizeof(int32_t) * nrhs, hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipMemcpyAsync(dn.data(), K.done, sizeof(int32_t) * nrhs, hipMemcpyDeviceToHost, st));
    const int64_t hsz = (int64_t)K.m * (K.m + 1);
    std::vector<double> H((size_t)hsz * nrhs), g((size_t)(K.m + 1) * nrhs), hs((size_t)K.m * nrhs);
    BAE_HIP_CHECK(hipMemcpyAsync(H.data(), K.H, sizeof(double) * H.size(), hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipMemcpyAsync(g.data(), K.g, sizeof(double) * g.size(), hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipMemcpyAsync(hs.data(), K.hist, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    check_sum_error(c);
    GmresOut out;
    std::vector<double> y((size_t)K.m * nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r) {
        const int kk = (!skip.empty() && skip[r]) ? 0 : kd[r];
        const double* Hr = H.data() + r * hsz;
        const double* gr = g.data() + (size_t)r * (K.m + 1);
        double* yr = y.data() + (size_t)r * K.m;
        for (int i = kk - 1; i >= 0; --i) {
            double acc = gr[i];
            for (int j = i + 1; j < kk; ++j) acc -= Hr[(int64_t)j * (K.m + 1) + i] * yr[j];
            const double d = Hr[(int64_t)i * (K.m + 1) + i];
            yr[i] = d != 0.0 ? acc / d : 0.0;
        }
        kd[r] = kk;
        out.iters.push_back(kk);
        out.last_est.push_back(kk > 0 ? hs[(size_t)r * K.m + kk - 1] : 0.0);
        out.converged.push_back((!skip.empty() && skip[r]) ? 1 : (dn[r] && (kk == 0 || hs[(size_t)r * K.m + kk - 1] <= tol)));
        if (!(!skip.empty() && skip[r]))
            c->hist[r].insert(c->hist[r].end(), hs.begin() + (size_t)r * K.m, hs.begin() + (size_t)r * K.m + kk);
    }
    BAE_HIP_CHECK(hipMemcpyAsync(c->ycoef.p, y.data(), sizeof(double) * y.size(), hipMemcpyHostToDevice, st));
    DevMem kdev;
    kdev.alloc(sizeof(int32_t) * nrhs);
    BAE_HIP_CHECK(hipMemcpyAsync(kdev.p, kd.data(), sizeof(int32_t) * nrhs, hipMemcpyHostToDevice, st));
    launch_combination(K.V, n, K.ld_rhs, c->ycoef.as<double>(), K.m, kdev.as<int32_t>(), n, nrhs, xout, n,
                       accumulate ? 1 : 0, st);
    if (rc) {
        // x -= U (B y), B[l][j] = C_l' w_j summed from step j's slices
        const int nbd = dot_blocks(n);
        int kmax = 0;
        for (int r = 0; r < nrhs; ++r) kmax = std::max(kmax, kd[r]);
        std::vector<double> sl((size_t)kmax * nrhs * rc->p * nbd), z((size_t)nrhs * rc->p, 0.0);
        if (kmax > 0)
            BAE_HIP_CHECK(hipMemcpyAsync(sl.data(), rc->slices, sizeof(double) * sl.size(), hipMemcpyDeviceToHost, st));
        BAE_HIP_CHECK(hipStreamSynchronize(st));
        for (int r = 0; r < nrhs; ++r)
            for (int j = 0; j < kd[r]; ++j) {
                const double yj = y[(size_t)r * K.m + j];
                for (int l = 0; l < rc->p; ++l) {
                    const double* b = sl.data() + (((size_t)j * nrhs + r) * rc->p + l) * nbd;
                    double blj = 0.0;
                    for (int q = 0; q < nbd; ++q) blj += b[q];
                    z[(size_t)r * rc->p + l] -= blj * yj;
                }
            }
        DevMem zd, pn;
        upload(zd, z, st);
        std::vector<int32_t> pv(nrhs, rc->p);
        upload(pn, pv, st);
        launch_combination(rc->U, n, rc->ld, zd.as<double>(), rc->p, pn.as<int32_t>(), n, nrhs, xout, n, 1, st);
    }
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    return out;
}

// The right-hand side of the current operator's system: b, or [0; b] for the direct one.
static const double* rhs_vector(bae_ctx* c) { return c->op.direct ? c->bdir.as<double>() : c->b.as<double>(); }

static std::vector<double> host_norms(bae_ctx* c, const double* v, int nrhs, hipStream_t st) {
    norms2(c, v, c->op.n, nrhs, c->nrm.as<double>(), st);
    std::vector<double> h(nrhs);
    BAE_HIP_CHECK(hipMemcpyAsync(h.data(), c->nrm.p, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    for (auto& v2 : h) v2 = std::sqrt(v2);
    return h;
}

// r = b - A64 x ; returns ||r|| / ||b|| per RHS
static std::vector<double> residual(bae_ctx* c, int nrhs, const std::vector<double>& bn, hipStream_t st,
                                    int64_t* matvecs, int prec = BAE_PREC_FP64) {
    const int64_t n = c->op.n;
    bae_operator(c, c->x.as<double>(), n, c->tmp.as<double>(), n, nrhs, prec, st);
    (*matvecs)++;
    BAE_HIP_CHECK(hipMemcpyAsync(c->r.p, rhs_vector(c), sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, st));
    launch_axpby(-1.0, c->tmp.as<double>(), n, 1.0, c->r.as<double>(), n, n, nrhs, st);
    std::vector<double> rn = host_norms(c, c->r.as<double>(), nrhs, st);
    check_sum_error(c);
    for (int i = 0; i < nrhs; ++i) rn[i] = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
    return rn;
}

static void ensure_mplus(bae_ctx* c) {
    if (c->Mp.ps.count) return;
    const Geometry& G = c->geo;
    std::vector<int32_t> pts;
    pts.reserve(3 * G.n_mplus);
    for (int i = 0; i < G.n[0]; ++i)
        for (int j = 0; j < G.n[1]; ++j)
            for (int k = 0; k < G.n[2]; ++k)
                if (G.inside[((int64_t)i * G.n[1] + j) * G.n[2] + k]) pts.insert(pts.end(), {i, j, k});
    const std::vector<int32_t> ord = morton_order(pts.data(), (int64_t)pts.size() / 3, G.bbox_lo);
    c->Mp.set(pts, ord, c->stream);
}

int guard(const std::function<void()>& fn) {
    try {
        fn();
        return BAE_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return BAE_ERR_OOM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return BAE_ERR_ARG;
    }
}

}  // namespace bae

namespace bae {

bae_ctx* create_context(const bae_grid& gridv, const bae_options* opt, Geometry&& geo) {
    const bae_grid* grid = &gridv;
        auto c = std::make_unique<bae_ctx>();
        c->grid = *grid;
        if (opt) c->opt = *opt;
        c->max_rhs = c->opt.max_rhs > 0 ? c->opt.max_rhs : 16;
        if (c->max_rhs > 64) throw Error{BAE_ERR_ARG, "max_rhs must be <= 64"};
        const int m = c->opt.max_krylov > 0 ? c->opt.max_krylov : 400;
        if (m > 4096) throw Error{BAE_ERR_ARG, "max_krylov must be <= 4096"};
        if (c->opt.near_radius_fp64 || c->opt.near_radius_fp32)
            throw Error{BAE_ERR_ARG, "near radius: fixed by the kernels' LDS layout, pass 0"};
        c->device = c->opt.device;
        int ndev = 0;
        BAE_HIP_CHECK(hipGetDeviceCount(&ndev));
        if (c->device < 0 || c->device >= ndev) throw Error{BAE_ERR_ARG, "no such device"};
        BAE_HIP_CHECK(hipSetDevice(c->device));
        BAE_HIP_CHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        hipStream_t st = c->stream;

        c->geo = std::move(geo);
        Geometry& G = c->geo;
        c->s = grid->sigma * grid->h * grid->h;
        c->ngp = (int64_t)G.gp.size() / 3;
        c->ngm = (int64_t)G.gm.size() / 3;
        c->next = (int64_t)G.ext.size() / 3;
        c->nT = c->ngp + c->ngm;
        c->nS = c->ngm + c->next;
        if (c->s > 0.0 && G.max_offset > kMaxTableRadius)
            throw Error{BAE_ERR_ARG, "sigma > 0 needs offsets <= " + std::to_string(kMaxTableRadius)};

        // targets: gamma+ then gamma- (external order), Morton-sorted internally
        std::vector<int32_t> tp(G.gp);
        tp.insert(tp.end(), G.gm.begin(), G.gm.end());
        std::vector<int32_t> tord = morton_order(tp.data(), c->nT, G.bbox_lo);
        c->T.set(tp, tord, st);
        std::vector<int32_t> tpos(c->nT), tinv(c->nT);
        for (int64_t i = 0; i < c->nT; ++i) {
            tpos[i] = tord[i];
            tinv[tord[i]] = (int32_t)i;
        }
        upload(c->t_pos, tpos, st);
        // sources: gamma- then E, Morton-sorted internally
        std::vector<int32_t> sp(G.gm);
        sp.insert(sp.end(), G.ext.begin(), G.ext.end());
        std::vector<int32_t> sord = morton_order(sp.data(), c->nS, G.bbox_lo);
        c->S.set(sp, sord, st);
        // weight CSR rows in internal source order (Sec. 3.2 double layer, collected per source)
        std::vector<std::vector<std::pair<int32_t, double>>> rows(c->nS);
        for (int64_t q = 0; q < c->ngm; ++q) rows[q].push_back({(int32_t)q, (double)G.dcount[q]});
        for (size_t e = 0; e < G.edge_q.size(); ++e) rows[c->ngm + G.edge_k[e]].push_back({G.edge_q[e], -1.0});
        std::vector<int32_t> rowptr(c->nS + 1, 0), col;
        std::vector<double> coef;
        for (int64_t i = 0; i < c->nS; ++i) {
            for (auto& pr : rows[sord[i]]) {
                col.push_back(pr.first);
                coef.push_back(pr.second);
            }
            rowptr[i + 1] = (int32_t)col.size();
        }
        upload(c->csr_rowptr, rowptr, st);
        upload(c->csr_col, col, st);
        upload(c->csr_coef, coef, st);
        c->B = CSR{c->nS, c->S.ps.padded, c->csr_rowptr.as<int32_t>(), c->csr_col.as<int32_t>(),
                   c->csr_coef.as<double>()};
        {
            // single layer (Sec. 3.4): the same sources, weight q(n) on gamma-, none on E
            std::vector<int32_t> rp1(c->nS + 1, 0), col1;
            std::vector<double> coef1;
            for (int64_t i = 0; i < c->nS; ++i) {
                if (sord[i] < c->ngm) {
                    col1.push_back(sord[i]);
                    coef1.push_back(1.0);
                }
                rp1[i + 1] = (int32_t)col1.size();
            }
            upload(c->csr1_rowptr, rp1, st);
            upload(c->csr1_col, col1, st);
            upload(c->csr1_coef, coef1, st);
            c->B1 = CSR{c->nS, c->S.ps.padded, c->csr1_rowptr.as<int32_t>(), c->csr1_col.as<int32_t>(),
                        c->csr1_coef.as<double>()};
        }
        // closure rows
        std::vector<int32_t> ctq(c->ngm), ctp(c->ngm);
        for (int64_t q = 0; q < c->ngm; ++q) {
            ctq[q] = tinv[c->ngp + q];
            ctp[q] = tinv[G.partner[q]];
        }
        upload(c->cl_tq, ctq, st);
        upload(c->cl_tp, ctp, st);
        upload(c->cl_t, G.t, st);
        upload(c->partner_dev, G.partner, st);
        c->cl = Closure{c->ngm, c->cl_tq.as<int32_t>(), c->cl_tp.as<int32_t>(), c->cl_t.as<double>()};

        // LGF table: for sigma = 0 one table of the FP32 LDS radius shared by all contexts
        // (the far field takes over beyond it), else every offset that occurs.  The LDS
        // prefix covers the offsets that occur, but at least the far-field gap, beyond which
        // the expansion is accurate.
        const int R = c->s == 0.0 ? kLdsRadiusFar32 : std::max(G.max_offset, 1);
        c->table = get_table(c->device, c->s, R, st);
        c->tabs.near64 = c->table->d64.as<double>();
        c->tabs.near32 = c->table->d32.as<float>();
        c->tabs.full64 = c->table->d64.as<double>();
        c->tabs.full32 = c->table->d32.as<float>();
        c->tabs.full_r = c->table->R;
        const int need = std::max(G.max_offset, kFarGap);
        const bool far = c->s == 0.0;
        c->tabs.tab_r64 = std::min({far ? kLdsRadiusFar64 : kLdsRadius64, c->tabs.full_r, need});
        c->tabs.tab_r32 = std::min({far ? kLdsRadiusFar32 : kLdsRadius32, c->tabs.full_r, need});
        c->tabs.far_field = c->s == 0.0;
        // sigma > 0: the FP32 sum may use the Yukawa-form far field beyond the LDS radius, but
        // only where it matches this context's own exact table everywhere (FP64 keeps the table)
        c->tabs.kappa = std::sqrt(c->s);
        if (!far && c->tabs.full_r > c->tabs.tab_r32) {
            c->tabs.yukawa_err = yukawa_check(c->table->d64.as<double>(), c->tabs.full_r, c->tabs.tab_r32,
                                              c->tabs.kappa, st);
            c->tabs.yukawa32 = c->tabs.yukawa_err <= kYukawaTolerance;
        }
        c->sum_grid = lgf_sum_grid(c->device);
        BAE_HIP_CHECK(hipHostMalloc((void**)&c->pinned_flags, sizeof(int32_t) * (2 * c->max_rhs + 2),
                                    hipHostMallocMapped | hipHostMallocCoherent));
        BAE_HIP_CHECK(hipHostGetDevicePointer((void**)&c->flags_dev, c->pinned_flags, 0));
        std::memset(c->pinned_flags, 0, sizeof(int32_t) * (2 * c->max_rhs + 2));
        c->err_host = c->pinned_flags + 2 * c->max_rhs;
        c->err_dev = c->flags_dev + 2 * c->max_rhs;
        c->bad_host = c->pinned_flags + 2 * c->max_rhs + 1;
        c->bad_dev = c->flags_dev + 2 * c->max_rhs + 1;
        BAE_HIP_CHECK(hipEventCreateWithFlags(&c->rhs_ev, hipEventDisableTiming));
        c->wait_polls = c->opt.sum_wait_polls > 0 ? (uint32_t)c->opt.sum_wait_polls
                        : c->opt.sum_wait_polls < 0 ? 0u : kWaitPolls;
        c->plan.build(c->T.ps, c->S.ps, c->tabs, c->err_dev, c->wait_polls, st);

        // work buffers
        const int mr = c->max_rhs;
        c->w.alloc(sizeof(double) * c->S.ps.padded * mr);
        c->part_cap = (int64_t)c->plan.plan.chunks * c->nT * mr;
        c->part.alloc(sizeof(double) * c->part_cap);
        const int64_t n = c->ngm;
        KrylovState& K = c->K;
        K.m = m;
        K.n = n;
        K.ld_rhs = (int64_t)(m + 1) * n;
        c->kV.alloc(sizeof(double) * K.ld_rhs * mr);
        c->kH.alloc(sizeof(double) * (int64_t)m * (m + 1) * mr);
        c->kcs.alloc(sizeof(double) * m * mr);
        c->ksn.alloc(sizeof(double) * m * mr);
        c->kg.alloc(sizeof(double) * (m + 1) * mr);
        c->khist.alloc(sizeof(double) * m * mr);
        c->kbeta.alloc(sizeof(double) * mr);
        c->kdone.alloc(sizeof(int32_t) * mr);
        c->kkdone.alloc(sizeof(int32_t) * mr);
        K.V = c->kV.as<double>();
        K.H = c->kH.as<double>();
        K.cs = c->kcs.as<double>();
        K.sn = c->ksn.as<double>();
        K.g = c->kg.as<double>();
        K.hist = c->khist.as<double>();
        K.beta = c->kbeta.as<double>();
        K.done = c->kdone.as<int32_t>();
        K.kdone = c->kkdone.as<int32_t>();
        c->maxj = m + 1;
        c->vec_cap = n;
        use_double_layer(c.get());
        c->hA.alloc(sizeof(double) * c->maxj * mr);
        c->hB.alloc(sizeof(double) * c->maxj * mr);
        c->nrm.alloc(sizeof(double) * c->maxj * mr);
        c->dotpart.alloc(sizeof(double) * mr * (2 * (int64_t)c->maxj * dot_blocks(n) + norm_blocks(n)));
        c->ycoef.alloc(sizeof(double) * m * mr);
        for (DevMem* d : {&c->b, &c->x, &c->r, &c->tmp}) d->alloc(sizeof(double) * n * mr);
        c->up_gamma.alloc(sizeof(double) * c->nT * mr);
        c->gdev.alloc(sizeof(double) * n * mr);
        c->u_gamma.alloc(sizeof(double) * c->nT * mr);
        c->vsum.alloc(sizeof(double) * c->nT * mr);
        // batched / served solves: idle until started (done = 1, k = 0)
        c->ctl.alloc(sizeof(Ctl));
        const Ctl idle{0, 0, 0.0};
        BAE_HIP_CHECK(hipMemcpyAsync(c->ctl.p, &idle, sizeof(Ctl), hipMemcpyHostToDevice, st));
        launch_fill_int(K.done, mr, 1, st);
        launch_fill_int(K.kdone, mr, 0, st);
        BAE_HIP_CHECK(hipStreamSynchronize(st));
        return c.release();
}


void classify_pairs(const bae_ctx* c, bool fp32, int tab_r, bool far_ok, int far_gap, int64_t* cnt) {
    const PointSet& T = c->T.ps;
    const PointSet& S = c->S.ps;
    const int64_t nt = T.count, ns = S.count, nblk = S.nblk;
    // the kernels' classification, per (wavefront of 64 targets, source block)
    for (int64_t w0 = 0; w0 < nt; w0 += 64) {
        const int64_t w1 = std::min(nt, w0 + 64);
        int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {0, 0, 0};
        for (int64_t i = w0; i < w0 + 64; ++i) {
            const int64_t t = std::min(i, nt - 1);
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], T.hq[3 * t + a]);
                hi[a] = std::max(hi[a], T.hq[3 * t + a]);
            }
        }
        for (int64_t b = 0; b < nblk; ++b) {
            const int32_t* bb = &S.hbox[6 * b];
            int gap = 0, span = 0;
            for (int a = 0; a < 3; ++a) {
                gap = std::max(gap, std::max(bb[a] - hi[a], lo[a] - bb[3 + a]));
                span = std::max(span, std::max(bb[3 + a] - lo[a], hi[a] - bb[a]));
            }
            const int64_t s0 = b * kSourceBlock, s1 = std::min(ns, s0 + kSourceBlock);
            const int64_t pairs = (w1 - w0) * (s1 - s0);
            switch (block_class(gap, span, tab_r, far_ok, fp32, far_gap)) {
                case kClassTable: cnt[0] += pairs; break;
                case kClassFar: case kClassGather: cnt[1] += pairs; break;
                case kClassFar2: cnt[2] += pairs; break;
                default:
                    for (int64_t t = w0; t < w1; ++t)
                        for (int64_t s = s0; s < s1; ++s) {
                            int m = 0;
                            for (int a = 0; a < 3; ++a) m = std::max(m, std::abs(T.hq[3 * t + a] - S.hq[3 * s + a]));
                            cnt[m <= kQuant * tab_r ? 3 : 4]++;
                        }
            }
        }
    }
}

// Device bytes create_context will allocate for this geometry (admission control).
int64_t estimate_context_bytes(const Geometry& G, double s, const bae_options* opt) {
    const int mr = opt && opt->max_rhs > 0 ? opt->max_rhs : 16;
    const int m = opt && opt->max_krylov > 0 ? opt->max_krylov : 400;
    const int64_t ngp = (int64_t)G.gp.size() / 3, ngm = (int64_t)G.gm.size() / 3, next = (int64_t)G.ext.size() / 3;
    const int64_t nT = ngp + ngm, nS = ngm + next;
    auto padded = [](int64_t n) { return ((n + kSourceBlock - 1) / kSourceBlock) * kSourceBlock; };
    int64_t b = 0;
    b += (padded(nT) + padded(nS)) * (3 * 4 + 3 * 4 + 3 * 8 + 4 + 4);                   // point sets
    b += (padded(nT) / kSourceBlock + padded(nS) / kSourceBlock) * 6 * 4;              // block boxes
    b += nT * 4 + (nS + 1) * 4 + (ngm + (int64_t)G.edge_q.size()) * 12 + ngm * 16;    // maps, CSR, closure
    b += padded(nS) * 8 * mr;                                                          // weights
    b += (int64_t)lgf_sum_chunks(nT, (nS + kSourceBlock - 1) / kSourceBlock) * nT * mr * 8;   // partial sums
    b += ((nT + 63) / 64) * kMaxChunks * 4;                                               // work list
    b += nT * mr * 8;                                                                     // reduced sums
    b += ((int64_t)(m + 1) * ngm + (int64_t)m * (m + 1) + 4 * m + 8) * 8 * mr;        // Krylov state
    b += (int64_t)(m + 1) * mr * 8 * (3 + 2 * dot_blocks(ngm)) + (int64_t)m * mr * 8;  // CGS, dot slices, y
    b += (int64_t)norm_blocks(ngm) * mr * 8;                                           // norm slices
    b += 4 * ngm * mr * 8 + 2 * nT * mr * 8;                                           // b, x, r, tmp, u_p, u_gamma
    const int64_t pr = std::min<int64_t>(kRecycleDefault, m);
    b += (2 * ngm + (int64_t)m * dot_blocks(ngm)) * pr * mr * 8;                      // refined solves' recycling
    if (s > 0.0) b += table_size(std::max(32, G.max_offset)) * 12;                     // its own table
    return b;
}

}  // namespace bae

// ================================================================== C ABI
extern "C" {

const char* bae_status_string(int s) {
    switch (s) {
        case BAE_OK: return "ok";
        case BAE_NOT_CONVERGED: return "GMRES did not reach the tolerance";
        case BAE_ERR_ARG: return "invalid argument";
        case BAE_ERR_GEOMETRY: return "invalid geometry";
        case BAE_ERR_NONFINITE: return "non-finite input";
        case BAE_ERR_OOM: return "out of memory";
        case BAE_ERR_HIP: return "HIP runtime error";
        case BAE_ERR_STATE: return "call out of order";
        case BAE_ERR_ADMISSION: return "request exceeds the memory budget";
    }
    return "unknown status";
}

const char* bae_last_error(void) { return g_last_error.c_str(); }

int64_t bae_lgf_table_size(int32_t R) { return R < 0 ? 0 : table_size(R); }

int bae_lgf_table(double s, int32_t R, double* out_dev, void* stream) {
    return guard([&] {
        if (!out_dev || R < 0 || R > 4096 || !(s >= 0.0) || !std::isfinite(s)) throw Error{BAE_ERR_ARG, "bae_lgf_table: bad argument"};
        lgf_table_generate(s, R, out_dev, (hipStream_t)stream);
    });
}

int bae_lgf_table_noalloc(double s, int32_t R, double* out_dev, void* stream) {
    return guard([&] {
        if (!out_dev || R < 0 || !(s >= 0.0) || !std::isfinite(s))
            throw Error{BAE_ERR_ARG, "bae_lgf_table_noalloc: bad argument"};
        lgf_table_generate_noalloc(s, R, out_dev, (hipStream_t)stream);
    });
}

int bae_create(const bae_grid* grid, const bae_levelset* ls, const bae_options* opt, bae_ctx** out) {
    return guard([&] {
        if (!grid || !ls || !out) throw Error{BAE_ERR_ARG, "bae_create: null argument"};
        *out = nullptr;
        Geometry geo;
        build_geometry(*grid, *ls, geo);
        *out = create_context(*grid, opt, std::move(geo));
    });
}

int bae_destroy(bae_ctx* c) {
    if (!c) return BAE_OK;
    join_job(c);
    (void)hipSetDevice(c->device);
    if (c->rhs_ev) (void)hipEventDestroy(c->rhs_ev);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->pinned_flags) (void)hipHostFree(c->pinned_flags);
    hipStream_t st = c->stream;
    delete c;
    if (st) (void)hipStreamDestroy(st);
    return BAE_OK;
}

int bae_get_sizes(const bae_ctx* c, bae_sizes* o) {
    return guard([&] {
        if (!c || !o) throw Error{BAE_ERR_ARG, "null argument"};
        o->n_mplus = c->geo.n_mplus;
        o->n_gamma_plus = c->ngp;
        o->n_gamma_minus = c->ngm;
        o->n_ext = c->next;
        o->n_edges = (int64_t)c->geo.edge_q.size();
        o->n_sources = c->nS;
        o->n_targets = c->nT;
        o->n_empty_d = c->geo.n_empty_d;
        o->max_offset = c->geo.max_offset;
        o->table_radius = c->tabs.full_r;
        o->table_entries = table_size(c->tabs.full_r);
        o->lds_radius_fp32 = c->tabs.tab_r32;
        o->lds_radius_fp64 = c->tabs.tab_r64;
        o->far_field_fp32 = c->tabs.far32() ? 1 : 0;
        o->far_field_fp64 = c->tabs.far64() ? 1 : 0;
        o->far_field_err_fp32 = c->tabs.yukawa_err;
        size_t bytes = 0;
        for (const DevMem* d : {&c->T.x, &c->T.y, &c->T.z, &c->S.x, &c->S.y, &c->S.z, &c->Mp.x, &c->Mp.y, &c->Mp.z,
                                &c->T.xf, &c->T.yf, &c->T.zf, &c->S.xf, &c->S.yf, &c->S.zf, &c->Mp.xf, &c->Mp.yf,
                                &c->Mp.zf, &c->T.xd, &c->T.yd, &c->T.zd, &c->S.xd, &c->S.yd, &c->S.zd, &c->Mp.xd,
                                &c->Mp.yd, &c->Mp.zd, &c->T.xy16, &c->T.zl, &c->S.xy16, &c->S.zl, &c->Mp.xy16,
                                &c->Mp.zl, &c->T.bbox, &c->S.bbox, &c->Mp.bbox,
                                &c->t_pos, &c->csr_rowptr, &c->csr_col, &c->csr_coef, &c->cl_tq, &c->cl_tp, &c->cl_t,
                                &c->w, &c->part, &c->kV, &c->kH, &c->kcs, &c->ksn, &c->kg, &c->khist, &c->kbeta,
                                &c->kdone, &c->kkdone, &c->hA, &c->hB, &c->nrm, &c->dotpart, &c->ycoef, &c->b, &c->x,
                                &c->r, &c->tmp, &c->up_gamma, &c->u_gamma, &c->vsum, &c->wf, &c->plan.items,
                                &c->plan.counter})
            bytes += d->bytes;
        for (int a = 0; a < 3; ++a) {
            o->conv_box[a] = c->conv ? c->conv->e[a] : 0;
            o->conv_fft[a] = c->conv ? c->conv->M[a] : 0;
        }
        if (c->conv) bytes += (size_t)c->conv->bytes;
        o->device_bytes = (int64_t)bytes;
    });
}

int bae_get_sets(const bae_ctx* c, int32_t* gp, int32_t* gm, int32_t* ext) {
    return guard([&] {
        if (!c) throw Error{BAE_ERR_ARG, "null context"};
        if (gp) std::memcpy(gp, c->geo.gp.data(), sizeof(int32_t) * c->geo.gp.size());
        if (gm) std::memcpy(gm, c->geo.gm.data(), sizeof(int32_t) * c->geo.gm.size());
        if (ext) std::memcpy(ext, c->geo.ext.data(), sizeof(int32_t) * c->geo.ext.size());
    });
}

int bae_get_boundary_points(const bae_ctx* c, double* xstar, int32_t* partner, double* t) {
    return guard([&] {
        if (!c) throw Error{BAE_ERR_ARG, "null context"};
        if (xstar) std::memcpy(xstar, c->geo.xstar.data(), sizeof(double) * c->geo.xstar.size());
        if (partner) std::memcpy(partner, c->geo.partner.data(), sizeof(int32_t) * c->geo.partner.size());
        if (t) std::memcpy(t, c->geo.t.data(), sizeof(double) * c->geo.t.size());
    });
}

// ------------------------------------------------------------------ right-hand side
// Lazy per-context device maps: the linear grid index of every M+ point (internal Mp order)
// and of every gamma- node (lexicographic).
static void ensure_lin(bae_ctx* c) {
    ensure_mplus(c);
    const Geometry& G = c->geo;
    const int64_t nm = c->Mp.ps.count;
    if ((int64_t)c->mp_lin.size() == nm && c->gm_lin_dev.p) return;
    std::vector<int32_t> pts;
    pts.reserve(nm);
    for (int i = 0; i < G.n[0]; ++i)
        for (int j = 0; j < G.n[1]; ++j)
            for (int k = 0; k < G.n[2]; ++k)
                if (G.inside[((int64_t)i * G.n[1] + j) * G.n[2] + k])
                    pts.push_back((int32_t)(((int64_t)i * G.n[1] + j) * G.n[2] + k));
    c->mp_lin.resize(nm);
    for (int64_t a = 0; a < nm; ++a) c->mp_lin[a] = pts[c->Mp.perm[a]];
    std::vector<int32_t> gl(c->ngm);
    for (int64_t q = 0; q < c->ngm; ++q) {
        const int32_t* v = &G.gm[3 * q];
        gl[q] = (int32_t)(((int64_t)v[0] * G.n[1] + v[1]) * G.n[2] + v[2]);
    }
    upload(c->mp_lin_dev, c->mp_lin, c->stream);
    upload(c->gm_lin_dev, gl, c->stream);
    BAE_HIP_CHECK(hipStreamSynchronize(c->stream));
}

// Lazy set-up of the box of Algorithm 1 (its interior nodes n_d - 2 per axis): the interior
// index of every target and of every M+ point, and the M+ mask on the device.
static void ensure_box(bae_ctx* c) {
    if (c->box_ready) return;
    ensure_lin(c);
    const Geometry& G = c->geo;
    hipStream_t st = c->stream;
    for (int a = 0; a < 3; ++a) c->box_n[a] = G.n[a] - 2;
    const int N1 = c->box_n[1], N2 = c->box_n[2];
    c->box_nn = (int64_t)c->box_n[0] * N1 * N2;
    const int64_t nm = c->Mp.ps.count;
    auto interior = [&](int64_t i, int64_t j, int64_t k) { return (int32_t)(((i - 1) * N1 + (j - 1)) * N2 + (k - 1)); };
    std::vector<int32_t> tidx(c->nT), midx(nm);
    for (int64_t t = 0; t < c->nT; ++t) {
        const int32_t* v = t < c->ngp ? &G.gp[3 * t] : &G.gm[3 * (t - c->ngp)];
        tidx[t] = interior(v[0], v[1], v[2]);
    }
    for (int64_t a = 0; a < nm; ++a) {
        const int64_t l = c->mp_lin[a];
        midx[a] = interior(l / ((int64_t)G.n[1] * G.n[2]), (l / G.n[2]) % G.n[1], l % G.n[2]);
    }
    upload(c->box_tidx, tidx, st);
    upload(c->box_mpidx, midx, st);
    upload(c->inside_dev, G.inside, st);
    BAE_HIP_CHECK(hipStreamSynchronize(st));   // tidx, midx leave scope
    c->box_ready = true;
}

// The device part of the right-hand side, on stream st: with f (h^2 f at the M+ points
// already in c->wf, [nrhs][Mp padded]) the particular solution u_p on gamma -- the free-space
// volume potential (the LGF sum over the M+ sources as an FFT convolution) or, with `box`,
// Algorithm 1's finite-grid
// G_h[chi_{M+} f] (box.hip) -- then b = g - Phi u_p (Sec. 3.4) from g (device, [nrhs][ngm]).
static void rhs_on_device(bae_ctx* c, int nrhs, const double* g, int64_t ldg, bool has_f, bool box, hipStream_t st) {
    const int64_t nmp = c->Mp.ps.padded;
    if (has_f && box) {
        const int64_t nn = c->box_nn, nm = c->Mp.ps.count;
        launch_fill(c->box_u.as<double>(), nn * nrhs, 0.0, st);
        launch_scatter(c->wf.as<double>(), nmp, c->box_mpidx.as<int32_t>(), nm, c->box_u.as<double>(), nn, nrhs, st);
        for (int r = 0; r < nrhs; ++r)
            box_solve_fft(c->box_u.as<double>() + r * nn, c->box_n[0], c->box_n[1], c->box_n[2], c->s, st);
        launch_gather(c->box_u.as<double>(), nn, c->box_tidx.as<int32_t>(), c->nT, c->up_gamma.as<double>(), c->nT,
                      nrhs, 1.0, st);
    } else if (has_f) {
        // the free-space volume potential h^2 sum_{M+} G(m - n) f(n) on gamma, by the FFT
        // convolution (FP64), in internal target order, then into [gamma+; gamma-] order
        for (int r = 0; r < nrhs; ++r)
            c->conv->apply(c->wf.as<double>() + r * nmp, c->conv_midx.as<int32_t>(), c->Mp.ps.count,
                           c->conv_tidx.as<int32_t>(), c->nT, c->vsum.as<double>() + r * c->nT, 1.0, nullptr, st);
        launch_reduce_scatter(c->vsum.as<double>(), 1, c->nT, c->t_pos.as<int32_t>(), c->up_gamma.as<double>(), c->nT,
                              nrhs, 1.0, st);
    } else {
        launch_fill(c->up_gamma.as<double>(), c->nT * nrhs, 0.0, st);
    }
    launch_rhs(g, ldg, has_f ? c->up_gamma.as<double>() : nullptr, c->nT, c->partner_dev.as<int32_t>(),
               c->cl_t.as<double>(), c->ngp, c->ngm, c->b.as<double>(), c->ngm, nrhs, c->bad_dev, st);
    BAE_HIP_CHECK(hipEventRecord(c->rhs_ev, st));
    c->nrhs = nrhs;
    c->has_f = has_f;
    c->particular_box = has_f && box;
    c->rhs_ready = true;
    c->solved = false;
    c->has_grid = false;
}

static void check_rhs_args(bae_ctx* c, int32_t nrhs, const void* g, const void* f, bool box) {
    (void)f;
    (void)box;
    if (!c || !g) throw Error{BAE_ERR_ARG, "null argument"};
    if (nrhs < 1 || nrhs > c->max_rhs) throw Error{BAE_ERR_ARG, "nrhs out of range"};
}

// Host inputs: validated here, h^2 f gathered at the M+ points on the host (only those cross
// the bus), g staged on the device, then the device part on the context's stream.
static void set_rhs_impl(bae_ctx* c, int32_t nrhs, const double* g_xstar, const double* f_grid, bool box) {
    check_rhs_args(c, nrhs, g_xstar, f_grid, box);
    join_job(c);
    BAE_HIP_CHECK(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    const Geometry& G = c->geo;
    const int64_t n = c->ngm, N3 = (int64_t)G.n[0] * G.n[1] * G.n[2];
    for (int64_t i = 0; i < n * nrhs; ++i)
        if (!std::isfinite(g_xstar[i])) throw Error{BAE_ERR_NONFINITE, "boundary data not finite"};
    if (f_grid) {
        for (int64_t i = 0; i < N3 * nrhs; ++i)
            if (!std::isfinite(f_grid[i])) throw Error{BAE_ERR_NONFINITE, "source term not finite"};
        ensure_lin(c);
        if (box) ensure_box(c);
        else ensure_conv(c, true);
        const int64_t nm = c->Mp.ps.count, nmp = c->Mp.ps.padded;
        std::vector<double> wfh(nmp * nrhs, 0.0);
        const double h2 = G.h * G.h;
        for (int r = 0; r < nrhs; ++r)
            for (int64_t a = 0; a < nm; ++a) wfh[r * nmp + a] = h2 * f_grid[r * N3 + c->mp_lin[a]];
        if (c->wf.bytes < sizeof(double) * wfh.size()) c->wf.alloc(sizeof(double) * nmp * c->max_rhs);
        BAE_HIP_CHECK(hipMemcpyAsync(c->wf.p, wfh.data(), sizeof(double) * wfh.size(), hipMemcpyHostToDevice, st));
        if (box && c->box_u.bytes < sizeof(double) * c->box_nn * nrhs)
            c->box_u.alloc(sizeof(double) * c->box_nn * c->max_rhs);
        BAE_HIP_CHECK(hipStreamSynchronize(st));   // wfh leaves scope
    }
    BAE_HIP_CHECK(hipMemcpyAsync(c->gdev.p, g_xstar, sizeof(double) * n * nrhs, hipMemcpyHostToDevice, st));
    rhs_on_device(c, nrhs, c->gdev.as<double>(), n, f_grid != nullptr, box, st);
    BAE_HIP_CHECK(hipStreamSynchronize(st));
}

// Device inputs, on the caller's stream: nothing is read back, so non-finite values are
// flagged on the device and reported by the next solve.
static void set_rhs_device_impl(bae_ctx* c, int32_t nrhs, const double* g_dev, const double* f_dev, int32_t particular,
                                hipStream_t st) {
    if (particular != BAE_PARTICULAR_FREE && particular != BAE_PARTICULAR_BOX)
        throw Error{BAE_ERR_ARG, "unknown particular-solution kind"};
    const bool box = particular == BAE_PARTICULAR_BOX;
    check_rhs_args(c, nrhs, g_dev, f_dev, box);
    join_job(c);
    BAE_HIP_CHECK(hipSetDevice(c->device));
    if (f_dev) {
        // one-time set-up (host work and uploads on the context's stream) before any of the
        // caller's work is touched
        ensure_lin(c);
        if (box) ensure_box(c);
        else ensure_conv(c, true);
        const int64_t nmp = c->Mp.ps.padded;
        if (c->wf.bytes < sizeof(double) * nmp * nrhs) c->wf.alloc(sizeof(double) * nmp * c->max_rhs);
        if (box && c->box_u.bytes < sizeof(double) * c->box_nn * nrhs)
            c->box_u.alloc(sizeof(double) * c->box_nn * c->max_rhs);
        const Geometry& G = c->geo;
        const int64_t N3 = (int64_t)G.n[0] * G.n[1] * G.n[2];
        launch_finite_check(f_dev, N3, N3, nrhs, c->bad_dev, st);
        launch_fill(c->wf.as<double>(), nmp * nrhs, 0.0, st);
        launch_gather(f_dev, N3, c->mp_lin_dev.as<int32_t>(), c->Mp.ps.count, c->wf.as<double>(), nmp, nrhs,
                      G.h * G.h, st);
    }
    rhs_on_device(c, nrhs, g_dev, c->ngm, f_dev != nullptr, box, st);
}

// u on the grid (Algorithm 1's last step; Sec. 2.1 eq. "discrete_green_v"): the part of u_gamma
// beyond the particular solution, h_gamma = u_gamma - u_p, is lattice harmonic in M+, so its
// difference potential G_h[chi_{M-} L_h h_gamma] (h_gamma extended by zero off gamma; G_h by the
// box's sine transforms) reproduces it there, and u = u_p + G_h[chi_{M-} L_h h_gamma] on M+,
// u_gamma on gamma-, NaN elsewhere; assembled on the device in c->ugrid ([nrhs][n0 n1 n2]).
// u_p on M+ is the box solve's own (bae_set_rhs_box), the free-space volume potential (an LGF
// sum over the M+ sources at the M+ targets), or zero without f.
static void grid_solution(bae_ctx* c, int nrhs, hipStream_t st) {
    const Geometry& G = c->geo;
    ensure_box(c);
    const int64_t nm = c->Mp.ps.count, nn = c->box_nn;
    const int64_t N3 = (int64_t)G.n[0] * G.n[1] * G.n[2];
    if (c->box_h.bytes < sizeof(double) * nn) c->box_h.alloc(sizeof(double) * nn);
    if (c->box_w.bytes < sizeof(double) * nn) c->box_w.alloc(sizeof(double) * nn);
    DevMem hg, um;
    hg.alloc(sizeof(double) * c->nT * nrhs);
    um.alloc(sizeof(double) * nm * nrhs);
    // h_gamma = u_gamma - u_p on gamma
    BAE_HIP_CHECK(hipMemcpyAsync(hg.p, c->u_gamma.p, sizeof(double) * c->nT * nrhs, hipMemcpyDeviceToDevice, st));
    launch_axpby(-1.0, c->up_gamma.as<double>(), c->nT, 1.0, hg.as<double>(), c->nT, c->nT, nrhs, st);
    for (int r = 0; r < nrhs; ++r) {
        launch_fill(c->box_h.as<double>(), nn, 0.0, st);
        launch_scatter(hg.as<double>() + r * c->nT, c->nT, c->box_tidx.as<int32_t>(), c->nT, c->box_h.as<double>(), nn, 1,
                    st);
        difference_source(c->box_h.as<double>(), c->inside_dev.as<uint8_t>(), G.n, c->s, c->box_w.as<double>(), st);
        box_solve_fft(c->box_w.as<double>(), c->box_n[0], c->box_n[1], c->box_n[2], c->s, st);
        launch_gather(c->box_w.as<double>(), nn, c->box_mpidx.as<int32_t>(), nm, um.as<double>() + r * nm, nm, 1, 1.0,
                      st);
    }
    if (c->has_f) {
        DevMem up;
        up.alloc(sizeof(double) * nm * nrhs);
        if (c->particular_box)   // the finite-grid u_p is known at every node
            launch_gather(c->box_u.as<double>(), nn, c->box_mpidx.as<int32_t>(), nm, up.as<double>(), nm, nrhs, 1.0, st);
        else   // the free-space volume potential at the M+ targets, by the FFT convolution
            for (int r = 0; r < nrhs; ++r)
                c->conv->apply(c->wf.as<double>() + r * c->Mp.ps.padded, c->conv_midx.as<int32_t>(), nm,
                               c->conv_midx.as<int32_t>(), nm, up.as<double>() + r * nm, 1.0, nullptr, st);
        launch_axpby(1.0, up.as<double>(), nm, 1.0, um.as<double>(), nm, nm, nrhs, st);
        BAE_HIP_CHECK(hipStreamSynchronize(st));   // up leaves scope
    }
    if (c->ugrid.bytes < sizeof(double) * N3 * nrhs) c->ugrid.alloc(sizeof(double) * N3 * nrhs);
    launch_fill(c->ugrid.as<double>(), N3 * nrhs, NAN, st);
    launch_scatter(um.as<double>(), nm, c->mp_lin_dev.as<int32_t>(), nm, c->ugrid.as<double>(), N3, nrhs, st);
    launch_scatter(c->u_gamma.as<double>() + c->ngp, c->nT, c->gm_lin_dev.as<int32_t>(), c->ngm, c->ugrid.as<double>(),
                   N3, nrhs, st);
    BAE_HIP_CHECK(hipStreamSynchronize(st));   // hg, um leave scope
}

// ------------------------------------------------------------------ solve
static void check_solve_args(const bae_ctx* c, const bae_solve_params* p) {
    if (!c || !p) throw Error{BAE_ERR_ARG, "null argument"};
    if (!c->rhs_ready) throw Error{BAE_ERR_STATE, "bae_set_rhs must precede bae_solve"};
    if (p->precision != BAE_SOLVE_FP64 && p->precision != BAE_SOLVE_FP32_REFINED && p->precision != BAE_SOLVE_FFT)
        throw Error{BAE_ERR_ARG, "unknown solve precision"};
    if (!(p->tol > 0.0)) throw Error{BAE_ERR_ARG, "tol must be > 0"};
    if (p->formulation != BAE_LAYER_DOUBLE && p->formulation != BAE_LAYER_SINGLE && p->formulation != BAE_LAYER_DIRECT)
        throw Error{BAE_ERR_ARG, "unknown formulation"};
}

// The solve of Algorithm 1 on the context's stream (which the caller has already ordered
// after its own work): GMRES (FP64, or FP64 refinement around FP32-sum GMRES) from x0 = 0 or
// the given densities, then u_gamma and, if asked, u on the grid.  Returns BAE_OK or
// BAE_NOT_CONVERGED; throws Error.
static int solve_impl(bae_ctx* c, const bae_solve_params* p, bae_result* res) {
    check_solve_args(c, p);
    BAE_HIP_CHECK(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    // the layer potential of this solve (Sec. 3.4): every operator call below, the grid
    // solution included, forms its source weights through this map
    const LayerScope layer(c, p->formulation);
    const auto t0 = std::chrono::steady_clock::now();
    const int nrhs = c->nrhs;
    const int64_t n = c->op.n;
    const int maxit = p->maxit > 0 ? std::min(p->maxit, c->K.m) : c->K.m;
    c->hist.assign(nrhs, {});
    c->solved = false;
    c->has_grid = false;
    int64_t mv64 = 0, mv32 = 0;
    BAE_HIP_CHECK(hipStreamWaitEvent(st, c->rhs_ev, 0));   // the right-hand side's device work
    if (c->op.direct) {   // the direct system's right-hand side [0; b] (Sec. 3.4, eq. "direct_sys")
        launch_fill(c->bdir.as<double>(), c->nT * nrhs, 0.0, st);
        BAE_HIP_CHECK(hipMemcpy2DAsync(c->bdir.as<double>() + c->ngp, sizeof(double) * c->nT, c->b.p,
                                       sizeof(double) * c->ngm, sizeof(double) * c->ngm, nrhs,
                                       hipMemcpyDeviceToDevice, st));
    }
    std::vector<double> bn = host_norms(c, rhs_vector(c), nrhs, st);
    if (__atomic_exchange_n(c->bad_host, 0, __ATOMIC_ACQ_REL))
        throw Error{BAE_ERR_NONFINITE, "boundary data or source term not finite"};
    std::vector<int> iters(nrhs, 0), conv(nrhs, 0), outer(nrhs, 0);
    std::vector<double> est(nrhs, 0.0), relres;
    bool dq_in_vsum = false;   // the last operator call was the FP64 residual of the final q
    const bool warm = p->x0_dev != nullptr;
    if (warm) {
        BAE_HIP_CHECK(hipMemcpyAsync(c->x.p, p->x0_dev, sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, st));
        launch_finite_check(c->x.as<double>(), n, n, nrhs, c->bad_dev, st);
    } else {
        launch_fill(c->x.as<double>(), n * nrhs, 0.0, st);
    }
    if (p->precision == BAE_SOLVE_FP64 || p->precision == BAE_SOLVE_FFT) {
        // FP64 GMRES with the FP64 sum or its FFT convolution for every matvec
        const int mprec = p->precision == BAE_SOLVE_FFT ? BAE_PREC_FFT : BAE_PREC_FP64;
        // from x0: GMRES on A d = b - A x0, x = x0 + d
        if (warm) {
            relres = residual(c, nrhs, bn, st, &mv64, mprec);
            if (__atomic_exchange_n(c->bad_host, 0, __ATOMIC_ACQ_REL))
                throw Error{BAE_ERR_NONFINITE, "initial densities not finite"};
        }
        std::vector<int> skip;
        bool all = false;
        if (warm) {
            skip.assign(nrhs, 0);
            all = true;
            for (int r = 0; r < nrhs; ++r) {
                skip[r] = relres[r] <= p->tol;
                all &= skip[r] != 0;
            }
            dq_in_vsum = true;
        }
        if (!all) {   // (a warm start that already meets tol needs no iteration)
            GmresOut g = gmres(c, warm ? c->r.as<double>() : rhs_vector(c), nrhs, mprec, p->tol, maxit, skip,
                               c->x.as<double>(), warm, st, &mv64);
            for (int r = 0; r < nrhs; ++r) {
                iters[r] = g.iters[r];
                est[r] = g.last_est[r];
                conv[r] = g.converged[r];
            }
            relres = residual(c, nrhs, bn, st, &mv64, mprec);
            dq_in_vsum = true;
        }
        for (int r = 0; r < nrhs; ++r) conv[r] = conv[r] || relres[r] <= p->tol;
    } else {
        // inner tolerance of outer step k: just enough to reach tol from the current
        // residual, but never below the floor where the FP32 operator's own error (~1e-6
        // relative) makes further inner iterations useless
        const double floor_tol = p->inner_tol > 0 ? p->inner_tol : 1e-6;
        const int max_outer = p->max_outer > 0 ? p->max_outer : 8;
        // recycling costs a few host round trips per outer step: worth it once a matvec
        // is long (1e8 pair interactions, ~50 us), not for the smallest problems
        const bool long_matvec = (double)c->nT * (double)c->nS * nrhs >= 1e8;
        const int recycle_cap = p->recycle_dim < 0   ? 0
                                : p->recycle_dim > 0 ? p->recycle_dim
                                                     : (long_matvec ? kRecycleDefault : 0);
        Recycle rc;
        if (warm) {
            relres = residual(c, nrhs, bn, st, &mv64);   // r = b - A64 x0
            if (__atomic_exchange_n(c->bad_host, 0, __ATOMIC_ACQ_REL))
                throw Error{BAE_ERR_NONFINITE, "initial densities not finite"};
            dq_in_vsum = true;
        } else {
            BAE_HIP_CHECK(hipMemcpyAsync(c->r.p, rhs_vector(c), sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, st));
            relres.assign(nrhs, 1.0);
            for (int r = 0; r < nrhs; ++r) relres[r] = bn[r] > 0 ? 1.0 : 0.0;
        }
        for (int o = 0; o < max_outer; ++o) {
            std::vector<int> skip(nrhs, 0);
            bool all = true;
            double worst = 0.0;
            for (int r = 0; r < nrhs; ++r) {
                skip[r] = relres[r] <= p->tol;
                all &= skip[r] != 0;
                if (!skip[r]) worst = std::max(worst, relres[r]);
            }
            if (all) break;
            const double inner = std::min(0.1, std::max(floor_tol, 0.5 * p->tol / worst));
            // with a recycled space: its part of the residual first, then GMRES on the
            // rest to the same absolute target (tolerance relative to what is left)
            double gtol = inner;
            std::vector<double> rscale(relres);
            if (rc.p > 0) {
                recycle_project(c, rc, nrhs, skip, c->x.as<double>(), c->r.as<double>(), st);
                const std::vector<double> rn = host_norms(c, c->r.as<double>(), nrhs, st);
                double ratio = 1e300;
                for (int r = 0; r < nrhs; ++r) {
                    if (skip[r]) continue;
                    rscale[r] = bn[r] > 0 ? rn[r] / bn[r] : 0.0;
                    if (rn[r] > 0) ratio = std::min(ratio, relres[r] * bn[r] / rn[r]);
                }
                gtol = ratio < 1e300 ? std::min(0.5, inner * ratio) : inner;
            } else {
                for (int r = 0; r < nrhs; ++r) rscale[r] = relres[r];
            }
            GmresOut g = gmres(c, c->r.as<double>(), nrhs, BAE_PREC_FP32, gtol, maxit, skip, c->x.as<double>(), true,
                               st, &mv32, rc.p > 0 ? &rc : nullptr);
            for (int r = 0; r < nrhs; ++r) {
                iters[r] += g.iters[r];
                if (!skip[r]) {
                    outer[r]++;
                    est[r] = g.last_est[r] * rscale[r];
                }
            }
            if (o == 0 && recycle_cap > 0) build_recycle(c, nrhs, skip, recycle_cap, rc, st);
            relres = residual(c, nrhs, bn, st, &mv64);
            dq_in_vsum = true;
        }
        for (int r = 0; r < nrhs; ++r) conv[r] = relres[r] <= p->tol;
    }
    // u_gamma = D q + u_p on gamma.  The last call above is the FP64 residual of the final
    // q, whose operator left D q at every target (internal order) in vsum: scattering it
    // saves a double-layer evaluation.
    // (the direct formulation's unknowns are v on gamma itself: u_gamma = v + u_p.)
    if (c->op.direct)
        BAE_HIP_CHECK(hipMemcpyAsync(c->u_gamma.p, c->x.p, sizeof(double) * c->nT * nrhs, hipMemcpyDeviceToDevice, st));
    else if (dq_in_vsum && c->cl.n > 0)
        launch_reduce_scatter(c->vsum.as<double>(), 1, c->nT, c->t_pos.as<int32_t>(), c->u_gamma.as<double>(), c->nT,
                              nrhs, 1.0, st);
    else
        double_layer(c, c->x.as<double>(), n, c->u_gamma.as<double>(), c->nT, nrhs, BAE_PREC_FP64, st);
    launch_axpby(1.0, c->up_gamma.as<double>(), c->nT, 1.0, c->u_gamma.as<double>(), c->nT, c->nT, nrhs, st);
    if (p->compute_grid) grid_solution(c, nrhs, st);
    BAE_HIP_CHECK(hipStreamSynchronize(st));
    check_sum_error(c);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int status = BAE_OK;
    for (int r = 0; r < nrhs; ++r) {
        if (!conv[r]) status = BAE_NOT_CONVERGED;
        if (res) {
            res[r].status = conv[r] ? BAE_OK : BAE_NOT_CONVERGED;
            res[r].iterations = iters[r];
            res[r].outer_steps = outer[r];
            res[r].converged = conv[r];
            res[r].rel_residual_est = est[r];
            res[r].rel_residual_true = relres[r];
            res[r].seconds = secs;
            res[r].matvecs_fp64 = mv64;
            res[r].matvecs_fp32 = mv32;
        }
    }
    c->solved = true;
    c->has_grid = p->compute_grid != 0;
    c->dens_n = n;
    return status;
}

int bae_set_rhs(bae_ctx* c, int32_t nrhs, const double* g_xstar, const double* f_grid) {
    return guard([&] { set_rhs_impl(c, nrhs, g_xstar, f_grid, false); });
}

int bae_set_rhs_box(bae_ctx* c, int32_t nrhs, const double* g_xstar, const double* f_grid) {
    return guard([&] { set_rhs_impl(c, nrhs, g_xstar, f_grid, true); });
}

int bae_set_rhs_device(bae_ctx* c, int32_t nrhs, const double* g_dev, const double* f_dev, int32_t particular,
                       void* stream) {
    return guard([&] { set_rhs_device_impl(c, nrhs, g_dev, f_dev, particular, (hipStream_t)stream); });
}

int bae_get_particular(const bae_ctx* cc, int32_t r, double* up_grid) {
    return guard([&] {
        if (!cc || !up_grid) throw Error{BAE_ERR_ARG, "null argument"};
        bae_ctx* c = const_cast<bae_ctx*>(cc);
        join_job(c);
        if (!c->particular_box) throw Error{BAE_ERR_STATE, "no box particular solution (bae_set_rhs_box with f)"};
        if (r < 0 || r >= c->nrhs) throw Error{BAE_ERR_ARG, "rhs index out of range"};
        BAE_HIP_CHECK(hipSetDevice(c->device));
        BAE_HIP_CHECK(hipStreamSynchronize(c->stream));
        const Geometry& G = c->geo;
        const int N0 = c->box_n[0], N1 = c->box_n[1], N2 = c->box_n[2];
        const int64_t nn = c->box_nn, N3 = (int64_t)G.n[0] * G.n[1] * G.n[2];
        std::vector<double> u(nn);
        BAE_HIP_CHECK(hipMemcpy(u.data(), c->box_u.as<double>() + r * nn, sizeof(double) * nn, hipMemcpyDeviceToHost));
        std::fill(up_grid, up_grid + N3, 0.0);
        for (int i = 1; i <= N0; ++i)
            for (int j = 1; j <= N1; ++j)
                for (int k = 1; k <= N2; ++k)
                    up_grid[((int64_t)i * G.n[1] + j) * G.n[2] + k] = u[((int64_t)(i - 1) * N1 + (j - 1)) * N2 + (k - 1)];
    });
}

// Orders the context's stream after the work queued on `stream` so far (no host wait).
static void order_after(bae_ctx* c, hipStream_t stream) {
    hipEvent_t ev;
    BAE_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) throw Error{BAE_ERR_HIP, std::string("ordering on the caller's stream: ") + hipGetErrorString(e)};
}

int bae_solve(bae_ctx* c, const bae_solve_params* p, bae_result* res) {
    int status = BAE_OK;
    int rc = guard([&] {
        check_solve_args(c, p);
        join_job(c);
        c->job.state.store(0);
        BAE_HIP_CHECK(hipSetDevice(c->device));
        if (p->x0_dev) order_after(c, nullptr);   // the initial densities, written on the null stream
        status = solve_impl(c, p, res);
    });
    return rc != BAE_OK ? rc : status;
}

int bae_solve_async(bae_ctx* c, const bae_solve_params* p, void* stream) {
    return guard([&] {
        check_solve_args(c, p);
        join_job(c);
        BAE_HIP_CHECK(hipSetDevice(c->device));
        order_after(c, (hipStream_t)stream);
        c->job.state.store(1);
        c->job.status = BAE_OK;
        c->job.error.clear();
        c->job.res.assign(c->nrhs, bae_result{});
        const bae_solve_params prm = *p;
        c->job.th = std::thread([c, prm] {
            int status = BAE_OK;
            const int rc = guard([&] { status = solve_impl(c, &prm, c->job.res.data()); });
            c->job.status = rc != BAE_OK ? rc : status;
            if (rc != BAE_OK) c->job.error = bae_last_error();
            c->job.state.store(2);
        });
    });
}

int bae_solve_poll(const bae_ctx* c, int32_t* done) {
    return guard([&] {
        if (!c || !done) throw Error{BAE_ERR_ARG, "null argument"};
        *done = c->job.state.load() != 1;
    });
}

int bae_solve_wait(bae_ctx* c, void* stream, bae_result* res) {
    int status = BAE_OK;
    int rc = guard([&] {
        if (!c) throw Error{BAE_ERR_ARG, "null argument"};
        if (c->job.state.load() == 0) throw Error{BAE_ERR_STATE, "no solve started by bae_solve_async"};
        join_job(c);
        c->job.state.store(0);
        if (res) std::copy(c->job.res.begin(), c->job.res.end(), res);
        if (c->job.status < 0) throw Error{c->job.status, c->job.error};
        status = c->job.status;
        // the caller's later work on `stream` sees every output of the solve
        BAE_HIP_CHECK(hipSetDevice(c->device));
        hipEvent_t ev;
        BAE_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        hipError_t e = hipEventRecord(ev, c->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent((hipStream_t)stream, ev, 0);
        (void)hipEventDestroy(ev);
        if (e != hipSuccess) throw Error{BAE_ERR_HIP, std::string("ordering the caller's stream: ") + hipGetErrorString(e)};
    });
    return rc != BAE_OK ? rc : status;
}

// Output r (or all RHS for r = -1) of length len per RHS from the device buffer src (row
// stride len) into dst: host (dev = false) or device memory on `stream`.
static void copy_out(bae_ctx* c, int32_t r, const double* src, int64_t len, double* dst, bool dev, hipStream_t stream) {
    if (r < -1 || r >= c->nrhs) throw Error{BAE_ERR_ARG, "rhs index out of range"};
    const double* from = r < 0 ? src : src + r * len;
    const int64_t count = r < 0 ? len * c->nrhs : len;
    BAE_HIP_CHECK(hipSetDevice(c->device));
    if (dev) {
        BAE_HIP_CHECK(hipMemcpyAsync(dst, from, sizeof(double) * count, hipMemcpyDeviceToDevice, stream));
    } else {
        BAE_HIP_CHECK(hipMemcpyAsync(dst, from, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
        BAE_HIP_CHECK(hipStreamSynchronize(c->stream));
    }
}

static bae_ctx* solved_ctx(const bae_ctx* cc) {
    if (!cc) throw Error{BAE_ERR_ARG, "null argument"};
    bae_ctx* c = const_cast<bae_ctx*>(cc);
    join_job(c);
    if (!c->solved) throw Error{BAE_ERR_STATE, "no solution (solve first)"};
    return c;
}

int bae_get_density(const bae_ctx* cc, int32_t r, double* q) {
    return guard([&] {
        bae_ctx* c = solved_ctx(cc);
        if (!q) throw Error{BAE_ERR_ARG, "null argument"};
        copy_out(c, r, c->x.as<double>(), c->dens_n, q, false, nullptr);
    });
}

int bae_get_density_length(const bae_ctx* cc, int64_t* len) {
    return guard([&] {
        bae_ctx* c = solved_ctx(cc);
        if (!len) throw Error{BAE_ERR_ARG, "null argument"};
        *len = c->dens_n;
    });
}

int bae_get_gamma_values(const bae_ctx* cc, int32_t r, double* u) {
    return guard([&] {
        bae_ctx* c = solved_ctx(cc);
        if (!u) throw Error{BAE_ERR_ARG, "null argument"};
        copy_out(c, r, c->u_gamma.as<double>(), c->nT, u, false, nullptr);
    });
}

int bae_get_solution(const bae_ctx* cc, int32_t r, double* u) {
    return guard([&] {
        bae_ctx* c = solved_ctx(cc);
        if (!u) throw Error{BAE_ERR_ARG, "null argument"};
        if (!c->has_grid) throw Error{BAE_ERR_STATE, "no grid solution (solve with compute_grid)"};
        const int64_t N3 = (int64_t)c->geo.n[0] * c->geo.n[1] * c->geo.n[2];
        copy_out(c, r, c->ugrid.as<double>(), N3, u, false, nullptr);
    });
}

int bae_get_density_device(const bae_ctx* cc, int32_t r, double* q_dev, void* stream) {
    return guard([&] {
        bae_ctx* c = solved_ctx(cc);
        if (!q_dev) throw Error{BAE_ERR_ARG, "null argument"};
        copy_out(c, r, c->x.as<double>(), c->dens_n, q_dev, true, (hipStream_t)stream);
    });
}

int bae_get_gamma_values_device(const bae_ctx* cc, int32_t r, double* u_dev, void* stream) {
    return guard([&] {
        bae_ctx* c = solved_ctx(cc);
        if (!u_dev) throw Error{BAE_ERR_ARG, "null argument"};
        copy_out(c, r, c->u_gamma.as<double>(), c->nT, u_dev, true, (hipStream_t)stream);
    });
}

int bae_get_solution_device(const bae_ctx* cc, int32_t r, double* u_dev, void* stream) {
    return guard([&] {
        bae_ctx* c = solved_ctx(cc);
        if (!u_dev) throw Error{BAE_ERR_ARG, "null argument"};
        if (!c->has_grid) throw Error{BAE_ERR_STATE, "no grid solution (solve with compute_grid)"};
        const int64_t N3 = (int64_t)c->geo.n[0] * c->geo.n[1] * c->geo.n[2];
        copy_out(c, r, c->ugrid.as<double>(), N3, u_dev, true, (hipStream_t)stream);
    });
}

int bae_get_history(const bae_ctx* cc, int32_t r, double* h, int32_t cap, int32_t* len) {
    return guard([&] {
        bae_ctx* c = solved_ctx(cc);
        if (!len) throw Error{BAE_ERR_ARG, "null argument"};
        if (r < 0 || r >= c->nrhs) throw Error{BAE_ERR_ARG, "rhs index out of range"};
        const auto& v = c->hist[r];
        *len = (int32_t)v.size();
        if (h) std::memcpy(h, v.data(), sizeof(double) * std::min<size_t>(v.size(), cap > 0 ? cap : 0));
    });
}

int bae_apply_double_layer(bae_ctx* c, const double* q, double* v, int32_t nrhs, int32_t prec, void* stream) {
    return guard([&] {
        if (!c || !q || !v) throw Error{BAE_ERR_ARG, "null argument"};
        if (nrhs < 1 || nrhs > c->max_rhs) throw Error{BAE_ERR_ARG, "nrhs out of range"};
        if (prec != BAE_PREC_FP64 && prec != BAE_PREC_FP32 && prec != BAE_PREC_FFT)
            throw Error{BAE_ERR_ARG, "unknown precision"};
        BAE_HIP_CHECK(hipSetDevice(c->device));
        join_job(c);
        check_sum_error(c);   // a sum queued by an earlier call gave up
        double_layer(c, q, c->ngm, v, c->nT, nrhs, prec, (hipStream_t)stream);
    });
}

int bae_apply_single_layer(bae_ctx* c, const double* q, double* v, int32_t nrhs, int32_t prec, void* stream) {
    return guard([&] {
        if (!c || !q || !v) throw Error{BAE_ERR_ARG, "null argument"};
        if (nrhs < 1 || nrhs > c->max_rhs) throw Error{BAE_ERR_ARG, "nrhs out of range"};
        if (prec != BAE_PREC_FP64 && prec != BAE_PREC_FP32 && prec != BAE_PREC_FFT)
            throw Error{BAE_ERR_ARG, "unknown precision"};
        BAE_HIP_CHECK(hipSetDevice(c->device));
        join_job(c);
        check_sum_error(c);   // a sum queued by an earlier call gave up
        const LayerScope layer(c, BAE_LAYER_SINGLE);
        double_layer(c, q, c->ngm, v, c->nT, nrhs, prec, (hipStream_t)stream);
    });
}

int bae_apply_operator(bae_ctx* c, const double* q, double* aq, int32_t nrhs, int32_t prec, void* stream) {
    return guard([&] {
        if (!c || !q || !aq) throw Error{BAE_ERR_ARG, "null argument"};
        if (nrhs < 1 || nrhs > c->max_rhs) throw Error{BAE_ERR_ARG, "nrhs out of range"};
        if (prec != BAE_PREC_FP64 && prec != BAE_PREC_FP32 && prec != BAE_PREC_FFT)
            throw Error{BAE_ERR_ARG, "unknown precision"};
        BAE_HIP_CHECK(hipSetDevice(c->device));
        join_job(c);
        check_sum_error(c);   // a sum queued by an earlier call gave up
        bae_operator(c, q, c->ngm, aq, c->ngm, nrhs, prec, (hipStream_t)stream);
    });
}

int bae_apply_direct(bae_ctx* c, const double* v, double* y, int32_t nrhs, int32_t prec, void* stream) {
    return guard([&] {
        if (!c || !v || !y) throw Error{BAE_ERR_ARG, "null argument"};
        if (nrhs < 1 || nrhs > c->max_rhs) throw Error{BAE_ERR_ARG, "nrhs out of range"};
        if (prec != BAE_PREC_FP64 && prec != BAE_PREC_FP32 && prec != BAE_PREC_FFT)
            throw Error{BAE_ERR_ARG, "unknown precision"};
        join_job(c);
        BAE_HIP_CHECK(hipSetDevice(c->device));
        check_sum_error(c);   // a sum queued by an earlier call gave up
        const LayerScope layer(c, BAE_LAYER_DIRECT);
        bae_operator(c, v, c->nT, y, c->nT, nrhs, prec, (hipStream_t)stream);
    });
}

int bae_lgf_sum_repeat(bae_ctx* c, const double* q, int32_t nrhs, int32_t prec, int32_t repeats, void* stream) {
    return guard([&] {
        if (!c || !q) throw Error{BAE_ERR_ARG, "null argument"};
        if (nrhs < 1 || nrhs > c->max_rhs) throw Error{BAE_ERR_ARG, "nrhs out of range"};
        if (prec != BAE_PREC_FP64 && prec != BAE_PREC_FP32 && prec != BAE_PREC_FFT)
            throw Error{BAE_ERR_ARG, "unknown precision"};
        if (repeats < 1 || repeats > 1000) throw Error{BAE_ERR_ARG, "repeats must be in [1, 1000]"};
        BAE_HIP_CHECK(hipSetDevice(c->device));
        join_job(c);
        check_sum_error(c);   // a sum queued by an earlier call gave up
        const hipStream_t st = (hipStream_t)stream;
        launch_weights(c->B, q, c->ngm, c->w.p, c->S.ps.padded, nrhs, weight_prec(prec), st);
        for (int i = 0; i < repeats; ++i) {
            int chunks = 0;
            apply_lgf(c, c->w.p, nrhs, prec, &chunks, st);
        }
    });
}

int bae_sum_stats(const bae_ctx* c, int32_t prec, int64_t* counts) {
    return guard([&] {
        if (!c || !counts) throw Error{BAE_ERR_ARG, "null argument"};
        if (prec != BAE_PREC_FP64 && prec != BAE_PREC_FP32)
            throw Error{BAE_ERR_ARG, "precision: BAE_PREC_FP64 or BAE_PREC_FP32 (the sum kernels)"};
        const bool fp32 = prec == BAE_PREC_FP32;
        const int tab_r = fp32 ? c->tabs.tab_r32 : c->tabs.tab_r64;
        for (int i = 0; i < 5; ++i) counts[i] = 0;
        classify_pairs(c, fp32, tab_r, fp32 ? c->tabs.far32() : c->tabs.far64(),
                       fp32 ? c->tabs.far_gap32() : c->tabs.far_gap64(), counts);
    });
}

int bae_lgf_eval(bae_ctx* c, const int32_t* off, int64_t count, double* out, int32_t prec, void* stream) {
    return guard([&] {
        if (!c || (count > 0 && (!off || !out)) || count < 0) throw Error{BAE_ERR_ARG, "bad argument"};
        if (prec != BAE_PREC_FP64 && prec != BAE_PREC_FP32)
            throw Error{BAE_ERR_ARG, "precision: BAE_PREC_FP64 or BAE_PREC_FP32 (the sum kernels)"};
        BAE_HIP_CHECK(hipSetDevice(c->device));
        lgf_eval_launch(off, count, out, prec, c->tabs, (hipStream_t)stream);
    });
}

}  // extern "C"
