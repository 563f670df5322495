// Host-side state of one BAE context (shared by the C ABI in bae.cpp and the batch engine).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <functional>
#include <thread>
#include <memory>
#include <string>
#include <vector>

#include "conv.hpp"
#include "internal.hpp"
#include "ops.hpp"

namespace bae {

// ------------------------------------------------------------------ device memory
struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t n) {
        release();
        if (n == 0) n = 8;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error{BAE_ERR_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
        }
        bytes = n;
    }
    template <typename T>
    T* as() const { return (T*)p; }
};

template <typename T>
inline void upload(DevMem& m, const std::vector<T>& v, hipStream_t st) {
    m.alloc(sizeof(T) * v.size());
    if (!v.empty()) BAE_HIP_CHECK(hipMemcpyAsync(m.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
}

// ------------------------------------------------------------------ LGF table cache
// GMRES control of one context in device memory (used by the batched and served solves,
// where problems advance independently).
struct Ctl {
    int k;        // current Arnoldi step
    int maxit;    // iteration cap of the current GMRES
    double tol;   // relative tolerance of the current GMRES
};

struct Table {
    int device = 0;
    double s = 0.0;
    int R = 0;
    DevMem d64, d32;
};

std::shared_ptr<Table> get_table(int device, double s, int R, hipStream_t st);
int guard(const std::function<void()>& fn);

// ------------------------------------------------------------------ context
// IEEE binary16 encoding of an integer in [0, kMaxLatticeCoord] (exact: at most 11
// significant bits).
inline uint16_t half_bits(int32_t v) {
    if (v < 0 || v > kMaxLatticeCoord) throw Error{BAE_ERR_ARG, "lattice coordinate outside [0, 2048]"};
    if (v == 0) return 0;
    int e = 0;
    while ((v >> (e + 1)) != 0) ++e;                                  // v in [2^e, 2^(e+1))
    const uint32_t frac = e <= 10 ? ((uint32_t)v << (10 - e)) & 0x3FFu : ((uint32_t)v >> (e - 10)) & 0x3FFu;
    return (uint16_t)(((uint32_t)(e + 15) << 10) | frac);
}

struct PointBuf {
    DevMem x, y, z, xf, yf, zf, xd, yd, zd, xy16, zl, bbox;
    PointSet ps;
    std::vector<int32_t> perm;   // internal index -> index in the lexicographic list
    // pts3: lattice points (3 * count, AoS); order: the internal (Morton) order.  The device
    // copies are quantised (kQuant x index) and padded to whole blocks with the last point.
    void set(const std::vector<int32_t>& pts3, const std::vector<int32_t>& order, hipStream_t st) {
        const int64_t n = (int64_t)order.size();
        const int64_t nblk = (n + kSourceBlock - 1) / kSourceBlock;
        const int64_t np = nblk * kSourceBlock;
        std::vector<uint32_t> h[3];
        std::vector<float> hf[3];
        std::vector<double> hd[3];
        std::vector<uint32_t> hxy(np);
        std::vector<float> hzl(np);
        ps.hq.assign(3 * np, 0);
        for (int a = 0; a < 3; ++a) {
            h[a].resize(np);
            hf[a].resize(np);
            hd[a].resize(np);
            for (int64_t i = 0; i < np; ++i) {
                const int32_t v = kQuant * pts3[3 * order[std::min(i, n - 1)] + a];
                if (v < 0) throw Error{BAE_ERR_ARG, "lattice point outside the grid"};
                ps.hq[3 * i + a] = v;
                h[a][i] = (uint32_t)v;
                hf[a][i] = (float)v;
                hd[a][i] = (double)v;
            }
        }
        for (int64_t i = 0; i < np; ++i) {
            const int32_t* p = &pts3[3 * order[std::min(i, n - 1)]];
            hxy[i] = (uint32_t)half_bits(p[0]) | ((uint32_t)half_bits(p[1]) << 16);
            hzl[i] = (float)p[2];
        }
        ps.hbox.assign(6 * nblk, 0);
        for (int64_t b = 0; b < nblk; ++b)
            for (int a = 0; a < 3; ++a) {
                int lo = 1 << 30, hi = -(1 << 30);
                for (int64_t i = b * kSourceBlock; i < (b + 1) * kSourceBlock; ++i) {
                    lo = std::min(lo, ps.hq[3 * i + a]);
                    hi = std::max(hi, ps.hq[3 * i + a]);
                }
                ps.hbox[6 * b + a] = lo;
                ps.hbox[6 * b + 3 + a] = hi;
            }
        upload(x, h[0], st);
        upload(y, h[1], st);
        upload(z, h[2], st);
        upload(xf, hf[0], st);
        upload(yf, hf[1], st);
        upload(zf, hf[2], st);
        upload(xd, hd[0], st);
        upload(yd, hd[1], st);
        upload(zd, hd[2], st);
        upload(xy16, hxy, st);
        upload(zl, hzl, st);
        upload(bbox, ps.hbox, st);
        ps.count = n;
        ps.padded = np;
        ps.x = x.as<uint32_t>();
        ps.y = y.as<uint32_t>();
        ps.z = z.as<uint32_t>();
        ps.xf = xf.as<float>();
        ps.yf = yf.as<float>();
        ps.zf = zf.as<float>();
        ps.xd = xd.as<double>();
        ps.yd = yd.as<double>();
        ps.zd = zd.as<double>();
        ps.xy16 = xy16.as<uint32_t>();
        ps.zl = zl.as<float>();
        ps.bbox = bbox.as<int32_t>();
        ps.nblk = nblk;
        perm = order;
        BAE_HIP_CHECK(hipStreamSynchronize(st));   // host vectors are released on return
    }
};

// A work list on the device (see SumPlan).
struct PlanBuf {
    SumPlan plan;
    DevMem items, counter;
    // err_dev: the device view of the error word the sum's bounded waits set on giving up
    void build(const PointSet& T, const PointSet& S, const SumTables& tabs, int32_t* err_dev, uint32_t polls,
               hipStream_t st);
};

}  // namespace bae

using namespace bae;

struct bae_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bae_grid grid{};
    bae_options opt{};
    double s = 0.0;
    Geometry geo;
    int64_t ngp = 0, ngm = 0, next = 0, nT = 0, nS = 0;

    PointBuf T, S, Mp;         // targets gamma, sources gamma- u E, interior M+ (lazy)
    DevMem t_pos;              // internal target index -> position in [gamma+; gamma-]
    DevMem csr_rowptr, csr_col, csr_coef;
    CSR B;
    // single-layer weights map (Sec. 3.4): w(n) = q(n) for n in gamma-, nothing for E
    DevMem csr1_rowptr, csr1_col, csr1_coef;
    CSR B1;
    // The operator of the current solve (set per solve, the double layer outside one):
    // source weights map, source points, their work list, and the number of unknowns.
    struct OpView {
        const CSR* B = nullptr;
        const PointSet* S = nullptr;
        PlanBuf* plan = nullptr;
        int64_t n = 0;
        bool direct = false;   // the direct formulation (Sec. 3.1): unknowns v on gamma
    } op;
    // direct formulation: its weights map from v on gamma ([gamma+; gamma-]) onto the sources
    // gamma (the targets' own point set), its work list (gamma x gamma), the RHS [0; b]
    bool direct_ready = false;
    DevMem csrd_rowptr, csrd_col, csrd_coef;
    CSR Bd;
    PlanBuf plan_dir;
    DevMem t_inv;              // position in [gamma+; gamma-] -> internal target index
    DevMem bdir;               // [rhs][nT]
    int64_t vec_cap = 0;       // elements per RHS of b, x, r, tmp and the Krylov vectors
    int64_t dens_n = 0;        // length of the last solve's density (|gamma-|, or |gamma| for direct)
    int batch_refs = 0;        // batches holding this context (they keep pointers to its vectors)
    // the LGF sum by FFT convolution on the box of N+ u E (lazy): the plan, and the box index
    // of every source (gamma- u E), target (gamma, also the direct formulation's sources) and
    // M+ point, each in its point set's internal order
    std::unique_ptr<ConvPlan> conv;
    DevMem conv_sidx, conv_tidx, conv_midx;
    DevMem cl_tq, cl_tp, cl_t;
    Closure cl;
    std::shared_ptr<Table> table;
    SumTables tabs;
    PlanBuf plan;              // work list of the operator's sum (targets gamma, sources gamma- u E)
    int sum_grid = 1;          // workgroups of the persistent sum kernels (one per CU)

    int max_rhs = 16;
    DevMem w, part;
    int64_t part_cap = 0;
    KrylovState K;
    DevMem kV, kH, kcs, ksn, kg, khist, kbeta, kdone, kkdone;
    int maxj = 0;
    DevMem hA, hB, nrm, dotpart, ycoef;
    DevMem b, x, r, tmp;       // [rhs][ngm]
    DevMem rcU, rcC, rcS;      // Krylov recycling of refined solves: U, C [rhs][p][ngm], C'w slices
    DevMem up_gamma;           // [rhs][nT] external order
    DevMem u_gamma;            // [rhs][nT]
    DevMem vsum;               // [rhs][nT] chunk-reduced sums (operator scratch)
    DevMem wf;                 // [rhs][|M+|] h^2 f in Mp order
    std::vector<int32_t> mp_lin;   // linear grid index of each M+ point in Mp order (lazy)
    // box of Algorithm 1 (bae_set_rhs_box and the grid solution): u_p on the interior nodes per
    // RHS, and the interior index of every target and of every M+ point
    bool particular_box = false;
    bool box_ready = false;
    int box_n[3] = {0, 0, 0};  // interior nodes per axis (n_d - 2)
    int64_t box_nn = 0;
    DevMem box_u, box_tidx, box_mpidx;
    DevMem box_h, box_w;       // reconstruction scratch: the density on the box, chi_{M-} L_h of it
    DevMem inside_dev;         // M+ mask of the grid (uint8)
    DevMem ctl;                // Ctl of RHS 0 for batched / served solves
    int nrhs = 0;
    bool has_f = false, rhs_ready = false, solved = false;
    std::vector<std::vector<double>> hist;  // per rhs
    bool has_grid = false;                  // ugrid holds the last solve's grid solution
    DevMem ugrid;                           // [rhs][n0 n1 n2], NaN outside N+
    DevMem gdev;                            // [max_rhs][ngm] boundary data staged from the host
    DevMem partner_dev;                     // gamma+ index of each gamma- node's partner
    DevMem mp_lin_dev, gm_lin_dev;          // linear grid index of each M+ (Mp order) / gamma- node (lazy)
    hipEvent_t rhs_ev = nullptr;            // end of the last right-hand side's device work
    // a solve started by bae_solve_async, driven by a host thread of its own
    struct Job {
        std::thread th;
        std::atomic<int> state{0};          // 0 none, 1 running, 2 finished (not yet collected)
        int status = 0;
        std::string error;
        std::vector<bae_result> res;
    } job;
    int32_t* pinned_flags = nullptr;        // host pinned, coherent and mapped, 2 * max_rhs + 1
    int32_t* flags_dev = nullptr;           // the same memory as the device sees it
    int32_t* err_host = nullptr;            // word 2 max_rhs: set by an LGF sum whose bounded wait gave up
    int32_t* err_dev = nullptr;
    int32_t* bad_host = nullptr;            // word 2 max_rhs + 1: set by a non-finite device input
    int32_t* bad_dev = nullptr;
    uint32_t wait_polls = kWaitPolls;
};

namespace bae {
// Throws BAE_ERR_HIP when an LGF sum launched on the context since the last check gave up
// on a bounded wait (its results are incomplete); clears the word and resets the work
// counter first, so the context stays usable.
void check_sum_error(bae_ctx* c);
// Waits for the host thread of a solve started by bae_solve_async (its results stay for
// bae_solve_wait).
void join_job(bae_ctx* c);
// Pair counts of the LGF sum over gamma x (gamma- u E) by the kernels' block classification
// (table, far / gather, FP32 far, mixed within / beyond the LDS radius), added to cnt[5].
void classify_pairs(const bae_ctx* c, bool fp32, int tab_r, bool far_ok, int far_gap, int64_t* cnt);
// Device part of bae_create for an already classified geometry (throws Error).
bae_ctx* create_context(const bae_grid& grid, const bae_options* opt, Geometry&& geo);
int64_t estimate_context_bytes(const Geometry& G, double s, const bae_options* opt);
}  // namespace bae
