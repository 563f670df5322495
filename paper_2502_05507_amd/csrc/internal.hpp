// Internal declarations of the BAE / LGF library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bae.h"

namespace bae {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
struct Error {
    int code;
    std::string msg;
};
#define BAE_HIP_CHECK(expr)                                                                  \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            throw ::bae::Error{BAE_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// ------------------------------------------------------------------ geometry (host)
struct Geometry {
    int n[3];
    double origin[3];
    double h;
    std::vector<uint8_t> inside;            // n0*n1*n2, M+
    std::vector<int32_t> gp, gm, ext;       // 3*count, lexicographic
    std::vector<int32_t> edge_q, edge_k;    // (index in gm, index in ext) per pair q, k in D_q
    std::vector<int32_t> partner;           // index in gp
    std::vector<double> t, xstar;           // |gm|, 3*|gm|
    std::vector<int32_t> dcount;            // |D_q|
    int64_t n_mplus = 0;
    int64_t n_empty_d = 0;
    int max_offset = 0;
    int bbox_lo[3], bbox_hi[3];             // of N+ u E
};
// Throws Error on invalid input.
void build_geometry(const bae_grid& g, const bae_levelset& ls, Geometry& out);
// Morton (Z-order) permutation of integer points (3*count int32): perm[new] = old.
std::vector<int32_t> morton_order(const int32_t* pts, int64_t count, const int lo[3]);

// ------------------------------------------------------------------ LGF table (device)
int64_t table_size(int R);
// FP64 table G_s for 0<=a<=b<=c<=R into out (device), on stream.
void lgf_table_generate(double s, int R, double* out, hipStream_t stream);
// The same with no allocation: scratch in a static device array (R <= kNoAllocMaxR);
// asynchronous on stream; calls that overlap on one GPU race on the scratch.
constexpr int kNoAllocMaxR = 2048;
void lgf_table_generate_noalloc(double s, int R, double* out, hipStream_t stream);

// ------------------------------------------------------------------ LGF sum (device)
// Points are grouped in blocks of kSourceBlock consecutive (Morton-ordered) points; each
// block carries its bounding box so a wavefront can classify a whole block before
// touching its points.  Device coordinates are quantised: kQuant x the lattice index.
constexpr int kSourceBlock = 64;
constexpr int kQuant = 4;
constexpr int kLdsRadiusFar32 = 60;       // LDS table radius of the FP32 sum, sigma = 0 (159 KB)
constexpr int kLdsRadiusFar64 = 47;       // ... of the FP64 sum, sigma = 0 (157 KB)
constexpr int kLdsRadius32 = 59;          // ... FP32, sigma > 0 and batched sums (151 KB + index arrays)
constexpr int kLdsRadius64 = 46;          // ... FP64, sigma > 0 and batched sums (147 KB + index arrays)
constexpr int kMaxTableRadius = 1200;     // largest resident table (sigma > 0)
constexpr int kFarGap = 32;               // far field used beyond this gap (sigma = 0)
constexpr double kYukawaTolerance = 1e-6; // sigma > 0 FP32 far field: largest accepted relative error
constexpr int kSumThreads = 1024;         // threads per workgroup of the LGF sum
constexpr int kMaxChunks = 64;            // source chunks (partial sums per target)
constexpr int kGroupTiles = 16;           // 64-target tiles per work item of the LGF sum
constexpr uint32_t kWaitPolls = 1u << 22;  // polls (s_sleep 1 each, ~0.1 s in all) of a bounded wait
constexpr int kMaxLatticeCoord = 2048;    // largest lattice coordinate: every integer up to 2048
                                          // is exact in binary16 (the FP32 far field's differences)

// Pair classes of a (64-target wavefront, source block) pair; gap and span in quantised
// units (the smallest and largest max-norm distance between the two bounding boxes).
// Far blocks (every pair beyond far_gap, where the far field holds) are kClassFar in FP64
// and kClassFar2 in FP32.
enum BlockClass { kClassTable = 0, kClassFar = 1, kClassFar2 = 2, kClassGather = 3, kClassMixed = 4 };
__host__ __device__ inline int block_class(int gap, int span, int tab_r, bool far_ok, bool fp32, int far_gap) {
    if (span <= kQuant * tab_r) return kClassTable;
    if (far_ok) {
        if (gap > kQuant * far_gap) return fp32 ? kClassFar2 : kClassFar;
    } else if (gap > kQuant * tab_r) {
        return kClassGather;
    }
    return kClassMixed;
}

// A set of lattice points on the device: SoA quantised coordinates as uint32, float and
// double, the lattice coordinates as packed binary16 (x, y) and float z, and per-block
// quantised bounding boxes [nblk][lo xyz, hi xyz].
struct PointSet {
    int64_t count = 0;
    int64_t padded = 0;        // nblk * kSourceBlock; entries past count repeat the last point
    uint32_t* x = nullptr;
    uint32_t* y = nullptr;
    uint32_t* z = nullptr;
    float* xf = nullptr;
    float* yf = nullptr;
    float* zf = nullptr;
    double* xd = nullptr;
    double* yd = nullptr;
    double* zd = nullptr;
    uint32_t* xy16 = nullptr;  // lattice (x, y) as two binary16 (exact: coordinates <= kMaxLatticeCoord)
    float* zl = nullptr;       // lattice z
    int32_t* bbox = nullptr;
    int64_t nblk = 0;
    std::vector<int32_t> hq;   // host copy of the quantised coordinates (3 * padded, AoS)
    std::vector<int32_t> hbox; // host copy of the block boxes
};

struct SumTables {
    const double* near64 = nullptr;          // table prefix staged in LDS (device)
    const float* near32 = nullptr;
    const double* full64 = nullptr;          // full table (device), radius full_r
    const float* full32 = nullptr;
    int full_r = 0;
    int tab_r64 = 0, tab_r32 = 0;            // LDS radii: min(build radius, full_r)
    bool far_field = false;                  // sigma == 0: expansion beyond the LDS table
    bool yukawa32 = false;                   // sigma > 0, FP32: the checked Yukawa-form expansion
    double kappa = 0.0;                      // sqrt(s)
    double yukawa_err = -1.0;                // its largest relative error beyond tab_r32 (when checked)
    bool far32() const { return far_field || yukawa32; }
    bool far64() const { return far_field; }
    int far_gap32() const { return far_field ? kFarGap : tab_r32; }
    int far_gap64() const { return kFarGap; }
};

// Work list of one (targets, sources) pair: items (group of kGroupTiles consecutive
// 64-target tiles, source chunk), ordered by decreasing estimated cost so the dynamically
// scheduled workgroups finish together.
struct SumPlan {
    int chunks = 1, blk_per_chunk = 1;
    int64_t nitems = 0;
    uint32_t* items = nullptr;     // device: group | chunk << 20
    unsigned long long* counter = nullptr;   // device: work counter, 0 between launches
    int32_t* err = nullptr;        // device view of the error word a bounded wait sets on giving up
    uint32_t wait_polls = kWaitPolls;   // polls of each bounded wait of the sum's work hand-off
    int64_t class_pairs[2][5] = {{0}};   // [fp64, fp32][class] pairs (mixed split: 3 table, 4 other)
};
// Host: chunking, per-item cost, order and pair statistics (items left on the host in
// 'host_items'); the caller uploads them.
void plan_sum(const PointSet& T, const PointSet& S, const SumTables& tabs, SumPlan& plan,
              std::vector<uint32_t>& host_items);
int lgf_sum_chunks(int64_t nt, int64_t nblk);
int lgf_sum_grid(int device);    // workgroups of the persistent sum kernels

// v[r][t] (partials per source chunk: part[r][chunk][t]) = sum_s w[r][s] G(T_t - S_s).
// w is FP64 when prec == BAE_PREC_FP64, FP32 otherwise.  Returns number of chunks used.
// skip: optional device flag; when it is set at launch time the kernels do nothing.
int lgf_sum_launch(const PointSet& T, const PointSet& S, const void* w, int nrhs, int prec,
                   const SumTables& tabs, const SumPlan& plan, double* part, int64_t part_capacity,
                   int grid, hipStream_t st, const int32_t* skip = nullptr);
void lgf_eval_launch(const int32_t* off, int64_t count, double* out, int prec, const SumTables& tabs,
                     hipStream_t st);
// Largest relative difference between the sigma > 0 far-field form (evaluated in FP64) and
// the exact table over every offset with max-norm in (from_r, R]; host result.
double yukawa_check(const double* table, int R, int from_r, double kappa, hipStream_t st);

}  // namespace bae
