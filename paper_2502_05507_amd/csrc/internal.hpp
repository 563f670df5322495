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

// ------------------------------------------------------------------ LGF sum (device)
// Points are grouped in blocks of kSourceBlock consecutive (Morton-ordered) points; each
// block carries its integer bounding box so a wavefront can classify a whole block as
// near, far or mixed before touching its points.
constexpr int kSourceBlock = 64;

// A set of integer lattice points on the device: SoA int32 coordinates, the same
// coordinates as float and double, and per-block bounding boxes [nblk][lo xyz, hi xyz].
struct PointSet {
    int64_t count = 0;
    int64_t padded = 0;        // nblk * kSourceBlock; entries past count repeat the last point
    int32_t* x = nullptr;
    int32_t* y = nullptr;
    int32_t* z = nullptr;
    float* xf = nullptr;
    float* yf = nullptr;
    float* zf = nullptr;
    double* xd = nullptr;
    double* yd = nullptr;
    double* zd = nullptr;
    int32_t* bbox = nullptr;
    int64_t nblk = 0;
};

enum SumMode { MODE_NEAR_FAR = 0, MODE_TABLE = 1 };

struct SumTables {
    int near_r64 = 0, near_r32 = 0;         // LDS radii
    const double* near64 = nullptr;          // prefix of the full table (device)
    const float* near32 = nullptr;
    const double* full64 = nullptr;          // full table (device), radius full_r
    const float* full32 = nullptr;
    int full_r = 0;
    bool far_field = false;                  // sigma == 0: expansion beyond the near radius
};

// v[r][t] (partials per source chunk: part[r][chunk][t]) = sum_s w[r][s] G(T_t - S_s).
// w is FP64 when prec == BAE_PREC_FP64, FP32 otherwise.  Returns number of chunks used.
int lgf_sum_launch(const PointSet& T, const PointSet& S, const void* w, int nrhs, int prec,
                   const SumTables& tabs, double* part, int64_t part_capacity, hipStream_t st);
int lgf_sum_chunks(int64_t nt, int64_t ns);
void lgf_eval_launch(const int32_t* off, int64_t count, double* out, int prec, const SumTables& tabs,
                     hipStream_t st);

}  // namespace bae
