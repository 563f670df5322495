// The LGF sum as an FFT convolution on the grid box (conv.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "internal.hpp"

namespace bae {

// v(t) = sum_s w(s) G_s(t - s) for lattice points t, s of one box, by zero-padded FFTs:
// the box of extents e (lo its first node) is embedded in a periodic grid of M_d >= 2 e_d - 1
// nodes, on which the kernel sampled at the wrapped offsets is a circulant (Hockney's
// method), so the cyclic convolution equals the free-space sum at every node of the box.
struct ConvPlan {
    int lo[3] = {0, 0, 0}, e[3] = {0, 0, 0}, M[3] = {0, 0, 0}, H[3] = {0, 0, 0};
    FftDev fx, fy, fz;            // transforms along the three axes (lengths M0, M1, M2)
    double* ghat = nullptr;       // [H0][H1][H2] real: the kernel's transform on one octant
    double* R = nullptr;          // [e0][e1][e2] real: weights in, potentials out
    double2* C = nullptr;         // [e0][M1][M2] complex: the partly transformed grid
    int64_t bytes = 0;
    ~ConvPlan();
    // Plans, the kernel's transform (G exactly as the FP64 sum evaluates it: the table within
    // tab_r64, the far-field expansion beyond it when the sum has one, else the full table).
    void build(const int lo_[3], const int hi_[3], const SumTables& tabs, hipStream_t st);
    // out[t] = scale sum_s w[s] G(T_t - S_s) with sidx / tidx the box index of every source /
    // target (ns, nt); one right-hand side; skipped while *skip is set (when given).
    void apply(const double* w, const int32_t* sidx, int64_t ns, const int32_t* tidx, int64_t nt, double* out,
               double scale, const int32_t* skip, hipStream_t st);
    int64_t index(int i, int j, int k) const {   // box index of lattice node (i, j, k)
        return ((int64_t)(i - lo[0]) * e[1] + (j - lo[1])) * e[2] + (k - lo[2]);
    }
};

// Smallest length >= n whose prime factors are 2, 3 and 5 (the LDS FFT's register radices).
int fft_smooth_length(int n);

}  // namespace bae
