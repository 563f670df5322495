// FFTs in LDS and the sine transforms of the finite auxiliary problem (fft.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace bae {

constexpr int kFftMaxLen = 4608;     // longest transform: two LDS buffers of it fit the 160 KB
constexpr int kFftMaxFactors = 16;
constexpr size_t kFftLdsBytes = 159 * 1024;   // dynamic LDS: 160 KB less 1 KB for the kernels' line tables

// Complex lines of length M that one block transforms at once: c M <= 8192 points (the
// in-place stages' register staging), and the c lines plus the root table (M more points,
// 16 B each) within the LDS; at most `cap`, at least 1 (M <= kFftMaxLen).
inline int fft_lines_per_block(int M, int cap) {
    const int by_points = 8192 / M;
    const int by_lds = (int)(kFftLdsBytes / (16 * (size_t)M)) - 1;
    return std::max(1, std::min(cap, std::min(by_points, by_lds)));
}

// A transform length with its radices and root table e^(-2 pi i t / M), t < M (device).
struct FftDev {
    int M = 0;
    int nf = 0;
    int f[kFftMaxFactors] = {};
    const double2* tw = nullptr;
};

// Radices of M in the order the stages apply them (4s, 2, 3s, 5s, then other primes).
std::vector<int> fft_factors(int M);
// The plan of length M on the current device (cached until the process ends).
FftDev fft_plan(int M, hipStream_t st);
// DST-I (X_k = sum_n x_n sin(pi n k / (N + 1)), unnormalised) of every line along `axis` of
// the row-major [n0][n1][n2] array x, in place, times scale.
void dst_axis(double* x, int n0, int n1, int n2, int axis, double scale, hipStream_t st);
// W = chi_{M-} L_h H on the interior nodes of the full grid n[3] (H, W: [n0-2][n1-2][n2-2];
// inside: the M+ mask of the full grid): the source of Algorithm 1's reconstruction step.
void difference_source(const double* H, const uint8_t* inside, const int* n, double s, double* W, hipStream_t st);
// u = G_h q on the n0 x n1 x n2 interior nodes of a box (zero on its boundary), in place:
// DST-I along the three axes, division by the eigenvalues of L_h, DST-I again.
void box_solve_fft(double* x, int n0, int n1, int n2, double s, hipStream_t st);

}  // namespace bae
