// Host-side geometry of the unfitted method: level sets, point sets, the exterior
// layer of the double layer, and the hat-function Dirichlet closure.
//
// Paper Sec. 2.1: M+ = nodes inside Omega (phi < 0; Sec. 4.2 convention), M- the rest,
// gamma+ = M+ nodes with a 6-neighbour in M-, gamma- = M- nodes with a 6-neighbour in M+,
// N+ = M+ u gamma-.  Sec. 3.2: D_q = neighbours of q in gamma- lying outside N+; E = union.
// Sec. 2.1 eq. "bc": one boundary point per gamma- node on the grid edge to an M+
// neighbour; on that edge the hat functions reduce to linear interpolation, so the
// closure row is (1-t) u(q) + t u(p) = g(x*).  Readings: smallest t wins, ties in the
// direction order -x,+x,-y,+y,-z,+z; t by 60 bisection halvings keeping the phi >= 0 end
// (analytic level sets) or by linear interpolation of node values (sampled level sets).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace bae {

static const int kDir[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

static double level_set(const bae_levelset& ls, double x, double y, double z) {
    const double dx = x - ls.center[0], dy = y - ls.center[1], dz = z - ls.center[2];
    const double* p = ls.params;
    switch (ls.kind) {
        case BAE_LS_SPHERE:
            return dx * dx + dy * dy + dz * dz - p[0] * p[0];
        case BAE_LS_ELLIPSOID: {
            const double a = dx / p[0], b = dy / p[1], c = dz / p[2];
            return a * a + b * b + c * c - 1.0;
        }
        case BAE_LS_TORUS: {
            const double q = std::sqrt(dx * dx + dy * dy) - p[0];
            return q * q + dz * dz - p[1] * p[1];
        }
        case BAE_LS_STAR: {
            const double rho = std::sqrt(dx * dx + dy * dy + dz * dz);
            const double theta = std::atan2(std::sqrt(dx * dx + dy * dy), dz);
            const double az = std::atan2(dy, dx);
            return rho - p[0] * (1.0 + p[1] * std::sin(p[2] * theta) * std::cos(p[3] * az));
        }
    }
    return NAN;
}

void build_geometry(const bae_grid& g, const bae_levelset& ls, Geometry& G) {
    for (int a = 0; a < 3; ++a)
        if (g.n[a] < 5 || g.n[a] > kMaxLatticeCoord + 1) throw Error{BAE_ERR_ARG, "grid: n must be in [5, 2049]"};
    if (!(g.h > 0) || !std::isfinite(g.h)) throw Error{BAE_ERR_ARG, "grid: h must be finite and > 0"};
    if (!(g.sigma >= 0) || !std::isfinite(g.sigma)) throw Error{BAE_ERR_ARG, "grid: sigma must be finite and >= 0"};
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(g.origin[a])) throw Error{BAE_ERR_ARG, "grid: non-finite origin"};
    if (ls.kind < BAE_LS_SPHERE || ls.kind > BAE_LS_SAMPLED) throw Error{BAE_ERR_ARG, "level set: unknown kind"};
    if (ls.kind == BAE_LS_SAMPLED && !ls.phi_samples) throw Error{BAE_ERR_ARG, "level set: samples missing"};
    if (ls.kind != BAE_LS_SAMPLED)
        for (int a = 0; a < 8; ++a)
            if (!std::isfinite(ls.params[a])) throw Error{BAE_ERR_NONFINITE, "level set: non-finite parameter"};

    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const int64_t N = (int64_t)n0 * n1 * n2;
    std::memcpy(G.n, g.n, sizeof(G.n));
    std::memcpy(G.origin, g.origin, sizeof(G.origin));
    G.h = g.h;
    auto lin = [&](int i, int j, int k) { return ((int64_t)i * n1 + j) * n2 + k; };
    auto X = [&](int a, int i) { return g.origin[a] + g.h * i; };

    std::vector<double> phi(N);
    for (int i = 0; i < n0; ++i)
        for (int j = 0; j < n1; ++j)
            for (int k = 0; k < n2; ++k) {
                const int64_t l = lin(i, j, k);
                phi[l] = ls.kind == BAE_LS_SAMPLED ? ls.phi_samples[l] : level_set(ls, X(0, i), X(1, j), X(2, k));
                if (!std::isfinite(phi[l])) throw Error{BAE_ERR_NONFINITE, "level set: non-finite value at a node"};
            }
    G.inside.assign(N, 0);
    int64_t nin = 0;
    for (int64_t l = 0; l < N; ++l) {
        G.inside[l] = phi[l] < 0.0;
        nin += G.inside[l];
    }
    if (nin == 0) throw Error{BAE_ERR_GEOMETRY, "empty interior M+"};
    G.n_mplus = nin;
    for (int i = 0; i < n0; ++i)
        for (int j = 0; j < n1; ++j)
            for (int k = 0; k < n2; ++k)
                if (G.inside[lin(i, j, k)] &&
                    (i < 2 || j < 2 || k < 2 || i > n0 - 3 || j > n1 - 3 || k > n2 - 3))
                    throw Error{BAE_ERR_GEOMETRY, "interior within two nodes of the grid edge"};

    // gamma sets (M+ keeps two nodes from the edge, so every neighbour below is in the grid)
    std::vector<uint8_t> nplus(G.inside);
    std::vector<int32_t> gp_index(N, -1);
    G.gp.clear();
    G.gm.clear();
    for (int i = 1; i < n0 - 1; ++i)
        for (int j = 1; j < n1 - 1; ++j)
            for (int k = 1; k < n2 - 1; ++k) {
                const int64_t l = lin(i, j, k);
                bool nb_in = false, nb_out = false;
                for (int d = 0; d < 6; ++d) {
                    const uint8_t v = G.inside[lin(i + kDir[d][0], j + kDir[d][1], k + kDir[d][2])];
                    nb_in |= v != 0;
                    nb_out |= v == 0;
                }
                if (G.inside[l] && nb_out) {
                    gp_index[l] = (int32_t)(G.gp.size() / 3);
                    G.gp.insert(G.gp.end(), {i, j, k});
                }
                if (!G.inside[l] && nb_in) {
                    G.gm.insert(G.gm.end(), {i, j, k});
                    nplus[l] = 1;
                }
            }
    const int64_t ngm = (int64_t)G.gm.size() / 3;

    // D_q and E
    std::vector<int32_t> ext_index(N, -1);
    for (int64_t q = 0; q < ngm; ++q)
        for (int d = 0; d < 6; ++d) {
            const int i = G.gm[3 * q] + kDir[d][0], j = G.gm[3 * q + 1] + kDir[d][1], k = G.gm[3 * q + 2] + kDir[d][2];
            if (!nplus[lin(i, j, k)]) ext_index[lin(i, j, k)] = 0;
        }
    G.ext.clear();
    for (int i = 0; i < n0; ++i)
        for (int j = 0; j < n1; ++j)
            for (int k = 0; k < n2; ++k)
                if (ext_index[lin(i, j, k)] == 0) {
                    ext_index[lin(i, j, k)] = (int32_t)(G.ext.size() / 3);
                    G.ext.insert(G.ext.end(), {i, j, k});
                }
    G.edge_q.clear();
    G.edge_k.clear();
    G.dcount.assign(ngm, 0);
    for (int64_t q = 0; q < ngm; ++q)
        for (int d = 0; d < 6; ++d) {
            const int i = G.gm[3 * q] + kDir[d][0], j = G.gm[3 * q + 1] + kDir[d][1], k = G.gm[3 * q + 2] + kDir[d][2];
            if (!nplus[lin(i, j, k)]) {
                G.edge_q.push_back((int32_t)q);
                G.edge_k.push_back(ext_index[lin(i, j, k)]);
                G.dcount[q]++;
            }
        }
    G.n_empty_d = 0;
    for (int64_t q = 0; q < ngm; ++q) G.n_empty_d += G.dcount[q] == 0;

    // closure
    G.partner.assign(ngm, -1);
    G.t.assign(ngm, 0.0);
    G.xstar.assign(3 * ngm, 0.0);
    for (int64_t q = 0; q < ngm; ++q) {
        const int qi = G.gm[3 * q], qj = G.gm[3 * q + 1], qk = G.gm[3 * q + 2];
        const double xq[3] = {X(0, qi), X(1, qj), X(2, qk)};
        double best = 2.0;
        for (int d = 0; d < 6; ++d) {
            const int pi = qi + kDir[d][0], pj = qj + kDir[d][1], pk = qk + kDir[d][2];
            const int64_t lp = lin(pi, pj, pk);
            if (!G.inside[lp]) continue;
            const double xp[3] = {X(0, pi), X(1, pj), X(2, pk)};
            double t;
            if (ls.kind == BAE_LS_SAMPLED) {
                const double fq = phi[lin(qi, qj, qk)], fp = phi[lp];
                t = fq / (fq - fp);
            } else {
                double lo = 0.0, hi = 1.0;
                for (int it = 0; it < 60; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    const double v = level_set(ls, xq[0] + mid * (xp[0] - xq[0]), xq[1] + mid * (xp[1] - xq[1]),
                                               xq[2] + mid * (xp[2] - xq[2]));
                    if (v < 0.0) hi = mid;
                    else lo = mid;
                }
                t = lo;
            }
            if (t < best) {
                best = t;
                G.partner[q] = gp_index[lp];
                for (int a = 0; a < 3; ++a) G.xstar[3 * q + a] = xq[a] + t * (xp[a] - xq[a]);
            }
        }
        G.t[q] = best;
    }

    // bounding box of N+ u E and the largest offset component
    for (int a = 0; a < 3; ++a) {
        G.bbox_lo[a] = 1 << 30;
        G.bbox_hi[a] = -(1 << 30);
    }
    auto grow = [&](int i, int j, int k) {
        const int v[3] = {i, j, k};
        for (int a = 0; a < 3; ++a) {
            G.bbox_lo[a] = std::min(G.bbox_lo[a], v[a]);
            G.bbox_hi[a] = std::max(G.bbox_hi[a], v[a]);
        }
    };
    for (int i = 0; i < n0; ++i)
        for (int j = 0; j < n1; ++j)
            for (int k = 0; k < n2; ++k)
                if (nplus[lin(i, j, k)]) grow(i, j, k);
    for (size_t e = 0; e < G.ext.size(); e += 3) grow(G.ext[e], G.ext[e + 1], G.ext[e + 2]);
    G.max_offset = 0;
    for (int a = 0; a < 3; ++a) G.max_offset = std::max(G.max_offset, G.bbox_hi[a] - G.bbox_lo[a]);
}

static inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

std::vector<int32_t> morton_order(const int32_t* p, int64_t count, const int lo[3]) {
    std::vector<std::pair<uint64_t, int32_t>> key(count);
    for (int64_t i = 0; i < count; ++i) {
        const uint64_t a = (uint64_t)(p[3 * i] - lo[0]), b = (uint64_t)(p[3 * i + 1] - lo[1]),
                       c = (uint64_t)(p[3 * i + 2] - lo[2]);
        key[i] = {spread3(a) << 2 | spread3(b) << 1 | spread3(c), (int32_t)i};
    }
    std::sort(key.begin(), key.end());
    std::vector<int32_t> perm(count);
    for (int64_t i = 0; i < count; ++i) perm[i] = key[i].second;
    return perm;
}

}  // namespace bae
