// Grouping of a batch of unequal layouts (host code only).
//
// The batched kernels work on groups of equal order: a layout of n_a antennas
// is embedded in a group of padded order N = n_pad * N_m as the block
// diagonal [Z 0; 0 I], whose LU with partial pivoting is that of Z followed by
// the identity (the padding rows are zero in Z's columns, so they never win a
// pivot search, and Z's rows are zero in the padding columns), and whose
// solution for a right-hand side padded with zeros is the layout's solution
// padded with zeros.  Padding costs work, groups cost latency (each group runs
// its own chain of panel factorisations), so the grouping is a cut of the
// layouts sorted by size into contiguous runs, chosen by dynamic programming
// to minimise the modelled time
//   sum over groups of  t_group + t_order * N + t_system * c * N^3
// (c systems of padded order N per group).
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "../../include/harp.h"

namespace {

constexpr double kDefaultCost[3] = {1.0e-4, 3.0e-6, 1.3e-13};

}  // namespace

extern "C" harp_status harp_batch_plan(const int32_t* n_ant, int32_t n_sys, int32_t n_mbf, int32_t pad_multiple,
                                       int32_t max_order, int32_t max_batch, const double* cost, int32_t* order,
                                       int32_t* group_begin, int32_t* group_pad, int32_t* n_groups) {
    if (!n_ant || !order || !group_begin || !group_pad || !n_groups) return HARP_E_ARG;
    if (n_sys <= 0 || n_mbf <= 0 || pad_multiple <= 0 || max_batch <= 0 || max_order <= 0) return HARP_E_ARG;
    const double* c = cost ? cost : kDefaultCost;
    for (int i = 0; i < 3; ++i)
        if (!(c[i] >= 0.0)) return HARP_E_ARG;
    std::vector<int32_t> idx(n_sys);
    std::iota(idx.begin(), idx.end(), 0);
    for (int i = 0; i < n_sys; ++i)
        if (n_ant[i] <= 0) return HARP_E_ARG;
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return n_ant[a] < n_ant[b]; });
    auto padded = [&](int32_t na) { return int64_t((na + pad_multiple - 1) / pad_multiple) * pad_multiple; };
    if (padded(n_ant[idx[n_sys - 1]]) * n_mbf > max_order) return HARP_E_ARG;

    // best[j]: cheapest cut of the first j sorted systems; from[j]: start of its last group
    std::vector<double> best(size_t(n_sys) + 1, 0.0);
    std::vector<int32_t> from(size_t(n_sys) + 1, 0);
    for (int j = 1; j <= n_sys; ++j) {
        const double N = double(padded(n_ant[idx[j - 1]]) * n_mbf);
        const double per_sys = c[2] * N * N * N;
        const double fixed = c[0] + c[1] * N;
        best[j] = -1.0;
        for (int i = std::max(0, j - max_batch); i < j; ++i) {
            const double t = best[i] + fixed + per_sys * (j - i);
            if (best[j] < 0.0 || t < best[j]) {
                best[j] = t;
                from[j] = i;
            }
        }
    }
    std::vector<int32_t> cuts;
    for (int j = n_sys; j > 0; j = from[j]) cuts.push_back(j);
    std::reverse(cuts.begin(), cuts.end());
    int g = 0, start = 0;
    for (int32_t end : cuts) {
        group_begin[g] = start;
        group_pad[g] = int32_t(padded(n_ant[idx[end - 1]]));
        ++g;
        start = end;
    }
    group_begin[g] = n_sys;
    *n_groups = g;
    std::copy(idx.begin(), idx.end(), order);
    return HARP_OK;
}

// ---------------------------------------------------------------------------
// Overlapping-subarray tessellation (Section II-D, subarray figure).
//
// Flat-top regular hexagons of circumradius R tile the plane with centres on
// the lattice c(i, j) = o + (1.5 R i, sqrt(3) R (j + i / 2)); the hexagon of a
// centre is exactly the set of points nearer to it than to any other centre,
// so an antenna's inner cell is its nearest centre.  A point d from a centre
// lies in the concentric flat-top hexagon of circumradius Rh iff
//   max(2 |d_y| / sqrt(3), |d_x| + |d_y| / sqrt(3)) <= Rh.
// ---------------------------------------------------------------------------

namespace {

constexpr double kSqrt3 = 1.73205080756887729353;

inline double hex_radius(double dx, double dy) {
    const double ay = std::fabs(dy) / kSqrt3;
    return std::max(2.0 * ay, std::fabs(dx) + ay);
}

struct Cell {
    int64_t i, j;
    bool operator<(const Cell& o) const { return i != o.i ? i < o.i : j < o.j; }
    bool operator==(const Cell& o) const { return i == o.i && j == o.j; }
};

}  // namespace

extern "C" harp_status harp_tessellate(const double* x, const double* y, int32_t n_ant, double r_in, double r_ext,
                                       double ox, double oy, int32_t* n_cells, int64_t* n_members,
                                       int64_t* cell_begin, int32_t* cell_inner, int32_t* members,
                                       double* centers) {
    if (!x || !y || !n_cells || !n_members || n_ant <= 0) return HARP_E_ARG;
    if (!(r_in > 0.0) || !(r_ext >= 0.0) || !std::isfinite(r_in) || !std::isfinite(r_ext) || !std::isfinite(ox) ||
        !std::isfinite(oy))
        return HARP_E_ARG;
    const double R = r_in, Rout = r_in + r_ext;
    auto centre = [&](const Cell& c, double* cx, double* cy) {
        *cx = ox + 1.5 * R * double(c.i);
        *cy = oy + kSqrt3 * R * (double(c.j) + 0.5 * double(c.i));
    };
    // inner cell of every antenna: the nearest centre among the lattice points
    // around the fractional lattice coordinates (ties: smallest (i, j))
    std::vector<Cell> own(n_ant);
    for (int a = 0; a < n_ant; ++a) {
        if (!std::isfinite(x[a]) || !std::isfinite(y[a])) return HARP_E_ARG;
        const double fi = (x[a] - ox) / (1.5 * R);
        const double fj = (y[a] - oy) / (kSqrt3 * R) - 0.5 * fi;
        const int64_t i0 = int64_t(std::floor(fi)), j0 = int64_t(std::floor(fj));
        Cell best{0, 0};
        double bd = -1.0;
        for (int64_t i = i0 - 1; i <= i0 + 2; ++i) {
            for (int64_t j = j0 - 2; j <= j0 + 2; ++j) {
                double cx, cy;
                centre(Cell{i, j}, &cx, &cy);
                const double d = (x[a] - cx) * (x[a] - cx) + (y[a] - cy) * (y[a] - cy);
                if (bd < 0.0 || d < bd || (d == bd && Cell{i, j} < best)) {
                    bd = d;
                    best = Cell{i, j};
                }
            }
        }
        own[a] = best;
    }
    std::vector<Cell> cells(own);
    std::sort(cells.begin(), cells.end());
    cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
    const int nc = int(cells.size());
    // subarray of each cell: its inner antennas (ascending), then every other
    // antenna inside the outer hexagon (ascending)
    int64_t total = 0;
    std::vector<int32_t> list;
    std::vector<int64_t> begin(size_t(nc) + 1, 0);
    std::vector<int32_t> inner(nc, 0);
    const bool write = members != nullptr;
    if (write && (!cell_begin || !cell_inner || !centers)) return HARP_E_ARG;
    for (int c = 0; c < nc; ++c) {
        double cx, cy;
        centre(cells[c], &cx, &cy);
        begin[c] = total;
        list.clear();
        for (int a = 0; a < n_ant; ++a)
            if (own[a] == cells[c]) list.push_back(a);
        inner[c] = int32_t(list.size());
        for (int a = 0; a < n_ant; ++a)
            if (!(own[a] == cells[c]) && hex_radius(x[a] - cx, y[a] - cy) <= Rout) list.push_back(a);
        if (write) {
            std::copy(list.begin(), list.end(), members + total);
            cell_inner[c] = inner[c];
            centers[2 * c] = cx;
            centers[2 * c + 1] = cy;
        }
        total += int64_t(list.size());
    }
    begin[nc] = total;
    if (write) std::copy(begin.begin(), begin.end(), cell_begin);
    *n_cells = nc;
    *n_members = total;
    return HARP_OK;
}
