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
#include <stdint.h>

#include <algorithm>
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
