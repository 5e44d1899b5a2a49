// Host-only driver for the address / undefined-behaviour sanitizer build of
// the oracle's C reaction sums and the library's host planners (batch
// grouping and hexagonal tessellation).  Every call is checked against the
// invariants its documentation states; the sanitizers abort on any invalid
// access or undefined operation.  Prints "sanitize ok" and exits 0 when all
// checks pass.
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <random>
#include <vector>

#include "../../include/harp.h"

extern "C" {
void oracle_dyadic(double k, double dx, double dy, double dz, double* out);
void oracle_reaction(double k, double omega_mu, int nT, const double* T, int nS, const double* S, double Rx, double Ry,
                     double Rz, double reg, double* out);
void oracle_reaction_grid(double k, double omega_mu, int n_mbf, int n_samp, const double* samples, int n_pts,
                          const double* Rx, const double* Ry, double reg, double* out);
}

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static void plan_case(std::mt19937_64& rng, int n_sys, int lo, int hi, int n_mbf, int pad, int max_order,
                      int max_batch, const double* cost) {
    std::uniform_int_distribution<int> d(lo, hi);
    std::vector<int32_t> na(n_sys), order(n_sys), gb(n_sys + 1), gp(n_sys);
    for (auto& v : na) v = d(rng);
    int32_t ng = 0;
    const harp_status s = harp_batch_plan(na.data(), n_sys, n_mbf, pad, max_order, max_batch, cost, order.data(),
                                          gb.data(), gp.data(), &ng);
    const int need = ((*std::max_element(na.begin(), na.end()) + pad - 1) / pad) * pad * n_mbf;
    if (need > max_order) {
        CHECK(s == HARP_E_ARG);
        return;
    }
    CHECK(s == HARP_OK);
    CHECK(ng >= 1 && ng <= n_sys);
    CHECK(gb[0] == 0 && gb[ng] == n_sys);
    std::vector<int> seen(n_sys, 0);
    for (int g = 0; g < ng; ++g) {
        CHECK(gb[g + 1] > gb[g] && gb[g + 1] - gb[g] <= max_batch);
        CHECK(gp[g] % pad == 0 && gp[g] * n_mbf <= max_order);
        for (int k = gb[g]; k < gb[g + 1]; ++k) {
            CHECK(order[k] >= 0 && order[k] < n_sys);
            seen[order[k]] += 1;
            CHECK(na[order[k]] <= gp[g]);
        }
    }
    for (int v : seen) CHECK(v == 1);
}

static void tess_case(std::mt19937_64& rng, int n_ant, double radius, double r_in, double r_ext, double ox,
                      double oy) {
    std::uniform_real_distribution<double> u(-radius, radius);
    std::vector<double> x(n_ant), y(n_ant);
    for (int a = 0; a < n_ant; ++a) {
        x[a] = u(rng);
        y[a] = u(rng);
    }
    int32_t nc = 0;
    int64_t nm = 0;
    CHECK(harp_tessellate(x.data(), y.data(), n_ant, r_in, r_ext, ox, oy, &nc, &nm, nullptr, nullptr, nullptr,
                          nullptr) == HARP_OK);
    std::vector<int64_t> begin(nc + 1);
    std::vector<int32_t> inner(nc), members(std::max<int64_t>(nm, 1));
    std::vector<double> centers(2 * size_t(nc));
    CHECK(harp_tessellate(x.data(), y.data(), n_ant, r_in, r_ext, ox, oy, &nc, &nm, begin.data(), inner.data(),
                          members.data(), centers.data()) == HARP_OK);
    std::vector<int> owner(n_ant, 0);
    for (int c = 0; c < nc; ++c) {
        CHECK(begin[c + 1] - begin[c] >= inner[c] && inner[c] >= 1);
        for (int64_t k = begin[c]; k < begin[c + 1]; ++k) {
            CHECK(members[k] >= 0 && members[k] < n_ant);
            if (k < begin[c] + inner[c]) owner[members[k]] += 1;
        }
    }
    for (int v : owner) CHECK(v == 1);
    // invalid arguments are refused
    CHECK(harp_tessellate(x.data(), y.data(), n_ant, 0.0, r_ext, ox, oy, &nc, &nm, nullptr, nullptr, nullptr,
                          nullptr) == HARP_E_ARG);
    CHECK(harp_tessellate(x.data(), y.data(), n_ant, r_in, -1.0, ox, oy, &nc, &nm, nullptr, nullptr, nullptr,
                          nullptr) == HARP_E_ARG);
}

int main() {
    std::mt19937_64 rng(20170313);
    // batch plans: random sizes, single systems, tight batch limits, default
    // and custom costs, a system too large for the order limit
    const double cost[3] = {2e-5, 1e-6, 1e-13};
    for (int t = 0; t < 200; ++t) {
        std::uniform_int_distribution<int> nsys(1, 60), mb(1, 12), pm(1, 16);
        plan_case(rng, nsys(rng), 1, 520, 8, pm(rng), 8192, mb(rng), (t & 1) ? cost : nullptr);
    }
    plan_case(rng, 1, 5, 5, 4, 8, 8192, 1, nullptr);
    plan_case(rng, 30, 500, 520, 8, 8, 2048, 4, nullptr);   // every system beyond max_order
    {
        int32_t na = 3, order = 0, gb[2], gp = 0, ng = 0;
        CHECK(harp_batch_plan(&na, 0, 8, 8, 8192, 4, nullptr, &order, gb, &gp, &ng) == HARP_E_ARG);
        const double bad[3] = {-1.0, 0.0, 0.0};
        CHECK(harp_batch_plan(&na, 1, 8, 8, 8192, 4, bad, &order, gb, &gp, &ng) == HARP_E_ARG);
    }
    // tessellations: random layouts, one antenna, large extension, offset origin
    for (int t = 0; t < 40; ++t) tess_case(rng, 1 + int(rng() % 400), 40.0, 3.0 + double(t % 5), 2.0 * (t % 4),
                                           0.3 * (t % 3), -0.7 * (t % 2));
    tess_case(rng, 1, 1.0, 6.0, 0.0, 0.0, 0.0);
    tess_case(rng, 50, 10.0, 6.0, 100.0, 0.0, 0.0);
    // oracle reaction sums: a random element of 3 MBFs x 7 samples
    const int nm = 3, ns = 7;
    std::normal_distribution<double> g(0.0, 1.0);
    std::vector<double> smp(size_t(nm) * ns * 8);
    for (int i = 0; i < nm * ns; ++i) {
        double* r = &smp[size_t(i) * 8];
        r[0] = 0.25 * g(rng);
        r[1] = 0.25 * g(rng);
        r[2] = std::fabs(g(rng));
        const bool z = (rng() & 1) != 0;
        r[3] = z ? 0.0 : 1.0;
        r[4] = 0.0;
        r[5] = z ? 1.0 : 0.0;
        r[6] = g(rng);
        r[7] = g(rng);
    }
    double dy[18];
    oracle_dyadic(2.1, 0.3, -1.2, 0.7, dy);
    for (double v : dy) CHECK(std::isfinite(v));
    double out[2], back[2];
    oracle_reaction(2.1, 790.0, ns, &smp[0], ns, &smp[size_t(ns) * 8], 3.0, 1.0, 0.0, 0.0, out);
    oracle_reaction(2.1, 790.0, ns, &smp[size_t(ns) * 8], ns, &smp[0], -3.0, -1.0, 0.0, 0.0, back);
    CHECK(std::isfinite(out[0]) && std::isfinite(out[1]));
    // reciprocity of the exact reaction
    CHECK(std::fabs(out[0] - back[0]) <= 1e-12 * std::fabs(out[0]) + 1e-300 &&
          std::fabs(out[1] - back[1]) <= 1e-12 * std::fabs(out[1]) + 1e-300);
    const int np = 5;
    std::vector<double> Rx(np), Ry(np), grid(size_t(np) * nm * nm * 2);
    for (int p = 0; p < np; ++p) {
        Rx[p] = 2.0 + p;
        Ry[p] = -1.0 + 0.5 * p;
    }
    oracle_reaction_grid(2.1, 790.0, nm, ns, smp.data(), np, Rx.data(), Ry.data(), 0.02, grid.data());
    for (double v : grid) CHECK(std::isfinite(v));
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("sanitize ok\n");
    return 0;
}
