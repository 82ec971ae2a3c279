// Host-only driver of the library's CPU-side logic, built with the address
// and undefined-behaviour sanitizers on the host code: the chunk planners
// (Alg. "chunker" and Alg. "chunkknl") on random row-pointer shapes and
// budgets, plan queries, host CSR validation, and the triangle-count
// relabelling on random symmetric graphs. No GPU call is made. Exit code 0
// when every checked property holds.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "../../include/mlspgemm.h"

static int fails = 0;
#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                 \
        }                                                            \
    } while (0)

static std::vector<int32_t> row_ptr(std::mt19937 &g, int n, int maxlen)
{
    std::vector<int32_t> rp(n + 1, 0);
    std::uniform_int_distribution<int> len(0, maxlen);
    for (int i = 0; i < n; ++i) rp[i + 1] = rp[i] + len(g);
    return rp;
}

static void planners(std::mt19937 &g)
{
    for (int it = 0; it < 300; ++it) {
        std::uniform_int_distribution<int> dn(0, 3000), dl(0, 40);
        const int nA = dn(g), nB = dn(g) + 1;
        auto arp = row_ptr(g, nA, dl(g)), brp = row_ptr(g, nB, dl(g)), crp = row_ptr(g, nA, dl(g) * 3);
        spgemm_csr A{nA, nB, arp[nA], arp.data(), nullptr, nullptr};
        spgemm_csr B{nB, 1000, brp[nB], brp.data(), nullptr, nullptr};
        const int64_t total = 4ll * (nA + 1) * 2 + 4ll * (nB + 1) + 12ll * (arp[nA] + brp[nB] + crp[nA]);
        std::uniform_real_distribution<double> fr(0.02, 3.0);
        std::uniform_int_distribution<int> nb(1, 4), mp(1, 6);
        const size_t budget = (size_t)(total * fr(g)) + (1u << 20);
        for (int knl = 0; knl < 2; ++knl) {
            spgemm_plan *plan = nullptr;
            const int nbuf = nb(g), minp = mp(g);
            spgemm_status st = knl ? spgemm_chunked_plan_knl(&A, &B, crp.data(), budget, nbuf, minp, &plan)
                                   : spgemm_chunked_plan(&A, &B, crp.data(), budget, nbuf, minp, &plan);
            CHECK(st == SPGEMM_OK || st == SPGEMM_ERR_BUDGET);
            if (st != SPGEMM_OK) { CHECK(plan == nullptr); continue; }
            spgemm_plan_info info;
            CHECK(spgemm_plan_info_get(plan, &info) == SPGEMM_OK);
            CHECK(info.ws_bytes <= (int64_t)budget);
            CHECK(info.algo == (knl ? 3 : info.algo) && info.algo >= 1 && info.algo <= 3);
            for (int which = 0; which < 2; ++which) {
                const int np = which == 0 ? info.n_ac_parts : info.n_b_parts;
                const int rows = which == 0 ? nA : nB;
                std::vector<int32_t> ranges(2 * (size_t)np);
                CHECK(spgemm_plan_parts(plan, which, ranges.data(), np) == SPGEMM_OK);
                int32_t at = 0;
                for (int p = 0; p < np; ++p) {   // contiguous cover of the rows
                    CHECK(ranges[2 * p] == at && ranges[2 * p + 1] >= at);
                    at = ranges[2 * p + 1];
                }
                CHECK(at == rows);
            }
            std::vector<spgemm_plan_step> steps(info.n_steps);
            CHECK(spgemm_plan_steps(plan, steps.data(), info.n_steps) == SPGEMM_OK);
            int64_t h2d = 0, d2h = 0;
            for (auto &s : steps) {
                CHECK(s.slot >= 0 && s.slot < info.nbuf_inner);
                if (s.kind == 0) h2d += s.bytes;
                if (s.kind == 1) d2h += s.bytes;
            }
            CHECK(h2d == info.h2d_bytes && d2h == info.d2h_bytes);
            spgemm_plan_destroy(plan);
        }
    }
}

static void validation(std::mt19937 &g)
{
    for (int it = 0; it < 300; ++it) {
        std::uniform_int_distribution<int> dn(0, 200);
        const int n = dn(g), m = dn(g) + 1;
        std::vector<int32_t> rp(n + 1, 0), ci;
        std::uniform_real_distribution<double> u(0, 1);
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < m; ++j)
                if (u(g) < 0.1) ci.push_back(j);
            rp[i + 1] = (int32_t)ci.size();
        }
        spgemm_csr M{n, m, (int64_t)ci.size(), rp.data(), ci.empty() ? nullptr : ci.data(), nullptr};
        CHECK(spgemm_validate_host(&M) == SPGEMM_OK);
        if (!ci.empty()) {   // plant one error
            std::vector<int32_t> bad = ci;
            std::uniform_int_distribution<size_t> at(0, bad.size() - 1);
            bad[at(g)] = (u(g) < 0.5) ? m : -1;
            spgemm_csr Mb{n, m, (int64_t)bad.size(), rp.data(), bad.data(), nullptr};
            CHECK(spgemm_validate_host(&Mb) == SPGEMM_ERR_BAD_CSR);
        }
    }
}

static void relabel(std::mt19937 &g)
{
    for (int it = 0; it < 100; ++it) {
        std::uniform_int_distribution<int> dn(0, 400);
        const int n = dn(g);
        std::vector<std::set<int>> adj(n);
        std::uniform_real_distribution<double> u(0, 1);
        const double p = u(g) * 0.1;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if (u(g) < p) { adj[i].insert(j); adj[j].insert(i); }
        std::vector<int32_t> rp(n + 1, 0), ci;
        for (int i = 0; i < n; ++i) {
            for (int j : adj[i]) ci.push_back(j);
            rp[i + 1] = (int32_t)ci.size();
        }
        spgemm_csr G{n, n, (int64_t)ci.size(), rp.data(), ci.empty() ? nullptr : ci.data(), nullptr};
        std::vector<int32_t> perm(n > 0 ? n : 1), lrp(n + 1), lci(ci.size() / 2 + 1);
        int64_t nnzL = -1;
        CHECK(spgemm_tc_lower(&G, perm.data(), lrp.data(), lci.data(), &nnzL) == SPGEMM_OK);
        CHECK(nnzL == (int64_t)ci.size() / 2);
        std::vector<int> seen(n, 0);
        for (int i = 0; i < n; ++i) { CHECK(perm[i] >= 0 && perm[i] < n); if (perm[i] >= 0 && perm[i] < n) seen[perm[i]]++; }
        for (int i = 0; i < n; ++i) CHECK(seen[i] == 1);
        for (int i = 0; i < n; ++i)
            for (int q = lrp[i]; q < lrp[i + 1]; ++q) CHECK(lci[q] < i && (q == lrp[i] || lci[q] > lci[q - 1]));
    }
}

int main()
{
    std::mt19937 g(12345);
    planners(g);
    validation(g);
    relabel(g);
    std::printf("host driver: %d failed checks\n", fails);
    return fails == 0 ? 0 : 1;
}
