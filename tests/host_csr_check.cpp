// Host-side sweep of the CSR ingest, the sliced-ELL build and the row order
// (built by tests/test_host_sanitize.py with AddressSanitizer and UBSan; no
// GPU involved): random Hermitian patterns with duplicate entries, unsorted
// rows, complex values and, now and then, an out-of-range column that must be
// rejected.  Prints "ok <accepted> rejected <rejected>".
#include <cstdio>
#include <random>
#include <vector>
#include "../paper_2209_00806_amd/csrc/tbpm_engine.h"
using namespace tbpm;
int main() {
    std::mt19937_64 g(7);
    int ok = 0, rej = 0;
    for (int trial = 0; trial < 400; ++trial) {
        const int64_t n = 1 + g() % 200;
        // symmetric pattern with conjugate values, duplicates and unsorted rows
        std::vector<std::vector<std::pair<int32_t, std::pair<double, double>>>> rows(n);
        const int pairs = (int)(g() % (3 * n + 1));
        for (int q = 0; q < pairs; ++q) {
            const int32_t i = (int32_t)(g() % n), j = (int32_t)(g() % n);
            if (i == j) continue;
            const double re = ((int)(g() % 5) - 2) * 0.5, im = (trial % 3 == 0) ? ((int)(g() % 3) - 1) * 0.25 : 0.0;
            rows[i].push_back({j, {re, im}});
            rows[j].push_back({i, {re, -im}});
        }
        std::vector<int64_t> rp(n + 1, 0);
        std::vector<int32_t> col;
        std::vector<double> val;
        for (int64_t i = 0; i < n; ++i) {
            for (auto &e : rows[i]) {
                int32_t c = e.first;
                if (trial % 11 == 0 && g() % 17 == 0) c = (int32_t)n;  // sometimes out of range
                col.push_back(c);
                val.push_back(e.second.first);
                val.push_back(e.second.second);
            }
            rp[i + 1] = (int64_t)col.size();
        }
        std::vector<double> ons(n, 0.1);
        HostCsr h;
        tbpm_status s = canonical_csr(n, rp.data(), col.empty() ? nullptr : col.data(), val.empty() ? nullptr : val.data(), ons.data(), h);
        if (s != TBPM_OK) { ++rej; continue; }
        double hmax = 0;
        s = check_values(h, hmax);
        if (s != TBPM_OK) { ++rej; continue; }
        HostEll e = build_sliced_ell(h.n, h.row_ptr.data(), h.col.data());
        std::vector<int32_t> perm = bisection_order(h.n, h.row_ptr.data(), h.col.data(), 1 + g() % 40);
        std::vector<char> seen(h.n, 0);
        for (int32_t p : perm) { if (p < 0 || p >= h.n || seen[p]) { std::printf("bad perm\n"); return 1; } seen[p] = 1; }
        ++ok;
        (void)e;
    }
    std::printf("ok %d rejected %d\n", ok, rej);
    return 0;
}
