// Host-side sweep of the CSR ingest, the sliced-ELL build and the row order
// (built by tests/test_host_sanitize.py with AddressSanitizer and UBSan; no
// GPU involved): random Hermitian patterns with duplicate entries, unsorted
// rows, complex values and, now and then, an out-of-range column that must be
// rejected.  The row order must not depend on the number of host threads
// that build it: every pattern is also ordered on three threads, and two
// graphs above the threading threshold (a periodic square lattice and a
// random graph of four components with isolated rows) on 1, 2, 5 and 16
// threads and on the automatic count.  Prints "ok <accepted> rejected
// <rejected> orders <checks passed>" (3: the two orders and the large
// pattern below, whose ingest runs on several threads).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <random>
#include <vector>
#include "../paper_2209_00806_amd/csrc/tbpm_engine.h"
using namespace tbpm;
static bool is_perm(const std::vector<int32_t> &perm, int64_t n) {
    if ((int64_t)perm.size() != n) return false;
    std::vector<char> seen(n, 0);
    for (int32_t p : perm) {
        if (p < 0 || p >= n || seen[p]) return false;
        seen[p] = 1;
    }
    return true;
}
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
        const int32_t leaf = 1 + (int32_t)(g() % 40);
        std::vector<int32_t> perm = bisection_order(h.n, h.row_ptr.data(), h.col.data(), leaf);
        if (!is_perm(perm, h.n)) { std::printf("bad perm\n"); return 1; }
        if (bisection_order(h.n, h.row_ptr.data(), h.col.data(), leaf, 3) != perm) {
            std::printf("order depends on the thread count (trial %d)\n", trial);
            return 1;
        }
        ++ok;
        (void)e;
    }
    int orders = 0;
    for (int graph = 0; graph < 2; ++graph) {
        std::vector<int64_t> rp;
        std::vector<int32_t> col;
        if (graph == 0) {  // periodic 320 x 320 square lattice
            const int32_t L = 320;
            rp.push_back(0);
            for (int32_t y = 0; y < L; ++y)
                for (int32_t x = 0; x < L; ++x) {
                    const int32_t nb[4] = {y * L + (x + L - 1) % L, y * L + (x + 1) % L, ((y + L - 1) % L) * L + x,
                                           ((y + 1) % L) * L + x};
                    std::vector<int32_t> r(nb, nb + 4);
                    std::sort(r.begin(), r.end());
                    col.insert(col.end(), r.begin(), r.end());
                    rp.push_back((int64_t)col.size());
                }
        } else {  // four random components of 32768 rows, every 97th row isolated
            const int32_t n = 131072, blk = n / 4;
            std::vector<std::vector<int32_t>> adj(n);
            for (int q = 0; q < 3 * n; ++q) {
                const int32_t i = (int32_t)(g() % n), j = (i / blk) * blk + (int32_t)(g() % blk);
                if (i == j || i % 97 == 0 || j % 97 == 0) continue;
                adj[i].push_back(j);
                adj[j].push_back(i);
            }
            rp.push_back(0);
            for (auto &r : adj) {
                std::sort(r.begin(), r.end());
                r.erase(std::unique(r.begin(), r.end()), r.end());
                col.insert(col.end(), r.begin(), r.end());
                rp.push_back((int64_t)col.size());
            }
        }
        const int64_t n = (int64_t)rp.size() - 1;
        const std::vector<int32_t> ref = bisection_order(n, rp.data(), col.data(), 32, 1);
        if (!is_perm(ref, n)) { std::printf("bad perm\n"); return 1; }
        for (int32_t t : {2, 5, 16, 0})
            if (bisection_order(n, rp.data(), col.data(), 32, t) != ref) {
                std::printf("order of graph %d depends on the thread count (%d threads)\n", graph, t);
                return 1;
            }
        ++orders;
    }
    // a pattern large enough for the ingest to run on several threads:
    // duplicates and unsorted rows merged as in a single pass, the Gershgorin
    // bound and the widest row, and the first of two planted errors (in rows
    // far apart) reported, as a pass in row order meets them
    {
        const int64_t n = 200000;  // 1.2M stored entries: above the threading threshold of 2^20
        std::vector<std::vector<std::pair<int32_t, std::pair<double, double>>>> rows(n);
        for (int64_t q = 0; q < 3 * n; ++q) {
            const int32_t i = (int32_t)(g() % n), j = (int32_t)(g() % n);
            if (i == j) continue;
            const double re = ((int)(g() % 9) - 4) * 0.25, im = ((int)(g() % 3) - 1) * 0.5;
            rows[i].push_back({j, {re, im}});
            rows[j].push_back({i, {re, -im}});
        }
        std::vector<int64_t> rp(n + 1, 0);
        std::vector<int32_t> col;
        std::vector<double> val, ons(n);
        for (int64_t i = 0; i < n; ++i) {
            for (auto &e : rows[i]) {
                col.push_back(e.first);
                val.push_back(e.second.first);
                val.push_back(e.second.second);
            }
            rp[i + 1] = (int64_t)col.size();
            ons[i] = 0.01 * (double)(i % 7);
        }
        HostCsr h;
        if (canonical_csr(n, rp.data(), col.data(), val.data(), ons.data(), h) != TBPM_OK) {
            std::printf("large pattern rejected: %s\n", last_error().c_str());
            return 1;
        }
        double gmax = 0.0;
        int64_t widest = 0;
        for (int64_t i = 0; i < n; ++i) {
            // merged row: ascending columns, duplicates summed in input order
            std::vector<std::pair<int32_t, std::pair<double, double>>> r = rows[i];
            std::stable_sort(r.begin(), r.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
            std::vector<std::pair<int32_t, std::pair<double, double>>> m;
            for (auto &e : r) {
                if (!m.empty() && m.back().first == e.first) {
                    m.back().second.first += e.second.first;
                    m.back().second.second += e.second.second;
                } else {
                    m.push_back(e);
                }
            }
            if (h.row_ptr[i + 1] - h.row_ptr[i] != (int64_t)m.size()) {
                std::printf("large pattern: row %lld merged wrongly\n", (long long)i);
                return 1;
            }
            double rs = std::fabs(ons[i]);
            for (size_t k = 0; k < m.size(); ++k) {
                const int64_t p = h.row_ptr[i] + (int64_t)k;
                if (h.col[p] != m[k].first || h.val[2 * p] != m[k].second.first ||
                    h.val[2 * p + 1] != m[k].second.second) {
                    std::printf("large pattern: row %lld merged wrongly\n", (long long)i);
                    return 1;
                }
                rs += std::hypot(m[k].second.first, m[k].second.second);
            }
            gmax = std::max(gmax, rs);
            widest = std::max<int64_t>(widest, (int64_t)m.size());
        }
        if (h.gershgorin != gmax || h.max_row != widest || !h.is_complex) {
            std::printf("large pattern: bound or widest row wrong\n");
            return 1;
        }
        // a diagonal entry early and a column out of range late: the diagonal
        // comes first in row order
        const int64_t early = 1000, late = n - 1000;
        auto c2 = col;
        c2[rp[early]] = (int32_t)early;
        c2[rp[late]] = (int32_t)n;
        HostCsr h2;
        if (canonical_csr(n, rp.data(), c2.data(), val.data(), ons.data(), h2) != TBPM_E_CSR ||
            last_error().find("diagonal entry in row 1000 ") == std::string::npos) {
            std::printf("large pattern: wrong first error: %s\n", last_error().c_str());
            return 1;
        }
        // a value that breaks Hermiticity early and a missing partner late
        auto v2 = val;
        v2[2 * rp[early]] += 1.0;
        c2 = col;
        c2[rp[late]] = (int32_t)((col[rp[late]] + 1) % n == late ? (col[rp[late]] + 2) % n : (col[rp[late]] + 1) % n);
        HostCsr h3;
        if (canonical_csr(n, rp.data(), c2.data(), v2.data(), ons.data(), h3) != TBPM_E_NOT_HERMITIAN ||
            last_error().find("H(1000,") != 0) {
            std::printf("large pattern: wrong first Hermiticity error: %s\n", last_error().c_str());
            return 1;
        }
        ++orders;
    }
    std::printf("ok %d rejected %d orders %d\n", ok, rej, orders);
    return 0;
}
