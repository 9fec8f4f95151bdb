// Host-side check of the fused launch shape's tile tables and of the
// bisection row order (built by tests/test_host_tables.py against the
// library's host.cpp; no GPU involved).
//
//   host_tables_check <row_ptr.bin> <col.bin> <val.bin> <inst_row0.bin> <order> <log2u> <unit_bytes> <tier>
//
// order 1 renumbers every member by bisection_order (as the library does)
// and checks that the result is a permutation.  The tables are then built by
// two_hop_tables, and a pair of Clenshaw orders is evaluated through them
// with the indexing of the fused kernel (staged rows, local indices, per-tile
// LDS layout), every index checked against its array, and compared with two
// orders computed directly from the CSR.  Exit status 0 and "OK" on success.
#include <algorithm>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <random>
#include <vector>

#include "../paper_2209_00806_amd/csrc/tbpm_internal.h"

using namespace tbpm;
using cd = std::complex<double>;

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAILED: %s (line %d)\n", #c, __LINE__);   \
            std::exit(1);                                          \
        }                                                          \
    } while (0)

template <class T>
static std::vector<T> read_all(const char *path) {
    std::ifstream f(path, std::ios::binary);
    f.seekg(0, std::ios::end);
    const size_t n = (size_t)f.tellg() / sizeof(T);
    f.seekg(0);
    std::vector<T> v(n);
    f.read(reinterpret_cast<char *>(v.data()), (std::streamsize)(n * sizeof(T)));
    return v;
}

int main(int argc, char **argv) {
    if (argc != 9) {
        std::printf("usage: host_tables_check rp col val inst order log2u unit_bytes tier\n");
        return 2;
    }
    std::vector<int64_t> rp = read_all<int64_t>(argv[1]);
    std::vector<int32_t> col = read_all<int32_t>(argv[2]);
    std::vector<double> val = read_all<double>(argv[3]);
    const std::vector<int64_t> inst = read_all<int64_t>(argv[4]);
    const int order = std::atoi(argv[5]), log2u = std::atoi(argv[6]), unit_bytes = std::atoi(argv[7]),
              tier = std::atoi(argv[8]);
    const int64_t N = (int64_t)rp.size() - 1, U = int64_t(1) << log2u;
    CHECK(inst.front() == 0 && inst.back() == N);

    if (order == 1) {
        // renumber each member on its own, as the library does
        std::vector<int32_t> perm(N), inv(N, -1);
        for (size_t m = 0; m + 1 < inst.size(); ++m) {
            const int64_t r0 = inst[m], n = inst[m + 1] - r0;
            std::vector<int64_t> mrp(n + 1, 0);
            std::vector<int32_t> mcol;
            for (int64_t r = 0; r < n; ++r) {
                for (int64_t p = rp[r0 + r]; p < rp[r0 + r + 1]; ++p) {
                    CHECK(col[p] >= r0 && col[p] < r0 + n);
                    mcol.push_back((int32_t)(col[p] - r0));
                }
                mrp[r + 1] = (int64_t)mcol.size();
            }
            const std::vector<int32_t> mp = bisection_order(n, mrp.data(), mcol.data(), 32);
            CHECK((int64_t)mp.size() == n);
            for (int64_t i = 0; i < n; ++i) {
                CHECK(mp[i] >= 0 && mp[i] < n);
                CHECK(inv[r0 + mp[i]] < 0);
                inv[r0 + mp[i]] = (int32_t)(r0 + i);
                perm[r0 + i] = (int32_t)(r0 + mp[i]);
            }
        }
        std::vector<int64_t> rp2(N + 1, 0);
        std::vector<int32_t> c2;
        std::vector<double> v2;
        for (int64_t i = 0; i < N; ++i) {
            std::vector<std::pair<int32_t, double>> row;
            for (int64_t p = rp[perm[i]]; p < rp[perm[i] + 1]; ++p) row.push_back({inv[col[p]], val[p]});
            std::sort(row.begin(), row.end());
            for (const auto &e : row) {
                c2.push_back(e.first);
                v2.push_back(e.second);
            }
            rp2[i + 1] = (int64_t)c2.size();
        }
        rp.swap(rp2);
        col.swap(c2);
        val.swap(v2);
    }

    const HostEll e = build_sliced_ell(N, rp.data(), col.data());
    const int64_t ES = (int64_t)e.col.size();
    std::vector<double> ev(ES, 0.0);
    for (int64_t q = 0; q < ES; ++q)
        if (e.csr_pos[q] >= 0) ev[q] = val[e.csr_pos[q]];
    const std::vector<int64_t> inst_row0(inst.begin(), inst.end());
    const size_t budget = fused_lds_budget(tier);
    TwoHopTables t;
    if (!two_hop_tables(e.slice_off, e.col, inst_row0, log2u, unit_bytes, budget, t)) {
        std::printf("NOFIT\n");
        return 3;
    }
    const int64_t lds_units = (int64_t)t.max_xy << log2u;
    CHECK(lds_units * unit_bytes <= (int64_t)budget);
    CHECK(t.inst_tile0.size() == inst.size() && t.inst_tile0.back() == (int32_t)t.tiles.size());
    CHECK(t.uoff.size() == t.tiles.size() + 1 && t.n1.size() == t.tiles.size());

    std::mt19937_64 g(7);
    std::normal_distribution<double> nd;
    std::vector<cd> x(N * U), v(N * U), b2(N * U);
    std::vector<double> ons(N);
    for (auto &z : x) z = cd(nd(g), nd(g));
    for (auto &z : v) z = cd(nd(g), nd(g));
    for (auto &z : b2) z = cd(nd(g), nd(g));
    for (auto &o : ons) o = nd(g);
    const cd a1(0.3, -0.2), be1(0.7, 0.1), a2(-0.4, 0.5), be2(0.2, -0.6);
    auto hx = [&](const std::vector<cd> &in, int64_t r, int64_t s) {
        cd acc = ons[r] * in[r * U + s];
        for (int64_t p = rp[r]; p < rp[r + 1]; ++p) acc += val[p] * in[(int64_t)col[p] * U + s];
        return acc;
    };
    double worst = 0;
    std::vector<int64_t> covered(N, 0);
    for (int first = 0; first <= 1; ++first) {
        const std::vector<cd> &xx = first ? v : x;
        std::vector<cd> bj(N * U), bjm(N * U);
        for (int64_t r = 0; r < N; ++r)
            for (int64_t s = 0; s < U; ++s)
                bj[r * U + s] = a1 * (first ? xx[r * U + s] : v[r * U + s]) + be1 * hx(xx, r, s) -
                                (first ? cd(0) : b2[r * U + s]);
        for (int64_t r = 0; r < N; ++r)
            for (int64_t s = 0; s < U; ++s)
                bjm[r * U + s] = a2 * v[r * U + s] + be2 * hx(bj, r, s) - (first ? cd(0) : xx[r * U + s]);
        std::vector<cd> out1(N * U, cd(NAN, NAN)), out2(N * U, cd(NAN, NAN));
        std::vector<cd> lds(lds_units);
        const uint32_t umask = (uint32_t)U - 1;
        for (size_t tile = 0; tile < t.tiles.size(); ++tile) {
            const TileDesc td = t.tiles[tile];
            const uint32_t n_own = (uint32_t)td.rows, row0 = (uint32_t)td.row0;
            CHECK(td.rows > 0 && td.row0 >= inst[td.inst] && td.row0 + td.rows <= inst[td.inst + 1]);
            const int32_t e_beg = t.uoff[tile], e_end = t.uoff[tile + 1];
            const uint32_t n1 = (uint32_t)t.n1[tile];
            CHECK(e_beg <= e_end && e_end <= (int32_t)t.ucol.size() && n1 <= (uint32_t)(e_end - e_beg));
            const uint32_t n_x = (n_own + (uint32_t)(e_end - e_beg)) << log2u, n_y = (n_own + n1) << log2u;
            CHECK(n_x + n_y <= lds_units);
            cd *xs = lds.data(), *ys = lds.data() + n_x;
            const int32_t hoff = t.hoff[tile], hw = t.hw[tile];
            auto grow_of = [&](uint32_t lr) -> uint32_t {
                if (lr < n_own) return row0 + lr;
                CHECK(e_beg + (int64_t)(lr - n_own) < e_end);
                const int32_t r = t.ucol[e_beg + lr - n_own];
                CHECK(r >= inst[td.inst] && r < inst[td.inst + 1]);
                return (uint32_t)r;
            };
            for (uint32_t i = 0; i < n_x; ++i) {
                const uint64_t gi = ((uint64_t)grow_of(i >> log2u) << log2u) + (i & umask);
                CHECK(gi < (uint64_t)(N * U));
                xs[i] = xx[gi];
            }
            for (uint32_t u = 0; u < n_y; ++u) {
                const uint32_t lr = u >> log2u, grow = grow_of(lr), gu = (grow << log2u) + (u & umask);
                const uint32_t sl = grow / kSliceRows;
                CHECK(sl + 1 < e.slice_off.size());
                const uint32_t off = (uint32_t)e.slice_off[sl];
                const int w = (int)((e.slice_off[sl + 1] - off) / kSliceRows);
                const uint32_t base = off + grow % kSliceRows;
                const bool own = lr < n_own;
                cd acc = ons[grow] * xs[u];
                for (int k = 0; k < w; ++k) {
                    const uint32_t slot = base + (uint32_t)k * kSliceRows;
                    CHECK(slot < (uint32_t)ES);
                    uint32_t l;
                    if (own) {
                        l = t.lidx[slot];
                    } else {
                        const int64_t hi = hoff + (int64_t)(lr - n_own) * hw + k;
                        CHECK(k < hw && hi < (int64_t)t.hidx.size());
                        l = t.hidx[hi];
                    }
                    const uint32_t li = (l << log2u) + (u & umask);
                    CHECK(li < n_x);
                    CHECK(grow_of(l) == (uint32_t)e.col[slot]);  // the staged row is the slot's column
                    acc += ev[slot] * xs[li];
                }
                const cd src = first ? xs[u] : v[gu];
                cd o = a1 * src + be1 * acc;
                if (!first) o -= b2[gu];
                ys[u] = o;
                if (own) out1[gu] = o;
            }
            for (uint32_t u = 0; u < (n_own << log2u); ++u) {
                const uint32_t lr = u >> log2u, row = row0 + lr, gu = (row << log2u) + (u & umask);
                const uint32_t sl = row / kSliceRows, off = (uint32_t)e.slice_off[sl];
                const int w = (int)((e.slice_off[sl + 1] - off) / kSliceRows);
                const uint32_t base = off + row % kSliceRows;
                cd acc = ons[row] * ys[u];
                for (int k = 0; k < w; ++k) {
                    const uint32_t slot = base + (uint32_t)k * kSliceRows;
                    const uint32_t li = ((uint32_t)t.lidx[slot] << log2u) + (u & umask);
                    CHECK(li < n_y);
                    acc += ev[slot] * ys[li];
                }
                const cd vv = first ? xs[u] : v[gu];
                cd o = a2 * vv + be2 * acc;
                if (!first) o -= xs[u];
                out2[gu] = o;
                if (first && (u & umask) == 0) ++covered[row];
            }
        }
        for (int64_t q = 0; q < N * U; ++q) {
            worst = std::max(worst, std::abs(out1[q] - bj[q]) / (1 + std::abs(bj[q])));
            worst = std::max(worst, std::abs(out2[q] - bjm[q]) / (1 + std::abs(bjm[q])));
        }
    }
    for (int64_t r = 0; r < N; ++r) CHECK(covered[r] == 1);  // every row owned by exactly one tile
    std::printf("OK tiles=%zu R=%lld max_rows=%zu err=%.3e\n", t.tiles.size(), (long long)t.R, t.max_xy, worst);
    return worst < 1e-12 ? 0 : 1;
}
