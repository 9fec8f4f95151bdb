// Host side of libtbpm: validation, sliced-ELL build, Chebyshev/Bessel
// coefficients, the propagation driver (HIP graph replay of one time step)
// and the C ABI entry points declared in include/tbpm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "tbpm_engine.h"
#include "tbpm_internal.h"

namespace tbpm {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

const std::string &last_error() { return g_last_error; }

tbpm_status fail(tbpm_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

tbpm_status hip_fail(hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return fail(TBPM_E_OOM, m);
    return fail(TBPM_E_DEVICE, m);
}

// ---------------------------------------------------------------------------
// Bessel functions J_m(z), m = 0..M-1, by Miller's backward recurrence
// J_{m-1} = (2m/z) J_m - J_{m+1}, started far above max(M, |z|) and
// normalised with J_0 + 2 sum_{k>=1} J_{2k} = 1 (Abramowitz & Stegun 9.1.46;
// the method is A&S 9.12 / Miller 1952).  J_m(-z) = (-1)^m J_m(z).
// ---------------------------------------------------------------------------
void bessel_j(double z, int32_t M, double *J) {
    if (M <= 0) return;
    if (z == 0.0) {
        J[0] = 1.0;
        for (int32_t m = 1; m < M; ++m) J[m] = 0.0;
        return;
    }
    const double az = std::fabs(z);
    const double top = std::max<double>(M, az);
    int64_t L = (int64_t)(top + 40.0 + 10.0 * std::cbrt(top));
    if (L & 1) ++L;
    std::vector<double> j(L + 2, 0.0);
    double jp1 = 0.0, jm = 1e-280;  // J_{L+1}, J_L (unnormalised)
    j[L] = jm;
    double norm = (L % 2 == 0) ? 2.0 * jm : 0.0;
    for (int64_t m = L; m >= 1; --m) {
        double jm1 = (2.0 * (double)m / az) * jm - jp1;
        jp1 = jm;
        jm = jm1;
        j[m - 1] = jm;
        if (m - 1 > 0 && ((m - 1) % 2 == 0)) norm += 2.0 * jm;
        if (std::fabs(jm) > 1e250) {  // rescale everything kept so far
            for (int64_t q = m - 1; q <= L; ++q) j[q] *= 1e-250;
            jm *= 1e-250;
            jp1 *= 1e-250;
            norm *= 1e-250;
        }
    }
    norm += j[0];
    for (int32_t m = 0; m < M; ++m) {
        double v = j[m] / norm;
        if (z < 0 && (m & 1)) v = -v;
        J[m] = v;
    }
}

int32_t num_terms(double z, double tol) {
    const double az = std::fabs(z);
    int32_t span = (int32_t)az + 64;
    for (;;) {
        std::vector<double> J(span + 1);
        bessel_j(z, span + 1, J.data());
        for (int32_t m = (int32_t)std::floor(az) + 1; m <= span; ++m)
            if (std::fabs(J[m]) < tol) return std::max<int32_t>(3, m);
        span *= 2;
        if (span > 1 << 22) return -1;
    }
}

// ---------------------------------------------------------------------------
// transposed slots: for every stored element (r, c) of the sliced ELL, the
// slot of (c, r); -1 for padding slots (column = row).  Empty if an element
// has no transposed partner (H is validated Hermitian, so this does not
// happen for a handle's matrix).
// ---------------------------------------------------------------------------
std::vector<int32_t> ell_partner_slots(int64_t n_rows, const std::vector<int64_t> &slice_off,
                                       const std::vector<int32_t> &col) {
    std::vector<int32_t> part(col.size(), -1);
    if (col.size() >= (size_t)INT32_MAX) return {};
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t q = r / kSliceRows, off = slice_off[q] + r % kSliceRows;
        const int64_t w = (slice_off[q + 1] - slice_off[q]) / kSliceRows;
        for (int64_t k = 0; k < w; ++k) {
            const int64_t s = off + k * kSliceRows;
            const int64_t c = col[s];
            if (c == r) continue;
            const int64_t qc = c / kSliceRows, offc = slice_off[qc] + c % kSliceRows;
            const int64_t wc = (slice_off[qc + 1] - slice_off[qc]) / kSliceRows;
            int64_t found = -1;
            for (int64_t kk = 0; kk < wc && found < 0; ++kk)
                if (col[offc + kk * kSliceRows] == r) found = offc + kk * kSliceRows;
            if (found < 0) return {};
            part[s] = (int32_t)found;
        }
    }
    return part;
}

// ---------------------------------------------------------------------------
// sliced ELL
// ---------------------------------------------------------------------------
HostEll build_sliced_ell(int64_t n_rows, const int64_t *row_ptr, const int32_t *col) {
    HostEll e;
    const int64_t n_slices = (n_rows + kSliceRows - 1) / kSliceRows;
    e.slice_off.assign(n_slices + 1, 0);
    for (int64_t q = 0; q < n_slices; ++q) {
        int64_t w = 0;
        const int64_t r1 = std::min(n_rows, (q + 1) * kSliceRows);
        for (int64_t r = q * kSliceRows; r < r1; ++r) w = std::max(w, row_ptr[r + 1] - row_ptr[r]);
        e.slice_off[q + 1] = e.slice_off[q] + w * kSliceRows;
    }
    const int64_t size = e.slice_off[n_slices];
    e.col.assign(size, 0);
    e.csr_pos.assign(size, -1);
    for (int64_t q = 0; q < n_slices; ++q) {
        const int64_t w = (e.slice_off[q + 1] - e.slice_off[q]) / kSliceRows;
        for (int64_t lr = 0; lr < kSliceRows; ++lr) {
            const int64_t r = q * kSliceRows + lr;
            const int64_t len = r < n_rows ? row_ptr[r + 1] - row_ptr[r] : 0;
            for (int64_t k = 0; k < w; ++k) {
                const int64_t slot = e.slice_off[q] + k * kSliceRows + lr;
                if (k < len) {
                    e.col[slot] = col[row_ptr[r] + k];
                    e.csr_pos[slot] = row_ptr[r] + k;
                } else {
                    e.col[slot] = (int32_t)(r < n_rows ? r : 0);
                }
            }
        }
    }
    return e;
}

// ---------------------------------------------------------------------------
// host threads
// ---------------------------------------------------------------------------
// Host threads for a pass over `work` items: up to 16 from 2^20 items on,
// else one.
int host_threads(int64_t work) {
    if (work < ((int64_t)1 << 20)) return 1;
    return (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
}

// f(chunk, lo, hi) for `threads` contiguous chunks of [0, n), chunk k on its
// own thread (k = 0 on the calling thread).  An exception in a chunk is
// rethrown as std::bad_alloc once every chunk has ended.
void run_chunks(int64_t n, int threads, const std::function<void(int, int64_t, int64_t)> &f) {
    threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n));
    std::atomic<bool> failed{false};
    auto chunk = [&](int k) {
        try {
            f(k, n * k / threads, n * (k + 1) / threads);
        } catch (...) {
            failed.store(true);
        }
    };
    std::vector<std::thread> pool;
    pool.reserve(threads);  // only a thread that cannot be started throws below
    int k = 1;
    for (; k < threads; ++k) {
        try {
            pool.emplace_back(chunk, k);
        } catch (const std::system_error &) {
            break;
        }
    }
    chunk(0);
    for (; k < threads; ++k) chunk(k);  // chunks no thread could be started for
    for (std::thread &th : pool) th.join();
    if (failed.load()) throw std::bad_alloc();
}

// ---------------------------------------------------------------------------
// CSR validation and canonicalisation (merge duplicates, sort columns)
// ---------------------------------------------------------------------------
tbpm_status canonical_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                          const double *onsite, HostCsr &out) {
    if (n < 1 || n >= (int64_t)INT32_MAX) return fail(TBPM_E_ARG, "n_orb must be in [1, 2^31-1)");
    if (!row_ptr || !onsite) return fail(TBPM_E_ARG, "row_ptr and onsite must not be NULL");
    if (row_ptr[0] != 0) return fail(TBPM_E_CSR, "row_ptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i])
            return fail(TBPM_E_CSR, "row_ptr is not non-decreasing at row " + std::to_string(i));
    const int64_t nnz = row_ptr[n];
    if (nnz > 0 && (!col || !val)) return fail(TBPM_E_ARG, "col_idx and val must not be NULL when nnz > 0");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(onsite[i])) return fail(TBPM_E_ARG, "non-finite on-site energy at " + std::to_string(i));
    // rows in contiguous chunks, one per thread; each chunk notes its first
    // invalid entry, and the first chunk that has one reports it, so the
    // error is the one a pass in row order meets first
    const int threads = host_threads(nnz);
    struct Bad {
        int64_t row = -1, c = 0;
        int kind = 0;  // 1 column out of range, 2 diagonal, 3 non-finite
    };
    std::vector<Bad> bad(threads);
    run_chunks(n, threads, [&](int k, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i)
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                const int64_t c = col[p];
                const int kind = (c < 0 || c >= n) ? 1 : c == i ? 2
                                 : (!std::isfinite(val[2 * p]) || !std::isfinite(val[2 * p + 1])) ? 3 : 0;
                if (kind) {
                    bad[k] = Bad{i, c, kind};
                    return;
                }
            }
    });
    for (const Bad &b : bad) {
        if (b.row < 0) continue;
        if (b.kind == 1)
            return fail(TBPM_E_CSR, "column " + std::to_string(b.c) + " out of range in row " + std::to_string(b.row));
        if (b.kind == 2)
            return fail(TBPM_E_CSR, "diagonal entry in row " + std::to_string(b.row) +
                                        " (pass on-site energies in 'onsite')");
        return fail(TBPM_E_ARG, "non-finite matrix element in row " + std::to_string(b.row));
    }
    // sort each row by column (stable) and sum duplicate columns; chunks
    // build their rows apart and are then joined in row order
    struct Part {
        std::vector<int32_t> col;
        std::vector<double> val;
        std::vector<int64_t> len;
    };
    std::vector<Part> parts(threads);
    run_chunks(n, threads, [&](int k, int64_t lo, int64_t hi) {
        Part &pt = parts[k];
        pt.col.reserve(row_ptr[hi] - row_ptr[lo]);
        pt.val.reserve(2 * (row_ptr[hi] - row_ptr[lo]));
        pt.len.reserve(hi - lo);
        std::vector<std::pair<int32_t, int64_t>> tmp;
        for (int64_t i = lo; i < hi; ++i) {
            const size_t before = pt.col.size();
            tmp.clear();
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) tmp.emplace_back(col[p], p);
            std::stable_sort(tmp.begin(), tmp.end(),
                             [](const std::pair<int32_t, int64_t> &a, const std::pair<int32_t, int64_t> &b) {
                                 return a.first < b.first;
                             });
            for (size_t q = 0; q < tmp.size(); ++q) {
                const int64_t p = tmp[q].second;
                if (q > 0 && tmp[q].first == tmp[q - 1].first) {
                    pt.val[pt.val.size() - 2] += val[2 * p];
                    pt.val[pt.val.size() - 1] += val[2 * p + 1];
                } else {
                    pt.col.push_back(tmp[q].first);
                    pt.val.push_back(val[2 * p]);
                    pt.val.push_back(val[2 * p + 1]);
                }
            }
            pt.len.push_back((int64_t)(pt.col.size() - before));
        }
    });
    out.n = n;
    out.row_ptr.assign(n + 1, 0);
    {
        int64_t i = 0;
        for (const Part &pt : parts)
            for (int64_t l : pt.len) {
                out.row_ptr[i + 1] = out.row_ptr[i] + l;
                ++i;
            }
    }
    out.col.resize(out.row_ptr[n]);
    out.val.resize(2 * out.row_ptr[n]);
    run_chunks(n, threads, [&](int k, int64_t lo, int64_t) {
        std::copy(parts[k].col.begin(), parts[k].col.end(), out.col.begin() + out.row_ptr[lo]);
        std::copy(parts[k].val.begin(), parts[k].val.end(), out.val.begin() + 2 * out.row_ptr[lo]);
    });
    parts.clear();
    out.onsite.assign(onsite, onsite + n);
    double hmax = 0.0;
    return check_values(out, hmax);
}

tbpm_status check_values(HostCsr &h, double &hmax) {
    const int64_t n = h.n;
    const int threads = host_threads(h.nnz());
    // per chunk of rows: the largest |H_ij| and |eps_i|, whether any value is
    // complex, the first entry without a conjugate partner, the Gershgorin
    // row sums and the widest row; maxima and the flag do not depend on the
    // order they are taken in, and the first chunk with a bad entry reports
    // it, as a pass in row order would
    struct Acc {
        double hmax = 0.0, g = 0.0;
        int64_t mr = 0;
        bool cplx = false;
        int64_t bad_row = -1, bad_p = 0;
    };
    std::vector<Acc> acc(threads);
    run_chunks(n, threads, [&](int k, int64_t lo, int64_t hi) {
        Acc &a = acc[k];
        for (int64_t p = h.row_ptr[lo]; p < h.row_ptr[hi]; ++p) {
            a.hmax = std::max(a.hmax, std::hypot(h.val[2 * p], h.val[2 * p + 1]));
            if (h.val[2 * p + 1] != 0.0) a.cplx = true;
        }
        for (int64_t i = lo; i < hi; ++i) a.hmax = std::max(a.hmax, std::fabs(h.onsite[i]));
    });
    hmax = 0.0;
    bool cplx = false;
    for (const Acc &a : acc) {
        hmax = std::max(hmax, a.hmax);
        cplx = cplx || a.cplx;
    }
    const double tol = 1e-13 * hmax;
    // 0: no partner, 1: partner's value is not the conjugate
    std::vector<int> bad_kind(threads, 0);
    run_chunks(n, threads, [&](int k, int64_t lo, int64_t hi) {
        Acc &a = acc[k];
        for (int64_t i = lo; i < hi; ++i) {
            for (int64_t p = h.row_ptr[i]; p < h.row_ptr[i + 1]; ++p) {
                const int32_t j = h.col[p];
                const int32_t *b = h.col.data() + h.row_ptr[j];
                const int32_t *e = h.col.data() + h.row_ptr[j + 1];
                const int32_t *f = std::lower_bound(b, e, (int32_t)i);
                if (f == e || *f != i) {
                    a.bad_row = i;
                    a.bad_p = p;
                    bad_kind[k] = 0;
                    return;
                }
                const int64_t q = f - h.col.data();
                const double dr = h.val[2 * p] - h.val[2 * q];
                const double di = h.val[2 * p + 1] + h.val[2 * q + 1];
                if (std::hypot(dr, di) > tol) {
                    a.bad_row = i;
                    a.bad_p = p;
                    bad_kind[k] = 1;
                    return;
                }
            }
        }
    });
    for (int k = 0; k < threads; ++k) {
        const Acc &a = acc[k];
        if (a.bad_row < 0) continue;
        const std::string i = std::to_string(a.bad_row), j = std::to_string(h.col[a.bad_p]);
        if (bad_kind[k] == 0)
            return fail(TBPM_E_NOT_HERMITIAN,
                        "entry (" + i + "," + j + ") has no transposed partner (" + j + "," + i + ")");
        return fail(TBPM_E_NOT_HERMITIAN, "H(" + i + "," + j + ") != conj(H(" + j + "," + i + "))");
    }
    h.is_complex = cplx;
    run_chunks(n, threads, [&](int k, int64_t lo, int64_t hi) {
        Acc &a = acc[k];
        for (int64_t i = lo; i < hi; ++i) {
            double r = std::fabs(h.onsite[i]);
            for (int64_t p = h.row_ptr[i]; p < h.row_ptr[i + 1]; ++p) r += std::hypot(h.val[2 * p], h.val[2 * p + 1]);
            a.g = std::max(a.g, r);
            a.mr = std::max(a.mr, h.row_ptr[i + 1] - h.row_ptr[i]);
        }
    });
    double g = 0.0;
    int64_t mr = 0;
    for (const Acc &a : acc) {
        g = std::max(g, a.g);
        mr = std::max(mr, a.mr);
    }
    h.gershgorin = g;
    h.max_row = mr;
    return TBPM_OK;
}

// ---------------------------------------------------------------------------
// two-hop tile tables (fused launch shape)
// ---------------------------------------------------------------------------
bool two_hop_tables(const std::vector<int64_t> &slice_off, const std::vector<int32_t> &col,
                    const std::vector<int64_t> &inst_row0, int32_t log2u, int32_t unit_bytes, size_t budget,
                    TwoHopTables &t) {
    const int64_t SR = kSliceRows;
    const int32_t n_inst = (int32_t)inst_row0.size() - 1;
    auto width = [&](int64_t r) { return (slice_off[r / SR + 1] - slice_off[r / SR]) / SR; };
    auto slot_of = [&](int64_t r, int64_t k) { return slice_off[r / SR] + k * SR + r % SR; };
    auto outside = [](int32_t c, int64_t r0, int64_t rows) { return c < r0 || c >= r0 + rows; };
    // the 1-hop rows e1 and the 2-hop rows e2 of a tile, sorted (per thread)
    struct Halo {
        std::vector<int32_t> e1, e2;
    };
    auto collect = [&](Halo &hl, int64_t r0, int64_t rows) {
        std::vector<int32_t> &e1 = hl.e1, &e2 = hl.e2;
        e1.clear();
        e2.clear();
        for (int64_t r = r0; r < r0 + rows; ++r)
            for (int64_t k = 0, w = width(r); k < w; ++k) {
                const int32_t c = col[slot_of(r, k)];
                if (outside(c, r0, rows)) e1.push_back(c);
            }
        std::sort(e1.begin(), e1.end());
        e1.erase(std::unique(e1.begin(), e1.end()), e1.end());
        for (int32_t h : e1)
            for (int64_t k = 0, w = width(h); k < w; ++k) {
                const int32_t c = col[slot_of(h, k)];
                if (outside(c, r0, rows) && !std::binary_search(e1.begin(), e1.end(), c)) e2.push_back(c);
            }
        std::sort(e2.begin(), e2.end());
        e2.erase(std::unique(e2.begin(), e2.end()), e2.end());
    };
    // a tile fits if its two LDS arrays fit the budget: b_{j+1} on x rows and
    // b_j on y rows (local indices are 16-bit)
    auto fits = [&](const Halo &hl, int64_t rows) {
        const size_t x = (size_t)rows + hl.e1.size() + hl.e2.size(), y = (size_t)rows + hl.e1.size();
        return ((x + y) << log2u) * (size_t)unit_bytes <= budget && x <= 65535;
    };
    // tiles of R rows of one member, halved until they fit: the tiles that
    // start at the multiples of R are independent, so they are taken in
    // contiguous chunks on host threads, and each chunk's tiles are visited
    // (visit(chunk, halo, member, r0, rows)) in row order; false if a single
    // row does not fit
    struct Top {
        int32_t inst;
        int64_t r0, rows;
    };
    std::vector<Top> tops;
    const int threads = host_threads((int64_t)col.size());
    auto tiling = [&](int64_t R, int &n_chunks,
                      const std::function<void(int, const Halo &, int32_t, int64_t, int64_t)> &visit) {
        tops.clear();
        for (int32_t i = 0; i < n_inst; ++i)
            for (int64_t r0 = inst_row0[i]; r0 < inst_row0[i + 1]; r0 += R)
                tops.push_back(Top{i, r0, std::min<int64_t>(R, inst_row0[i + 1] - r0)});
        n_chunks = (int)std::max<int64_t>(1, std::min<int64_t>(threads, (int64_t)tops.size()));
        std::atomic<bool> ok{true};
        run_chunks((int64_t)tops.size(), n_chunks, [&](int k, int64_t lo, int64_t hi) {
            Halo hl;
            std::vector<std::pair<int64_t, int64_t>> st;
            for (int64_t q = lo; q < hi && ok.load(std::memory_order_relaxed); ++q) {
                st.push_back({tops[q].r0, tops[q].rows});
                while (!st.empty()) {
                    const auto [a, rows] = st.back();
                    st.pop_back();
                    collect(hl, a, rows);
                    if (!fits(hl, rows)) {
                        if (rows == 1) {
                            ok.store(false);
                            return;
                        }
                        st.push_back({a + rows / 2, rows - rows / 2});
                        st.push_back({a, rows / 2});
                        continue;
                    }
                    visit(k, hl, tops[q].inst, a, rows);
                }
            }
        });
        return ok.load();
    };
    // R: the target tile size with the least staged traffic per pair of orders
    // (x on own + 1-hop + 2-hop rows, psi and b_{j+2} on own + 1-hop rows, two
    // outputs on own rows); ties go to the larger R.  Each cost is a sum of
    // integers, exact in any order.
    t.R = 0;
    double best = 0;
    for (int64_t cand : {256, 128, 64, 32, 16, 8, 4, 2, 1}) {
        std::vector<double> part(threads, 0.0);
        int n_chunks = 1;
        const bool ok = tiling(cand, n_chunks, [&](int k, const Halo &hl, int32_t, int64_t, int64_t rows) {
            part[k] += (double)(rows + hl.e1.size() + hl.e2.size()) + 2.0 * (double)(rows + hl.e1.size()) +
                       2.0 * (double)rows;
        });
        double cost = 0;
        for (double c : part) cost += c;
        if (ok && (t.R == 0 || cost < best * (1 - 1e-9))) {
            t.R = cand;
            best = cost;
        }
        if (t.R != 0 && t.R >= 4 * cand) break;  // smaller targets only split more
    }
    if (t.R == 0) return false;
    // the tables of each chunk are built apart and joined in tile order; the
    // local indices of a slot (lidx) are written in place, each by the tile
    // that owns the slot's row
    struct Part {
        std::vector<TileDesc> tiles;
        std::vector<int32_t> ucol, n1, hw, usz;  // usz: ucol entries of each tile
        std::vector<int64_t> hsz;               // hidx entries of each tile
        std::vector<uint16_t> hidx;
        size_t max_x = 0, max_y = 0, max_xy = 0;
    };
    std::vector<Part> parts(threads);
    t.lidx.assign(std::max<size_t>(col.size(), 1), 0);
    int n_chunks = 1;
    tiling(t.R, n_chunks, [&](int k, const Halo &hl, int32_t i, int64_t r0, int64_t rows) {
        Part &pt = parts[k];
        const std::vector<int32_t> &e1 = hl.e1, &e2 = hl.e2;
        const int64_t n1 = (int64_t)e1.size();
        pt.max_x = std::max(pt.max_x, (size_t)(rows + n1) + e2.size());
        pt.max_y = std::max(pt.max_y, (size_t)(rows + n1));
        pt.max_xy = std::max(pt.max_xy, (size_t)(2 * (rows + n1)) + e2.size());
        // local row numbering: own rows, then the 1-hop rows, then the 2-hop rows
        auto local = [&](int32_t c) -> uint16_t {
            if (!outside(c, r0, rows)) return (uint16_t)(c - r0);
            auto it = std::lower_bound(e1.begin(), e1.end(), c);
            if (it != e1.end() && *it == c) return (uint16_t)(rows + (it - e1.begin()));
            return (uint16_t)(rows + n1 + (std::lower_bound(e2.begin(), e2.end(), c) - e2.begin()));
        };
        for (int64_t r = r0; r < r0 + rows; ++r)
            for (int64_t k2 = 0, w = width(r); k2 < w; ++k2) t.lidx[slot_of(r, k2)] = local(col[slot_of(r, k2)]);
        int64_t hw = 0;
        for (int32_t h : e1) hw = std::max<int64_t>(hw, width(h));
        const size_t h0 = pt.hidx.size();
        pt.hw.push_back((int32_t)hw);
        for (int32_t h : e1) {
            const size_t at = pt.hidx.size();
            pt.hidx.resize(at + hw, 0);
            for (int64_t k2 = 0, w = width(h); k2 < w; ++k2) pt.hidx[at + k2] = local(col[slot_of(h, k2)]);
        }
        pt.hsz.push_back((int64_t)(pt.hidx.size() - h0));
        pt.ucol.insert(pt.ucol.end(), e1.begin(), e1.end());
        pt.ucol.insert(pt.ucol.end(), e2.begin(), e2.end());
        pt.usz.push_back((int32_t)(e1.size() + e2.size()));
        pt.n1.push_back((int32_t)n1);
        pt.tiles.push_back(TileDesc{r0, (int32_t)rows, i});
    });
    t.tiles.clear();
    t.inst_tile0.assign(n_inst + 1, 0);
    t.uoff.assign(1, 0);
    t.ucol.clear();
    t.n1.clear();
    t.hoff.clear();
    t.hw.clear();
    t.hidx.clear();
    t.max_x = t.max_y = t.max_xy = 0;
    for (int k = 0; k < n_chunks; ++k) {
        const Part &pt = parts[k];
        t.max_x = std::max(t.max_x, pt.max_x);
        t.max_y = std::max(t.max_y, pt.max_y);
        t.max_xy = std::max(t.max_xy, pt.max_xy);
        for (size_t q = 0; q < pt.tiles.size(); ++q) {
            t.hoff.push_back((int32_t)t.hidx.size());
            t.hidx.resize(t.hidx.size() + pt.hsz[q], 0);
            t.uoff.push_back((int32_t)(t.ucol.size() + pt.usz[q]));
            t.ucol.resize(t.ucol.size() + pt.usz[q]);
            t.tiles.push_back(pt.tiles[q]);
            t.inst_tile0[pt.tiles[q].inst + 1] = (int32_t)t.tiles.size();
        }
        t.n1.insert(t.n1.end(), pt.n1.begin(), pt.n1.end());
        t.hw.insert(t.hw.end(), pt.hw.begin(), pt.hw.end());
    }
    // copy each chunk's ucol and hidx into place
    {
        size_t u0 = 0, h0 = 0;
        for (int k = 0; k < n_chunks; ++k) {
            std::copy(parts[k].ucol.begin(), parts[k].ucol.end(), t.ucol.begin() + u0);
            std::copy(parts[k].hidx.begin(), parts[k].hidx.end(), t.hidx.begin() + h0);
            u0 += parts[k].ucol.size();
            h0 += parts[k].hidx.size();
        }
    }
    for (int32_t i = 0; i < n_inst; ++i) t.inst_tile0[i + 1] = std::max(t.inst_tile0[i + 1], t.inst_tile0[i]);
    if (t.ucol.size() >= (size_t)INT32_MAX || t.hidx.size() >= (size_t)INT32_MAX) return false;
    if (t.hidx.empty()) t.hidx.push_back(0);
    return true;
}

// ---------------------------------------------------------------------------
// locality order: recursive bisection of the row graph
// ---------------------------------------------------------------------------
std::vector<int32_t> bisection_order(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t leaf,
                                     int32_t max_threads) {
    std::vector<int32_t> order(n);
    for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
    // The parts of one level of the recursion are disjoint sets of rows, and
    // each part is reordered inside its own range of `order`, so the parts of
    // a level are processed by several threads at once; the result does not
    // depend on which thread takes which part.  Per-row state (seen, du, dv)
    // is touched only for the rows of the part being processed.  `mark` is
    // also read for neighbour rows that belong to other parts, so it is
    // atomic; every part and every breadth-first search takes a tag of its
    // own, so a row of another part never carries the reader's tag.
    std::unique_ptr<std::atomic<int32_t>[]> mark(new std::atomic<int32_t>[std::max<int64_t>(n, 1)]());
    std::vector<int32_t> seen(n, 0), du(n, 0), dv(n, 0);
    std::atomic<int32_t> tags{0};
    struct Scratch {
        std::vector<int32_t> q, rank;
    };
    // breadth-first order of the part (rows tagged `stamp`) from s, then from
    // the first unvisited row of each remaining piece, with the level of every
    // row in dist (pieces after the first continue the level count); returns
    // the last row
    auto bfs = [&](Scratch &w, int32_t stamp, int32_t s, int64_t lo, int64_t hi, std::vector<int32_t> &dist) {
        const int32_t visit = tags.fetch_add(1, std::memory_order_relaxed) + 1;
        std::vector<int32_t> &q = w.q;
        q.clear();
        int64_t next = lo;
        int32_t base = 0;
        while ((int64_t)q.size() < hi - lo) {
            if (q.size() > 0 || seen[s] == visit) {
                while (seen[order[next]] == visit) ++next;
                s = order[next];
                base = dist[q.back()] + 1;
            }
            seen[s] = visit;
            dist[s] = base;
            q.push_back(s);
            for (size_t h = q.size() - 1; h < q.size(); ++h)
                for (int64_t p = row_ptr[q[h]]; p < row_ptr[q[h] + 1]; ++p) {
                    const int32_t c = col[p];
                    if (mark[c].load(std::memory_order_relaxed) == stamp && seen[c] != visit) {
                        seen[c] = visit;
                        dist[c] = dist[q[h]] + 1;
                        q.push_back(c);
                    }
                }
        }
        return q.back();
    };
    // one part: reorder [lo, hi) and return the split point, or -1 when the
    // part is not split further
    auto part = [&](Scratch &w, int64_t lo, int64_t hi) -> int64_t {
        if (hi - lo < 2) return -1;
        const int32_t stamp = tags.fetch_add(1, std::memory_order_relaxed) + 1;
        for (int64_t k = lo; k < hi; ++k) mark[order[k]].store(stamp, std::memory_order_relaxed);
        // pseudo-peripheral rows u (reached last from the first row) and v
        // (reached last from u)
        const int32_t u = bfs(w, stamp, order[lo], lo, hi, du);
        const int32_t v = bfs(w, stamp, u, lo, hi, du);
        std::copy(w.q.begin(), w.q.end(), order.begin() + lo);
        if (hi - lo <= std::max<int64_t>(leaf, 2)) return -1;
        // split along the bisector of u and v: rows ordered by
        // d(u, r) - d(v, r) (ties in breadth-first order from u), so the cut
        // runs straight across the part rather than along a level of one
        // breadth-first search
        bfs(w, stamp, v, lo, hi, dv);
        // counting sort on the integer key (stable, so ties keep the order from u)
        int32_t kmin = INT32_MAX, kmax = INT32_MIN;
        for (int64_t k = lo; k < hi; ++k) {
            const int32_t key = du[order[k]] - dv[order[k]];
            kmin = std::min(kmin, key);
            kmax = std::max(kmax, key);
        }
        std::vector<int32_t> &rank = w.rank;
        rank.assign((size_t)(kmax - kmin) + 2, 0);
        for (int64_t k = lo; k < hi; ++k) ++rank[(size_t)(du[order[k]] - dv[order[k]] - kmin) + 1];
        for (size_t b = 1; b < rank.size(); ++b) rank[b] += rank[b - 1];
        w.q.assign(hi - lo, 0);
        for (int64_t k = lo; k < hi; ++k) w.q[rank[(size_t)(du[order[k]] - dv[order[k]] - kmin)]++] = order[k];
        std::copy(w.q.begin(), w.q.end(), order.begin() + lo);
        return lo + (hi - lo) / 2;
    };
    // threads for large graphs only (at most 16; one below 2^16 rows)
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int n_threads = max_threads > 0 ? max_threads : (n >= (1 << 16) ? (int)std::min(16u, hw) : 1);
    std::vector<std::pair<int64_t, int64_t>> level{{0, n}}, next;
    while (!level.empty()) {
        next.assign(2 * level.size(), {0, 0});
        std::atomic<size_t> at{0};
        std::atomic<bool> failed{false};
        // an exception must not leave a worker thread: it is recorded, and
        // the calling thread throws once every worker has ended
        auto run = [&]() {
            try {
                Scratch w;
                for (size_t k = at.fetch_add(1); k < level.size() && !failed.load(); k = at.fetch_add(1)) {
                    const auto [lo, hi] = level[k];
                    const int64_t mid = part(w, lo, hi);
                    if (mid >= 0) {
                        next[2 * k] = {lo, mid};
                        next[2 * k + 1] = {mid, hi};
                    }
                }
            } catch (...) {
                failed.store(true);
            }
        };
        const int t = (int)std::min<size_t>((size_t)n_threads, level.size());
        std::vector<std::thread> pool;
        pool.reserve(t);  // only a thread that cannot be started throws below
        for (int i = 1; i < t; ++i) {
            try {
                pool.emplace_back(run);
            } catch (const std::system_error &) {
                break;  // fewer threads: the calling thread still takes every remaining part
            }
        }
        run();
        for (std::thread &th : pool) th.join();
        if (failed.load()) throw std::bad_alloc();
        level.clear();
        for (const auto &pr : next)
            if (pr.second - pr.first >= 2) level.push_back(pr);
    }
    return order;
}


// ---------------------------------------------------------------------------
// Chebyshev coefficients of the Fermi-Dirac operator (Sec. "Tight-binding
// propagation method", decomposition of other operators): the discrete
// Fourier sum c_k = (2/N) Re sum_n g(cos(2 pi n/N)) e^{i 2 pi n k/N} of
// g(x) = 1/(exp(beta (rescale x - mu)) + 1), a_0 = c_0/2, a_k = c_k, with N
// doubled until the coefficients kept (up to the last |a_k| >= tol) use less
// than an eighth of the sum's length.
// ---------------------------------------------------------------------------
static void fft_inplace(std::vector<std::complex<double>> &z, bool inverse_sign) {
    const size_t n = z.size();
    for (size_t i = 1, j = 0; i < n; ++i) {  // bit reversal
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(z[i], z[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = (inverse_sign ? 2.0 : -2.0) * M_PI / (double)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> w(std::cos(ang * (double)k), std::sin(ang * (double)k));
                const std::complex<double> u = z[i + k], t = w * z[i + k + len / 2];
                z[i + k] = u + t;
                z[i + k + len / 2] = u - t;
            }
    }
}

std::vector<double> fermi_cheb_coeffs(double beta, double mu, double rescale, double tol) {
    for (size_t n = 1024; n <= (size_t(1) << 22); n <<= 1) {
        std::vector<std::complex<double>> z(n);
        for (size_t q = 0; q < n; ++q) {
            const double x = rescale * std::cos(2.0 * M_PI * (double)q / (double)n);
            z[q] = 0.5 * (1.0 - std::tanh(0.5 * beta * (x - mu)));  // overflow-free Fermi function
        }
        fft_inplace(z, true);  // sum_n g_n e^{+i 2 pi n k / N}
        std::vector<double> a(n / 2);
        for (size_t k = 0; k < n / 2; ++k) a[k] = 2.0 * z[k].real() / (double)n;
        a[0] *= 0.5;
        size_t K = 1;
        for (size_t k = 0; k < a.size(); ++k)
            if (std::fabs(a[k]) >= tol) K = k + 1;
        if (K < n / 8) {
            a.resize(K);
            return a;
        }
    }
    return {};
}
}  // namespace tbpm
