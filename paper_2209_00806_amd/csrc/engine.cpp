// Propagation driver of libtbpm.
//
// A time step is the Clenshaw evaluation of psi' = sum_{m<M} c_m T_m(H/f) psi
// (paper, Eq. (eq:psi_t); c_0 = J_0(z), c_m = 2(-i)^m J_m(z), z = f dt):
//   b_{M-2} = c_{M-2} v + 2 c_{M-1} H~ v                      (first pass, x = v)
//   b_{M-3} = (c_{M-3} - c_{M-1}) v + 2 H~ b_{M-2}            (b_{M-1} = c_{M-1} v folded in)
//   b_j     = c_j v + 2 H~ b_{j+1} - b_{j+2},   j = M-4 .. 1
//   psi'    = c_0 v + H~ b_1 - b_2                            (+ C_{k+1}, ||psi'||^2)
// i.e. M-1 sparse passes over three state-sized buffers (v, A, B): every pass
// writes its output over a buffer that only the same element reads.  The
// passes of one step and the correlation reduce are captured once in a HIP
// graph and replayed N_t - 1 times; a device step counter tells the reduce
// which C_k it is producing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "tbpm_engine.h"

namespace tbpm {

using cd = std::complex<double>;

// time steps per replayed graph
constexpr int32_t kStepsPerGraph = 16;

hipError_t DevBuf::ensure(size_t need) {
    if (need <= bytes && ptr) return hipSuccess;
    if (ptr) {
        hipError_t e = hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
        if (e != hipSuccess) return e;
    }
    if (need == 0) need = 256;
    hipError_t e = hipMalloc(&ptr, need);
    if (e != hipSuccess) {
        ptr = nullptr;
        return e;
    }
    bytes = need;
    return hipSuccess;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

hipError_t PinnedBuf::ensure(size_t need) {
    if (need <= bytes && ptr) return hipSuccess;
    if (ptr) {
        (void)hipHostFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    need = std::max<size_t>(need, 4096);
    hipError_t e = hipHostMalloc(&ptr, need, hipHostMallocDefault);
    if (e != hipSuccess) {
        ptr = nullptr;
        return e;
    }
    bytes = need;
    return hipSuccess;
}

void PinnedBuf::release() {
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

bool GraphKey::operator==(const GraphKey &o) const {
    if (s_pad != o.s_pad || s_user != o.s_user || fp32 != o.fp32 || mmax != o.mmax || n_inst != o.n_inst ||
        chunks != o.chunks || remap != o.remap || nt != o.nt || unroll != o.unroll || staged != o.staged || vec != o.vec ||
        fused != o.fused || n_tiles != o.n_tiles || tiles_chunks != o.tiles_chunks || tiles_unit != o.tiles_unit ||
        lds_units != o.lds_units || n_steps != o.n_steps || n_qe != o.n_qe || jc_states != o.jc_states ||
        steps != o.steps || ckpt != o.ckpt)
        return false;
    for (size_t i = 0; i < sizeof(bufs) / sizeof(bufs[0]); ++i)
        if (bufs[i] != o.bufs[i]) return false;
    return true;
}

#define TRY_HIP(expr, what)                            \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ---------------------------------------------------------------------------
// upload of one or several merged CSR matrices as one block-diagonal operator
// ---------------------------------------------------------------------------
// Sum over tiles of 128 consecutive rows of the distinct rows outside the tile
// that its rows reference: the 1-hop halo a tile of the fused shape stages.
static double halo_cost(const HostCsr &h, const std::vector<int32_t> &perm, const std::vector<int32_t> &inv) {
    const int64_t T = 128;
    const int64_t n_tiles = (h.n + T - 1) / T;
    // tiles in chunks on host threads; the counts are integers, so the sum
    // does not depend on the chunking
    const int threads = host_threads(h.nnz());
    std::vector<int64_t> part(threads, 0);
    run_chunks(n_tiles, threads, [&](int k, int64_t lo, int64_t hi) {
        std::vector<int32_t> ext;
        for (int64_t t = lo; t < hi; ++t) {
            const int64_t t0 = t * T, t1 = std::min<int64_t>(h.n, t0 + T);
            ext.clear();
            for (int64_t r = t0; r < t1; ++r) {
                const int64_t src = perm.empty() ? r : perm[r];
                for (int64_t p = h.row_ptr[src]; p < h.row_ptr[src + 1]; ++p) {
                    const int32_t c = perm.empty() ? h.col[p] : inv[h.col[p]];
                    if (c < t0 || c >= t1) ext.push_back(c);
                }
            }
            std::sort(ext.begin(), ext.end());
            part[k] += std::unique(ext.begin(), ext.end()) - ext.begin();
        }
    });
    int64_t cost = 0;
    for (int64_t c : part) cost += c;
    return (double)cost;
}

// Row order of one member: empty = the caller's order.  mode 0 keeps it,
// 1 takes the bisection order, -1 takes the bisection order for members of
// at least kReorderMinRows rows when it cuts the halo cost by 15% or more.
static std::vector<int32_t> member_order(const HostCsr &h, int32_t mode) {
    constexpr int64_t kReorderMinRows = 16384;
    if (mode == 0 || h.n < 2 || (mode < 0 && h.n < kReorderMinRows)) return {};
    std::vector<int32_t> perm = bisection_order(h.n, h.row_ptr.data(), h.col.data(), 32);
    if (mode < 0) {
        std::vector<int32_t> inv(h.n);
        for (int64_t i = 0; i < h.n; ++i) inv[perm[i]] = (int32_t)i;
        if (halo_cost(h, perm, inv) > 0.85 * halo_cost(h, {}, {})) return {};
    }
    return perm;
}

// ---------------------------------------------------------------------------
// upload of one or several merged CSR matrices as one block-diagonal operator
// (each member's rows in its chosen order; values, on-site energies, states
// and gradients are mapped to and from the caller's order)
// ---------------------------------------------------------------------------
tbpm_status Engine::upload(const HostCsr *const *members, int32_t n, const std::vector<int32_t> *const *orders) {
    int dev = 0;
    TRY_HIP(hipGetDevice(&dev), "hipGetDevice");
    device = dev;
    inst_row0.assign(n + 1, 0);
    int64_t nnz_total = 0;
    bool cplx = false;
    for (int32_t i = 0; i < n; ++i) {
        inst_row0[i + 1] = inst_row0[i] + members[i]->n;
        nnz_total += members[i]->nnz();
        cplx = cplx || members[i]->is_complex;
    }
    const int64_t N = inst_row0[n];
    if (N >= (int64_t)INT32_MAX) return fail(TBPM_E_ARG, "total number of orbitals must be < 2^31");
    member_perm.assign(n, {});
    bool any_perm = false;
    for (int32_t i = 0; i < n; ++i) {
        member_perm[i] = orders ? *orders[i] : member_order(*members[i], row_order);
        any_perm = any_perm || !member_perm[i].empty();
    }
    // merged CSR in the internal order; src_pos = position in the caller's merged CSR
    std::vector<int64_t> rp(N + 1, 0);
    std::vector<int32_t> col;
    col.reserve(nnz_total);
    std::vector<double> val;
    val.reserve(2 * nnz_total);
    std::vector<int64_t> src_pos;
    src_pos.reserve(nnz_total);
    std::vector<double> ons(N);
    std::vector<int32_t> perm_all(any_perm ? N : 0);
    int64_t base = 0;
    std::vector<int32_t> inv;
    std::vector<std::pair<int32_t, int64_t>> row;
    for (int32_t i = 0; i < n; ++i) {
        const HostCsr &h = *members[i];
        const std::vector<int32_t> &pm = member_perm[i];
        const int64_t r0 = inst_row0[i];
        if (!pm.empty()) {
            inv.assign(h.n, 0);
            for (int64_t k = 0; k < h.n; ++k) inv[pm[k]] = (int32_t)k;
        }
        for (int64_t r = 0; r < h.n; ++r) {
            const int64_t src = pm.empty() ? r : pm[r];
            row.clear();
            for (int64_t p = h.row_ptr[src]; p < h.row_ptr[src + 1]; ++p)
                row.push_back({pm.empty() ? h.col[p] : inv[h.col[p]], p});
            if (!pm.empty()) std::sort(row.begin(), row.end());
            for (const auto &[c, p] : row) {
                col.push_back((int32_t)(c + r0));
                val.push_back(h.val[2 * p]);
                val.push_back(h.val[2 * p + 1]);
                src_pos.push_back(base + p);
            }
            rp[r0 + r + 1] = (int64_t)col.size();
            ons[r0 + r] = h.onsite[src];
            if (any_perm) perm_all[r0 + r] = (int32_t)src;
        }
        base += h.nnz();
    }
    HostEll e = build_sliced_ell(N, rp.data(), col.data());
    const int64_t S = (int64_t)e.col.size();
    h_slice_off = e.slice_off;
    h_col = e.col;
    partner_ready = false;
    std::vector<double> v64(cplx ? 2 * S : S, 0.0);
    std::vector<float> v32(cplx ? 2 * S : S, 0.0f);
    for (int64_t q = 0; q < S; ++q) {
        const int64_t p = e.csr_pos[q];
        if (p < 0) continue;
        const int64_t p_src = src_pos[p];
        e.csr_pos[q] = p_src;
        if (cplx) {
            v64[2 * q] = val[2 * p];
            v64[2 * q + 1] = val[2 * p + 1];
            v32[2 * q] = (float)val[2 * p];
            v32[2 * q + 1] = (float)val[2 * p + 1];
        } else {
            v64[q] = val[2 * p];
            v32[q] = (float)val[2 * p];
        }
    }
    std::vector<float> ons32(N);
    for (int64_t r = 0; r < N; ++r) ons32[r] = (float)ons[r];

    mat.n_rows = N;
    mat.n_slices = (int64_t)e.slice_off.size() - 1;
    mat.ell_size = S;
    mat.max_width = 0;
    int32_t min_width = INT32_MAX;
    for (int64_t q = 0; q < mat.n_slices; ++q) {
        const int32_t wq = (int32_t)((e.slice_off[q + 1] - e.slice_off[q]) / kSliceRows);
        mat.max_width = std::max<int32_t>(mat.max_width, wq);
        min_width = std::min<int32_t>(min_width, wq);
    }
    mat.uniform_w = (mat.n_slices > 0 && min_width == mat.max_width) ? mat.max_width : 0;
    mat.is_complex = cplx;
    const size_t vb = (cplx ? 2 : 1) * (size_t)std::max<int64_t>(S, 1);
    if (S >= (int64_t)UINT32_MAX) return fail(TBPM_E_ARG, "sliced-ELL size must be < 2^32 entries");
    std::vector<uint32_t> soff32(e.slice_off.begin(), e.slice_off.end());
    TRY_HIP(hipMalloc(&mat.slice_off, sizeof(uint32_t) * soff32.size()), "hipMalloc slice_off");
    TRY_HIP(hipMalloc(&mat.col, sizeof(int32_t) * std::max<int64_t>(S, 1)), "hipMalloc col");
    TRY_HIP(hipMalloc(&mat.val64, sizeof(double) * vb), "hipMalloc val64");
    TRY_HIP(hipMalloc(&mat.val32, sizeof(float) * vb), "hipMalloc val32");
    TRY_HIP(hipMalloc(&mat.onsite64, sizeof(double) * N), "hipMalloc onsite64");
    TRY_HIP(hipMalloc(&mat.onsite32, sizeof(float) * N), "hipMalloc onsite32");
    TRY_HIP(hipMalloc(&mat.ell_csr, sizeof(int64_t) * std::max<int64_t>(S, 1)), "hipMalloc ell_csr");
    TRY_HIP(hipMemcpy(mat.slice_off, soff32.data(), sizeof(uint32_t) * soff32.size(), hipMemcpyHostToDevice),
            "upload slice_off");
    if (S > 0) {
        TRY_HIP(hipMemcpy(mat.col, e.col.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice), "upload col");
        TRY_HIP(hipMemcpy(mat.val64, v64.data(), sizeof(double) * v64.size(), hipMemcpyHostToDevice), "upload val64");
        TRY_HIP(hipMemcpy(mat.val32, v32.data(), sizeof(float) * v32.size(), hipMemcpyHostToDevice), "upload val32");
        TRY_HIP(hipMemcpy(mat.ell_csr, e.csr_pos.data(), sizeof(int64_t) * S, hipMemcpyHostToDevice), "upload ell_csr");
    }
    TRY_HIP(hipMemcpy(mat.onsite64, ons.data(), sizeof(double) * N, hipMemcpyHostToDevice), "upload onsite");
    TRY_HIP(hipMemcpy(mat.onsite32, ons32.data(), sizeof(float) * N, hipMemcpyHostToDevice), "upload onsite32");
    if (any_perm) {
        TRY_HIP(hipMalloc(&mat.perm, sizeof(int32_t) * N), "hipMalloc perm");
        TRY_HIP(hipMemcpy(mat.perm, perm_all.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice), "upload perm");
    }
    TRY_HIP(hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking), "hipStreamCreate");
    TRY_HIP(hipEventCreateWithFlags(&staging_done, hipEventDisableTiming), "hipEventCreate");
    return TBPM_OK;
}

void Engine::release() {
    if (graph_exec || graph_exec1) {
        (void)hipDeviceSynchronize();
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph_exec1) (void)hipGraphExecDestroy(graph_exec1);
        graph_exec = graph_exec1 = nullptr;
    }
    void *ptrs[] = {mat.slice_off, mat.col, mat.val64, mat.val32, mat.onsite64, mat.onsite32, mat.ell_csr, mat.perm};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    mat = DevMatrix{};
    DevBuf *bufs[] = {&v,        &ba,        &bb,      &phi0,      &partials,  &counter,  &coef,
                      &norm2_all, &tiles,    &inst_tile0, &ptr_tab, &inst_row0_dev, &bwd_store, &bwd_adj,
                      &bwd_gacc, &bwd_gdiag, &bwd_coef, &st_uoff, &st_ucol, &st_lidx, &fu_n1, &fu_hoff,
                      &fu_hw,    &fu_hidx,  &bc,       &bd,        &ckpt_slot, &corr_scratch, &qe_coef,
                      &qe_acc,   &qe_part,  &qe_norm2, &ac_ja,     &ac_jb,     &ac_csr,       &ac_zero,
                      &ac_vec,   &ac_block, &jc_tab,   &jc_norm,   &hay_u,     &hay_y,        &hay_s,
                      &kp_store, &kp_rblk,  &kp_vec,   &kp_parts, &bwd_partner};
    for (DevBuf *b : bufs) b->release();
    partner_ready = false;
    staging.release();
    if (staging_done) (void)hipEventDestroy(staging_done);
    staging_done = nullptr;
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    capture_stream = nullptr;
}

// ---------------------------------------------------------------------------
// tiles: each workgroup handles 256*chunks state elements of one member
// ---------------------------------------------------------------------------
tbpm_status Engine::build_tiles(int32_t s_pad, int32_t chunks, int32_t vs) {
    if (tiles_s == s_pad && tiles_chunks == chunks && tiles_unit == -vs && tiles.ptr) return TBPM_OK;
    tiles_unit = -vs;
    // a chunk is one workgroup's worth of units (vs states each)
    const int64_t rows_per_tile = std::max<int64_t>(1, (int64_t)kWG * chunks * vs / s_pad);
    h_tiles.clear();
    h_inst_tile0.assign(n_inst() + 1, 0);
    for (int32_t i = 0; i < n_inst(); ++i) {
        for (int64_t r = inst_row0[i]; r < inst_row0[i + 1]; r += rows_per_tile) {
            TileDesc t;
            t.row0 = r;
            t.rows = (int32_t)std::min<int64_t>(rows_per_tile, inst_row0[i + 1] - r);
            t.inst = i;
            h_tiles.push_back(t);
        }
        h_inst_tile0[i + 1] = (int32_t)h_tiles.size();
    }
    if (h_tiles.size() >= (size_t)INT32_MAX) return fail(TBPM_E_ARG, "too many tiles");
    TRY_HIP(hipDeviceSynchronize(), "sync before tile rebuild");
    TRY_HIP(tiles.ensure(sizeof(TileDesc) * std::max<size_t>(h_tiles.size(), 1)), "alloc tiles");
    TRY_HIP(inst_tile0.ensure(sizeof(int32_t) * h_inst_tile0.size()), "alloc inst_tile0");
    TRY_HIP(hipMemcpy(tiles.ptr, h_tiles.data(), sizeof(TileDesc) * h_tiles.size(), hipMemcpyHostToDevice),
            "upload tiles");
    TRY_HIP(hipMemcpy(inst_tile0.ptr, h_inst_tile0.data(), sizeof(int32_t) * h_inst_tile0.size(),
                      hipMemcpyHostToDevice),
            "upload inst_tile0");
    tiles_s = s_pad;
    tiles_chunks = chunks;
    return TBPM_OK;
}

// ---------------------------------------------------------------------------
// staged tiles: runs of at most 256 consecutive rows of one member; the rows
// of x a tile reads are its own rows plus a sorted list of external rows, and
// the staged set fits the LDS budget of the tier (the fused shape's tiers:
// 1/(tier+2) of a CU's 160 KiB).
// ---------------------------------------------------------------------------
tbpm_status Engine::build_staged_tiles(int32_t s_pad, int32_t log2u, int32_t unit_bytes, int32_t tier) {
    // the tables depend on the bytes of a row and the tier only (not on how a
    // row is split into units)
    const int32_t key = (unit_bytes << log2u) * 8 + tier;
    if (tiles_s == s_pad && tiles_chunks < 0 && tiles_unit == key && tiles.ptr) {
        stage_units = (int32_t)(stage_max_rows << log2u);
        return TBPM_OK;
    }
    const size_t budget = fused_lds_budget(tier);
    const int64_t SR = kSliceRows;
    std::vector<int32_t> ext;
    auto collect = [&](int64_t r0, int64_t rows) {
        ext.clear();
        for (int64_t r = r0; r < r0 + rows; ++r) {
            const int64_t q = r / SR, w = (h_slice_off[q + 1] - h_slice_off[q]) / SR;
            for (int64_t k = 0; k < w; ++k) {
                const int32_t c = h_col[h_slice_off[q] + k * SR + r % SR];
                if (c < r0 || c >= r0 + rows) ext.push_back(c);
            }
        }
        std::sort(ext.begin(), ext.end());
        ext.erase(std::unique(ext.begin(), ext.end()), ext.end());
    };
    // Tiles are the parts of the recursive halving of each member's rows
    // whose staged rows (own rows and the distinct rows they reference) fit
    // the budget.  The bisection row order splits a part at its middle, so
    // these are parts of that bisection: compact regions with short borders
    // (a fixed tile height, set by the worst tile, stages several times the
    // rows of such a part on lattices with long-range hoppings).
    const size_t cap = budget / ((size_t)unit_bytes << log2u);
    std::vector<int64_t> seen(mat.n_rows, -1);
    int64_t visit = 0;
    auto stage_rows = [&](int64_t r0, int64_t rows) {
        ++visit;
        size_t cnt = 0;
        for (int64_t r = r0; r < r0 + rows; ++r) {
            if (seen[r] != visit) {
                seen[r] = visit;
                ++cnt;
            }
            const int64_t q = r / SR, w = (h_slice_off[q + 1] - h_slice_off[q]) / SR;
            for (int64_t k = 0; k < w; ++k) {
                const int32_t c = h_col[h_slice_off[q] + k * SR + r % SR];
                if (seen[c] != visit) {
                    seen[c] = visit;
                    ++cnt;
                }
            }
        }
        return cnt;
    };
    std::vector<std::pair<int64_t, int64_t>> parts, stack;
    for (int32_t i = 0; i < n_inst(); ++i) {
        stack.assign(1, {inst_row0[i], inst_row0[i + 1]});
        while (!stack.empty()) {
            const auto [lo, hi] = stack.back();
            stack.pop_back();
            if (hi <= lo) continue;
            if ((size_t)(hi - lo) <= std::min<size_t>(cap, 256) && stage_rows(lo, hi - lo) <= cap) {
                parts.push_back({lo, hi});
                continue;
            }
            if (hi - lo == 1) return fail(TBPM_E_ARG, "no staged tile fits the LDS budget");
            const int64_t mid = lo + (hi - lo) / 2;
            stack.push_back({mid, hi});
            stack.push_back({lo, mid});
        }
    }
    int64_t R = 0;
    size_t max_stage = 0;
    h_tiles.clear();
    h_inst_tile0.assign(n_inst() + 1, 0);
    std::vector<int32_t> uoff(1, 0), ucol;
    std::vector<uint16_t> lidx(std::max<size_t>(h_col.size(), 1), 0);
    size_t pi = 0;
    for (int32_t i = 0; i < n_inst(); ++i) {
        for (; pi < parts.size() && parts[pi].first < inst_row0[i + 1]; ++pi) {
            const int64_t r0 = parts[pi].first, rows = parts[pi].second - r0;
            collect(r0, rows);
            R = std::max(R, rows);
            max_stage = std::max(max_stage, (size_t)rows + ext.size());
            for (int64_t r = r0; r < r0 + rows; ++r) {
                const int64_t q = r / SR, w = (h_slice_off[q + 1] - h_slice_off[q]) / SR;
                for (int64_t k = 0; k < w; ++k) {
                    const int64_t slot = h_slice_off[q] + k * SR + r % SR;
                    const int32_t c = h_col[slot];
                    int64_t local;
                    if (c >= r0 && c < r0 + rows)
                        local = c - r0;
                    else
                        local = rows + (std::lower_bound(ext.begin(), ext.end(), c) - ext.begin());
                    lidx[slot] = (uint16_t)local;
                }
            }
            ucol.insert(ucol.end(), ext.begin(), ext.end());
            uoff.push_back((int32_t)ucol.size());
            h_tiles.push_back(TileDesc{r0, (int32_t)rows, i});
        }
        h_inst_tile0[i + 1] = (int32_t)h_tiles.size();
    }
    if (ucol.size() >= (size_t)INT32_MAX) return fail(TBPM_E_ARG, "staged lists too large");
    TRY_HIP(hipDeviceSynchronize(), "sync before tile rebuild");
    TRY_HIP(tiles.ensure(sizeof(TileDesc) * h_tiles.size()), "alloc tiles");
    TRY_HIP(inst_tile0.ensure(sizeof(int32_t) * h_inst_tile0.size()), "alloc inst_tile0");
    TRY_HIP(st_uoff.ensure(sizeof(int32_t) * uoff.size()), "alloc staged offsets");
    TRY_HIP(st_ucol.ensure(sizeof(int32_t) * std::max<size_t>(ucol.size(), 1)), "alloc staged rows");
    TRY_HIP(st_lidx.ensure(sizeof(uint16_t) * lidx.size()), "alloc staged indices");
    TRY_HIP(hipMemcpy(tiles.ptr, h_tiles.data(), sizeof(TileDesc) * h_tiles.size(), hipMemcpyHostToDevice),
            "upload tiles");
    TRY_HIP(hipMemcpy(inst_tile0.ptr, h_inst_tile0.data(), sizeof(int32_t) * h_inst_tile0.size(),
                      hipMemcpyHostToDevice),
            "upload inst_tile0");
    TRY_HIP(hipMemcpy(st_uoff.ptr, uoff.data(), sizeof(int32_t) * uoff.size(), hipMemcpyHostToDevice),
            "upload staged offsets");
    if (!ucol.empty())
        TRY_HIP(hipMemcpy(st_ucol.ptr, ucol.data(), sizeof(int32_t) * ucol.size(), hipMemcpyHostToDevice),
                "upload staged rows");
    TRY_HIP(hipMemcpy(st_lidx.ptr, lidx.data(), sizeof(uint16_t) * lidx.size(), hipMemcpyHostToDevice),
            "upload staged indices");
    stage_max_rows = max_stage;
    stage_units = (int32_t)(max_stage << log2u);
    tiles_s = s_pad;
    tiles_chunks = -(int32_t)R;
    tiles_unit = key;
    return TBPM_OK;
}

// ---------------------------------------------------------------------------
// two-hop tiles for the fused launch shape (tables built on the host by
// two_hop_tables, then uploaded)
// ---------------------------------------------------------------------------
tbpm_status Engine::build_fused_tiles(int32_t s_pad, int32_t log2u, int32_t unit_bytes, int32_t tier) {
    // the tables depend on the bytes of a row and the budget only (not on
    // how a row is split into units)
    const int32_t row_bytes = unit_bytes << log2u;
    const int32_t key = (1 << 24) + row_bytes * 16 + tier;
    if (tiles_s == s_pad && tiles_chunks < 0 && tiles_unit == key && tiles.ptr) {
        fu_lds_units = (int32_t)(fu_max_rows << log2u);
        return TBPM_OK;
    }
    TwoHopTables t;
    if (!two_hop_tables(h_slice_off, h_col, inst_row0, log2u, unit_bytes, fused_lds_budget(tier), t))
        return fail(TBPM_E_ARG, "no two-hop tile fits the LDS budget");
    h_tiles = t.tiles;
    h_inst_tile0 = t.inst_tile0;
    const size_t nt = h_tiles.size();
    TRY_HIP(hipDeviceSynchronize(), "sync before tile rebuild");
    TRY_HIP(tiles.ensure(sizeof(TileDesc) * nt), "alloc tiles");
    TRY_HIP(inst_tile0.ensure(sizeof(int32_t) * h_inst_tile0.size()), "alloc inst_tile0");
    TRY_HIP(st_uoff.ensure(sizeof(int32_t) * t.uoff.size()), "alloc two-hop offsets");
    TRY_HIP(st_ucol.ensure(sizeof(int32_t) * std::max<size_t>(t.ucol.size(), 1)), "alloc two-hop rows");
    TRY_HIP(st_lidx.ensure(sizeof(uint16_t) * t.lidx.size()), "alloc two-hop indices");
    TRY_HIP(fu_n1.ensure(sizeof(int32_t) * nt), "alloc two-hop counts");
    TRY_HIP(fu_hoff.ensure(sizeof(int32_t) * nt), "alloc two-hop offsets");
    TRY_HIP(fu_hw.ensure(sizeof(int32_t) * nt), "alloc two-hop widths");
    TRY_HIP(fu_hidx.ensure(sizeof(uint16_t) * t.hidx.size()), "alloc two-hop halo indices");
    auto up = [](DevBuf &d, const void *src, size_t bytes) { return hipMemcpy(d.ptr, src, bytes, hipMemcpyHostToDevice); };
    TRY_HIP(up(tiles, h_tiles.data(), sizeof(TileDesc) * nt), "upload tiles");
    TRY_HIP(up(inst_tile0, h_inst_tile0.data(), sizeof(int32_t) * h_inst_tile0.size()), "upload inst_tile0");
    TRY_HIP(up(st_uoff, t.uoff.data(), sizeof(int32_t) * t.uoff.size()), "upload two-hop offsets");
    if (!t.ucol.empty()) TRY_HIP(up(st_ucol, t.ucol.data(), sizeof(int32_t) * t.ucol.size()), "upload two-hop rows");
    TRY_HIP(up(st_lidx, t.lidx.data(), sizeof(uint16_t) * t.lidx.size()), "upload two-hop indices");
    TRY_HIP(up(fu_n1, t.n1.data(), sizeof(int32_t) * nt), "upload two-hop counts");
    TRY_HIP(up(fu_hoff, t.hoff.data(), sizeof(int32_t) * nt), "upload two-hop offsets");
    TRY_HIP(up(fu_hw, t.hw.data(), sizeof(int32_t) * nt), "upload two-hop widths");
    TRY_HIP(up(fu_hidx, t.hidx.data(), sizeof(uint16_t) * t.hidx.size()), "upload two-hop halo indices");
    fu_max_rows = t.max_xy;
    fu_lds_units = (int32_t)(t.max_xy << log2u);
    tiles_s = s_pad;
    tiles_chunks = -(int32_t)t.R;
    tiles_unit = key;
    return TBPM_OK;
}

static PassCoef make_coef(cd a, cd b) { return PassCoef{a.real(), a.imag(), b.real(), b.imag()}; }

// The Clenshaw schedule of one step for per-member coefficient sets c[i][m]
// (zero-padded to mmax: extra zero coefficients leave the polynomial and every
// intermediate b_j unchanged) and scales f[i].
std::vector<PassPlan> plan_step(const std::vector<std::vector<cd>> &c, const std::vector<double> &f, int mmax) {
    const size_t n = c.size();
    std::vector<PassPlan> plan;
    auto add = [&](int kind, int x, int v, int b2, int out, auto alpha, auto beta) {
        PassPlan p{kind, x, v, b2, out, {}};
        p.coef.resize(n);
        for (size_t i = 0; i < n; ++i) p.coef[i] = make_coef(alpha(i), beta(i));
        plan.push_back(std::move(p));
    };
    const int M = mmax;
    if (M == 3) {
        add(kPassFirst, 0, 0, -1, 1, [&](size_t i) { return c[i][1]; },
            [&](size_t i) { return 2.0 * c[i][2] / f[i]; });
        add(kPassLastNoB2, 1, 0, -1, 0, [&](size_t i) { return c[i][0] - c[i][2]; },
            [&](size_t i) { return cd(1.0 / f[i], 0.0); });
        return plan;
    }
    add(kPassFirst, 0, 0, -1, 1, [&](size_t i) { return c[i][M - 2]; },
        [&](size_t i) { return 2.0 * c[i][M - 1] / f[i]; });
    add(kPassNoB2, 1, 0, -1, 2, [&](size_t i) { return c[i][M - 3] - c[i][M - 1]; },
        [&](size_t i) { return cd(2.0 / f[i], 0.0); });
    int cur = 2, prev = 1;  // cur holds b_{j+1}, prev holds b_{j+2}
    for (int j = M - 4; j >= 1; --j) {
        add(kPassMid, cur, 0, prev, prev, [&, j](size_t i) { return c[i][j]; },
            [&](size_t i) { return cd(2.0 / f[i], 0.0); });
        std::swap(cur, prev);
    }
    add(kPassLast, cur, 0, prev, 0, [&](size_t i) { return c[i][0]; },
        [&](size_t i) { return cd(1.0 / f[i], 0.0); });
    return plan;
}


int32_t cheb_coeffs(double z, double tol, std::vector<cd> &c) {
    const int32_t M = num_terms(z, tol);
    if (M < 0) return M;
    std::vector<double> J(M);
    bessel_j(z, M, J.data());
    c.resize(M);
    static const cd mi[4] = {cd(1, 0), cd(0, -1), cd(-1, 0), cd(0, 1)};  // (-i)^m
    for (int32_t m = 0; m < M; ++m) c[m] = (m == 0 ? 1.0 : 2.0) * J[m] * mi[m & 3];
    return M;
}

tbpm_status Engine::run(const RunArgs &a) {
    int dev = 0;
    TRY_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != device) return fail(TBPM_E_ARG, "handle was created on another device");
    const int32_t ni = n_inst();
    int32_t s_pad = 1, log2s = 0;
    while (s_pad < a.s_user) {
        s_pad <<= 1;
        ++log2s;
    }
    const bool fp32 = a.fp32;
    const size_t esize = fp32 ? 8 : 16;
    cfg = cfgs[fp32 ? 1 : 0];

    // coefficients per member
    std::vector<std::vector<cd>> c(ni);
    std::vector<double> f(ni);
    int mmax = 0;
    for (int32_t i = 0; i < ni; ++i) {
        const double z = a.rescale[i] * a.dt[i];
        const int32_t M = cheb_coeffs(z, a.tol, c[i]);
        if (M < 0) return fail(TBPM_E_ARG, "Bessel series does not converge for z = " + std::to_string(z));
        f[i] = a.rescale[i];
        mmax = std::max(mmax, M);
    }
    for (int32_t i = 0; i < ni; ++i) c[i].resize(mmax, cd(0.0, 0.0));
    const std::vector<PassPlan> plan = plan_step(c, f, mmax);
    const int n_passes = (int)plan.size();

    const int32_t chunks = cfg.wg_chunks;
    const int32_t vs = std::min(cfg.vec, s_pad);
    const int32_t log2u = log2s - (vs == 4 ? 2 : (vs == 2 ? 1 : 0));
    const int32_t unit_bytes = (int32_t)esize * vs;
    bool fused = cfg.fused != 0 && mmax >= 4;
    bool staged = cfg.staged != 0 && !fused;
    // the staged shape takes rows wider than kStagedRowBytes one block of
    // states at a time (units of a block: 2^log2ub)
    int32_t log2ub = log2u;
    while (staged && log2ub > 0 && ((int64_t)unit_bytes << log2ub) > kStagedRowBytes) --log2ub;
    tbpm_status st = TBPM_OK;
    if (fused && build_fused_tiles(s_pad, log2u, unit_bytes, cfg.fused) != TBPM_OK) fused = false;  // fall back
    if (staged && build_staged_tiles(s_pad, log2ub, unit_bytes, cfg.staged) != TBPM_OK) staged = false;
    if (!staged && !fused) st = build_tiles(s_pad, chunks, vs);
    if (st != TBPM_OK) return st;
    const int32_t n_tiles = (int32_t)h_tiles.size();
    const int64_t n_el = mat.n_rows * s_pad;
    if (n_el >= (int64_t)INT32_MAX) return fail(TBPM_E_ARG, "n_orb * n_states (padded to a power of two) must be < 2^31");

    TRY_HIP(v.ensure(esize * n_el), "alloc v");
    TRY_HIP(ba.ensure(esize * n_el), "alloc A");
    TRY_HIP(bb.ensure(esize * n_el), "alloc B");
    if (fused) {
        TRY_HIP(bc.ensure(esize * n_el), "alloc C");
        TRY_HIP(bd.ensure(esize * n_el), "alloc D");
    }
    TRY_HIP(phi0.ensure(16 * n_el), "alloc phi0");
    TRY_HIP(partials.ensure(sizeof(double) * 3 * (size_t)n_tiles * s_pad), "alloc partials");
    TRY_HIP(counter.ensure(sizeof(int32_t) * 64), "alloc counter");
    TRY_HIP(coef.ensure(sizeof(PassCoef) * (size_t)n_passes * ni), "alloc coef");
    TRY_HIP(norm2_all.ensure(sizeof(double) * (size_t)ni * a.n_steps * a.s_user), "alloc norm2");
    TRY_HIP(ptr_tab.ensure(sizeof(void *) * 3 * (size_t)ni), "alloc pointer table");
    TRY_HIP(inst_row0_dev.ensure(sizeof(int64_t) * (ni + 1)), "alloc inst_row0");

    // slot of each stored psi(k dt): checkpoints at k = m K (k <= n_steps - 2)
    // into slot m - 1, or the listed snapshot steps into their list position
    const size_t slot_bytes = a.ckpt ? sizeof(int32_t) * (size_t)a.n_steps : 0;
    if (a.ckpt) TRY_HIP(ckpt_slot.ensure(slot_bytes), "alloc checkpoint slots");
    const size_t qe_bytes = a.n_qe > 0 ? sizeof(double) * 2 * (size_t)a.n_steps * a.n_qe : 0;
    if (a.n_qe > 0) TRY_HIP(qe_coef.ensure(qe_bytes), "alloc quasi-eigenstate coefficients");
    const size_t jc_bytes = a.jc_states > 0 ? 2 * sizeof(void *) : 0;
    if (a.jc_states > 0) {
        TRY_HIP(jc_tab.ensure(jc_bytes), "alloc correlation table");
        TRY_HIP(jc_norm.ensure(sizeof(double) * (size_t)a.n_steps * a.jc_states), "alloc correlation scratch");
    }

    // stage the small tables through pinned memory, stream-ordered
    const size_t coef_bytes = sizeof(PassCoef) * (size_t)n_passes * ni;
    const size_t tab_bytes = sizeof(void *) * 3 * (size_t)ni;
    const size_t row_bytes = sizeof(int64_t) * (ni + 1);
    TRY_HIP(hipEventSynchronize(staging_done), "wait for staging");
    TRY_HIP(staging.ensure(coef_bytes + tab_bytes + row_bytes + slot_bytes + qe_bytes + jc_bytes), "alloc staging");
    char *sp = (char *)staging.ptr;
    PassCoef *hc = (PassCoef *)sp;
    for (int p = 0; p < n_passes; ++p)
        for (int32_t i = 0; i < ni; ++i) hc[p * ni + i] = plan[p].coef[i];
    const void **ht = (const void **)(sp + coef_bytes);
    for (int32_t i = 0; i < ni; ++i) {
        ht[i] = a.psi0[i];
        ht[ni + i] = a.corr[i];
        ht[2 * ni + i] = a.norm2 ? a.norm2[i] : nullptr;
    }
    std::memcpy(sp + coef_bytes + tab_bytes, inst_row0.data(), row_bytes);
    TRY_HIP(hipMemcpyAsync(coef.ptr, sp, coef_bytes, hipMemcpyHostToDevice, a.stream), "upload coefficients");
    TRY_HIP(hipMemcpyAsync(ptr_tab.ptr, sp + coef_bytes, tab_bytes, hipMemcpyHostToDevice, a.stream),
            "upload pointer table");
    TRY_HIP(hipMemcpyAsync(inst_row0_dev.ptr, sp + coef_bytes + tab_bytes, row_bytes, hipMemcpyHostToDevice,
                           a.stream),
            "upload row offsets");
    if (a.ckpt) {
        int32_t *hs = (int32_t *)(sp + coef_bytes + tab_bytes + row_bytes);
        for (int32_t k = 0; k < a.n_steps; ++k) hs[k] = -1;
        if (a.n_snap > 0) {
            for (int32_t q = 0; q < a.n_snap; ++q)
                if (a.snap_steps[q] > 0 && a.snap_steps[q] < a.n_steps) hs[a.snap_steps[q]] = q;
        } else {
            for (int32_t k = a.ckpt_every; k <= a.n_steps - 2; k += a.ckpt_every) hs[k] = k / a.ckpt_every - 1;
        }
        TRY_HIP(hipMemcpyAsync(ckpt_slot.ptr, hs, slot_bytes, hipMemcpyHostToDevice, a.stream), "upload slots");
    }
    if (a.n_qe > 0) {
        char *hq = sp + coef_bytes + tab_bytes + row_bytes + slot_bytes;
        std::memcpy(hq, a.qe_coef, qe_bytes);
        TRY_HIP(hipMemcpyAsync(qe_coef.ptr, hq, qe_bytes, hipMemcpyHostToDevice, a.stream),
                "upload quasi-eigenstate coefficients");
    }
    if (a.jc_states > 0) {
        void **hj = (void **)(sp + coef_bytes + tab_bytes + row_bytes + slot_bytes + qe_bytes);
        hj[0] = a.jc_corr;
        hj[1] = nullptr;
        TRY_HIP(hipMemcpyAsync(jc_tab.ptr, hj, jc_bytes, hipMemcpyHostToDevice, a.stream), "upload correlation table");
    }
    const int64_t n_el_all = mat.n_rows * s_pad;
    int32_t log2sp = 0;
    while ((1 << log2sp) < a.jc_states) ++log2sp;
    // per-step work after the correlation: quasi-eigenstate accumulation and
    // the optical-conductivity correlation
    auto enqueue_qe = [&](hipStream_t s) -> tbpm_status {
        if (a.n_qe > 0) {
            hipError_t e = launch_qe_accum(fp32, v.ptr, a.qe_acc, n_el_all, (const double *)qe_coef.ptr, a.n_qe,
                                           (const int32_t *)counter.ptr, s);
            if (e != hipSuccess) return hip_fail(e, "launch quasi-eigenstate accumulation");
        }
        if (a.jc_states > 0) {
            hipError_t e = launch_jcorr(fp32, (const TileDesc *)tiles.ptr, (int32_t)h_tiles.size(), log2sp, a.jc_states,
                                        log2s, v.ptr, mat.slice_off, mat.col, a.jc_val, (double *)partials.ptr, s);
            if (e != hipSuccess) return hip_fail(e, "launch current correlation");
            ReduceParams jr{};
            jr.partials = (const double *)partials.ptr;
            jr.n_tiles = (int32_t)h_tiles.size();
            jr.inst_tile0 = (const int32_t *)inst_tile0.ptr;
            jr.log2s = log2sp;
            jr.s_user = a.jc_states;
            jr.n_steps = a.n_steps;
            jr.counter = (const int32_t *)counter.ptr;
            jr.corr = (double *const *)jc_tab.ptr;
            jr.norm2 = (double *const *)jc_tab.ptr + 1;
            jr.norm2_all = (double *)jc_norm.ptr;
            e = launch_reduce(1, s_pad, jr, s);
            if (e != hipSuccess) return hip_fail(e, "launch current correlation reduce");
        }
        return TBPM_OK;
    };
    TRY_HIP(hipEventRecord(staging_done, a.stream), "record staging");

    void *bufptr[5] = {v.ptr, ba.ptr, bb.ptr, bc.ptr, bd.ptr};
    const double *const *d_psi0 = (const double *const *)ptr_tab.ptr;
    double *const *d_corr = (double *const *)ptr_tab.ptr + ni;
    double *const *d_norm2 = (double *const *)ptr_tab.ptr + 2 * ni;

    // C_0
    InitParams ip{};
    ip.tiles = (const TileDesc *)tiles.ptr;
    ip.n_tiles = n_tiles;
    ip.log2s = log2s;
    ip.s_user = a.s_user;
    ip.psi0 = d_psi0;
    ip.inst_row0 = (const int64_t *)inst_row0_dev.ptr;
    ip.v = v.ptr;
    ip.phi0 = (double *)phi0.ptr;
    ip.partials = (double *)partials.ptr;
    ip.counter = (int32_t *)counter.ptr;
    ip.perm = mat.perm;
    TRY_HIP(launch_init(fp32, ip, a.stream), "launch init");
    ReduceParams rp{};
    rp.partials = (const double *)partials.ptr;
    rp.n_tiles = n_tiles;
    rp.inst_tile0 = (const int32_t *)inst_tile0.ptr;
    rp.log2s = log2s;
    rp.s_user = a.s_user;
    rp.n_steps = a.n_steps;
    rp.counter = (const int32_t *)counter.ptr;
    rp.corr = d_corr;
    rp.norm2 = d_norm2;
    rp.norm2_all = (double *)norm2_all.ptr;
    TRY_HIP(launch_reduce(ni, s_pad, rp, a.stream), "launch reduce");
    st = enqueue_qe(a.stream);
    if (st != TBPM_OK) return st;

    // Fused schedule (plan: 0 FIRST, 1 NOB2, 2 .. n_passes-2 MID,
    // n_passes-1 LAST).  Orders run two per launch wherever they can: FIRST
    // and NOB2 as one pair, then MID orders in pairs; a pair reads its inputs
    // on rows other tiles write, so its outputs go to the two work buffers
    // (of A, B, C, D) it does not read.  The last MID and LAST run as one
    // pair when nothing but the correlation is taken from psi_{k+1} (no
    // stored states, quasi-eigenstates or current correlation): psi_{k+1}
    // then goes to a free buffer, which becomes the next step's psi
    // (bufptr[0] and that buffer trade places after every step, so a graph
    // of an even number of steps ends where it began).  With an even number
    // of MID orders FIRST then runs alone and NOB2 pairs with the first MID,
    // so that no MID is left over; otherwise a leftover MID runs alone, in
    // place over b_{j+2}, and LAST alone, in place over psi.
    // Entries: {plan index, pair kind or -1 for one order, x, b2, out1, out2}
    // with buffer indices into bufptr (-1: none).
    struct Launch {
        int p, kind, x, b2, o1, o2;
    };
    std::vector<Launch> sched;
    const bool last_pair = fused && n_passes >= 4 && !a.ckpt && a.n_qe == 0 && a.jc_states == 0;
    if (fused) {
        const int n_mid = n_passes - 3;
        int cur = 0, prev = -1;  // buffers of b_{j+1} and b_{j+2} (0: psi, -1: none)
        auto free_buf = [&](int k) {  // the k-th lowest work buffer other than cur and prev
            for (int b = 1; b <= 4; ++b)
                if (b != cur && b != prev && k-- == 0) return b;
            return -1;
        };
        auto pair = [&](int p, int kind) {
            const int o1 = free_buf(0), o2 = free_buf(1);
            sched.push_back({p, kind, cur, prev, o1, o2});
            prev = o1;
            cur = o2;
        };
        int p = 0;
        if (last_pair && n_mid % 2 == 0) {
            sched.push_back({0, -1, 0, -1, 1, -1});
            cur = 1;
            pair(1, kPairSecond);
            p = 3;
        } else {
            pair(0, kPairFirst);
            p = 2;
        }
        const int mid_end = last_pair ? n_passes - 2 : n_passes - 1;  // MIDs before the last launch
        for (; p + 1 < mid_end; p += 2) pair(p, kPairMid);
        for (; p < mid_end; ++p) {
            sched.push_back({p, -1, cur, prev, prev, -1});
            std::swap(cur, prev);
        }
        if (last_pair)
            sched.push_back({n_passes - 2, kPairLast, cur, prev, -1, free_buf(0)});
        else
            sched.push_back({n_passes - 1, -1, cur, prev, 0, -1});
    }

    // one time step; consecutive launches walk the tiles in opposite
    // directions (walk: the direction of the next launch)
    int32_t walk = 0;
    auto enqueue_step = [&](hipStream_t s) -> tbpm_status {
        if (fused) {
            for (size_t q = 0; q < sched.size(); ++q) {
                const Launch &l = sched[q];
                if (l.kind >= 0) {
                    FusedParams fp{};
                    fp.tiles = (const TileDesc *)tiles.ptr;
                    fp.n_tiles = n_tiles;
                    fp.xcd_remap = cfg.xcd_remap;
                    fp.log2s = log2s;
                    fp.bump_counter = (q == 0);
                    fp.col = mat.col;
                    fp.val = fp32 ? mat.val32 : mat.val64;
                    fp.slice_off = mat.slice_off;
                    fp.onsite = fp32 ? (const void *)mat.onsite32 : (const void *)mat.onsite64;
                    fp.x = bufptr[l.x];
                    fp.v = bufptr[0];
                    fp.b2 = l.b2 >= 0 ? bufptr[l.b2] : nullptr;
                    fp.out1 = l.o1 >= 0 ? bufptr[l.o1] : nullptr;
                    fp.out2 = bufptr[l.o2];
                    fp.coef1 = (const PassCoef *)coef.ptr + (size_t)l.p * ni;
                    fp.coef2 = (const PassCoef *)coef.ptr + (size_t)(l.p + 1) * ni;
                    fp.counter = (int32_t *)counter.ptr;
                    fp.uoff = (const int32_t *)st_uoff.ptr;
                    fp.n1 = (const int32_t *)fu_n1.ptr;
                    fp.ucol = (const int32_t *)st_ucol.ptr;
                    fp.lidx = (const uint16_t *)st_lidx.ptr;
                    fp.hoff = (const int32_t *)fu_hoff.ptr;
                    fp.hw = (const int32_t *)fu_hw.ptr;
                    fp.hidx = (const uint16_t *)fu_hidx.ptr;
                    fp.lds_units = fu_lds_units;
                    fp.uniform_w = mat.uniform_w;
                    fp.reverse = walk;
                    walk ^= 1;
                    fp.phi0 = (const double *)phi0.ptr;
                    fp.phi0_ld = s_pad;
                    fp.partials = (double *)partials.ptr;
                    hipError_t e = launch_pair(l.kind, fp32, mat.is_complex, cfg.nontemporal != 0, vs, fp, s);
                    if (e != hipSuccess) return hip_fail(e, "launch pair");
                    if (l.kind == kPairLast) std::swap(bufptr[0], bufptr[l.o2]);
                    continue;
                }
                const PassPlan &pl = plan[l.p];
                PassParams pp{};
                pp.tiles = (const TileDesc *)tiles.ptr;
                pp.n_tiles = n_tiles;
                pp.xcd_remap = cfg.xcd_remap;
                pp.log2s = log2s;
                pp.bump_counter = (q == 0);
                pp.col = mat.col;
                pp.val = fp32 ? mat.val32 : mat.val64;
                pp.slice_off = mat.slice_off;
                pp.onsite = fp32 ? (const void *)mat.onsite32 : (const void *)mat.onsite64;
                pp.x = bufptr[l.x];
                pp.v = bufptr[0];
                pp.b2 = l.b2 >= 0 ? bufptr[l.b2] : nullptr;
                pp.out = bufptr[l.o1];
                pp.coef = (const PassCoef *)coef.ptr + (size_t)l.p * ni;
                pp.counter = (int32_t *)counter.ptr;
                pp.phi0 = (const double *)phi0.ptr;
                pp.phi0_ld = s_pad;
                pp.partials = (double *)partials.ptr;
                pp.ckpt = a.ckpt;
                pp.perm = mat.perm;
                pp.ckpt_slot = a.ckpt ? (const int32_t *)ckpt_slot.ptr : nullptr;
                pp.ckpt_stride = mat.n_rows * a.s_user;
                pp.s_user = a.s_user;
                pp.uniform_w = mat.uniform_w;
                pp.reverse = walk;
                walk ^= 1;
                hipError_t e =
                    launch_pass(pl.kind, fp32, mat.is_complex, cfg.nontemporal != 0, cfg.unroll, vs, pp, s);
                if (e != hipSuccess) return hip_fail(e, "launch pass");
            }
            hipError_t e = launch_reduce(ni, s_pad, rp, s);
            if (e != hipSuccess) return hip_fail(e, "launch reduce");
            return enqueue_qe(s);
        }
        for (int p = 0; p < n_passes; ++p) {
            const PassPlan &pl = plan[p];
            PassParams pp{};
            pp.tiles = (const TileDesc *)tiles.ptr;
            pp.n_tiles = n_tiles;
            pp.xcd_remap = cfg.xcd_remap;
            pp.log2s = log2s;
            pp.bump_counter = (p == 0);
            pp.col = mat.col;
            pp.val = fp32 ? mat.val32 : mat.val64;
            pp.slice_off = mat.slice_off;
            pp.onsite = fp32 ? (const void *)mat.onsite32 : (const void *)mat.onsite64;
            pp.x = bufptr[pl.x];
            pp.v = bufptr[pl.v];
            pp.b2 = pl.b2 >= 0 ? bufptr[pl.b2] : nullptr;
            pp.out = bufptr[pl.out];
            pp.coef = (const PassCoef *)coef.ptr + (size_t)p * ni;
            pp.counter = (int32_t *)counter.ptr;
            pp.phi0 = (const double *)phi0.ptr;
            pp.phi0_ld = s_pad;
            pp.partials = (double *)partials.ptr;
            pp.ckpt = a.ckpt;
            pp.perm = mat.perm;
            pp.ckpt_slot = a.ckpt ? (const int32_t *)ckpt_slot.ptr : nullptr;
            pp.ckpt_stride = mat.n_rows * a.s_user;
            pp.s_user = a.s_user;
            pp.uoff = (const int32_t *)st_uoff.ptr;
            pp.ucol = (const int32_t *)st_ucol.ptr;
            pp.lidx = (const uint16_t *)st_lidx.ptr;
            pp.stage_units = stage_units;
            pp.log2ub = log2ub;
            pp.uniform_w = staged ? 0 : mat.uniform_w;
            pp.reverse = walk;
            walk ^= 1;
            hipError_t e = staged ? launch_pass_staged(pl.kind, fp32, mat.is_complex, cfg.nontemporal != 0, vs,
                                                  mat.max_width > kStagedWide, pp, s)
                                  : launch_pass(pl.kind, fp32, mat.is_complex, cfg.nontemporal != 0, cfg.unroll, vs,
                                                pp, s);
            if (e != hipSuccess) return hip_fail(e, "launch pass");
        }
        hipError_t e = launch_reduce(ni, s_pad, rp, s);
        if (e != hipSuccess) return hip_fail(e, "launch reduce");
        return enqueue_qe(s);
    };

    if (a.n_steps > 1) {
        if (a.flags & TBPM_FLAG_NO_GRAPH) {
            for (int32_t k = 1; k < a.n_steps; ++k) {
                st = enqueue_step(a.stream);
                if (st != TBPM_OK) return st;
            }
        } else {
            GraphKey key;
            key.s_pad = s_pad;
            key.s_user = a.s_user;
            key.fp32 = fp32;
            key.mmax = mmax;
            key.n_inst = ni;
            key.chunks = chunks;
            key.remap = cfg.xcd_remap;
            key.nt = cfg.nontemporal;
            key.unroll = cfg.unroll;
            key.staged = staged ? cfg.staged : 0;
            key.vec = vs;
            key.fused = fused ? cfg.fused : 0;
            key.n_tiles = n_tiles;
            key.tiles_chunks = tiles_chunks;
            key.tiles_unit = tiles_unit;
            key.lds_units = fused ? fu_lds_units : (staged ? stage_units : 0);

            key.n_steps = a.n_steps;
            key.n_qe = a.n_qe;
            key.jc_states = a.jc_states;
            key.ckpt = a.ckpt;
            const void *kb[22] = {v.ptr,       ba.ptr,      bb.ptr,        phi0.ptr,    partials.ptr, coef.ptr,
                                  tiles.ptr,   norm2_all.ptr, bc.ptr,      bd.ptr,      st_uoff.ptr,  st_ucol.ptr,
                                  st_lidx.ptr, fu_hidx.ptr, fu_n1.ptr,     fu_hoff.ptr, fu_hw.ptr,
                                  a.ckpt ? ckpt_slot.ptr : nullptr, a.n_qe > 0 ? qe_coef.ptr : nullptr,
                                  a.n_qe > 0 ? a.qe_acc : nullptr, a.jc_states > 0 ? a.jc_val : nullptr,
                                  a.jc_states > 0 ? jc_norm.ptr : nullptr};
            static_assert(sizeof(kb) == sizeof(key.bufs), "graph key buffers");
            std::memcpy(key.bufs, kb, sizeof(kb));
            // Graphs of kStepsPerGraph time steps (small operators are bound by
            // the cost of launching a graph, not by its kernels), and a graph of
            // one step for the remainder; the device step counter tells every
            // step's reduce which sample it writes.
            const int32_t n_adv = a.n_steps - 1;
            const int32_t spg = std::min<int32_t>(kStepsPerGraph, n_adv);
            const int32_t n_full = n_adv / spg, n_rest = n_adv % spg;
            auto cached = [&](hipGraphExec_t &exec, GraphKey &gkey, int32_t steps) -> tbpm_status {
                key.steps = steps;
                if (exec && key == gkey) return TBPM_OK;
                if (exec) {
                    TRY_HIP(hipDeviceSynchronize(), "sync before graph rebuild");
                    TRY_HIP(hipGraphExecDestroy(exec), "hipGraphExecDestroy");
                    exec = nullptr;
                }
                TRY_HIP(hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
                walk = 0;  // a graph of an even number of launches keeps the alternation across replays
                tbpm_status cst = TBPM_OK;
                for (int32_t q = 0; q < steps && cst == TBPM_OK; ++q) cst = enqueue_step(capture_stream);
                hipGraph_t g = nullptr;
                hipError_t ee = hipStreamEndCapture(capture_stream, &g);
                if (cst != TBPM_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return cst;
                }
                if (ee != hipSuccess) return hip_fail(ee, "end capture");
                hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ei != hipSuccess) {
                    exec = nullptr;
                    return hip_fail(ei, "hipGraphInstantiate");
                }
                gkey = key;
                return TBPM_OK;
            };
            // With the last pair a step moves psi to another buffer, so a graph
            // replayed more than once must hold an even number of steps: the
            // remainder is then one graph of n_rest steps, launched once (the
            // full graphs, when replayed, hold kStepsPerGraph steps, an even
            // number, and leave the buffers as they found them).
            static_assert(kStepsPerGraph % 2 == 0, "a replayed step graph must hold an even number of steps");
            const int32_t rest_steps = last_pair ? std::max<int32_t>(n_rest, 1) : 1;
            st = cached(graph_exec, graph_key, spg);
            if (st == TBPM_OK && n_rest > 0) st = cached(graph_exec1, graph_key1, rest_steps);
            if (st != TBPM_OK) return st;
            for (int32_t k = 0; k < n_full; ++k) TRY_HIP(hipGraphLaunch(graph_exec, a.stream), "hipGraphLaunch");
            for (int32_t k = 0; k < n_rest / rest_steps; ++k)
                TRY_HIP(hipGraphLaunch(graph_exec1, a.stream), "hipGraphLaunch");
        }
    }

    last_s_pad = s_pad;
    last_fp32 = fp32 ? 1 : 0;
    last_staged = fused ? 2 : (staged ? 1 : 0);
    last_vs = vs;
    last_log2ub = log2ub;
    if (a.flags & TBPM_FLAG_ASYNC) return TBPM_OK;
    TRY_HIP(hipStreamSynchronize(a.stream), "stream synchronize");
    TRY_HIP(hipGetLastError(), "kernel execution");
    // norm check (the spectrum must lie in [-f, f])
    std::vector<double> n2((size_t)ni * a.n_steps * a.s_user);
    TRY_HIP(hipMemcpy(n2.data(), norm2_all.ptr, sizeof(double) * n2.size(), hipMemcpyDeviceToHost), "read norms");
    for (int32_t i = 0; i < ni; ++i) {
        for (int32_t s = 0; s < a.s_user; ++s) {
            const double n0 = n2[(size_t)i * a.n_steps * a.s_user + s];
            if (!(n0 > 0.0)) continue;
            for (int32_t k = 0; k < a.n_steps; ++k) {
                const double r = n2[((size_t)i * a.n_steps + k) * a.s_user + s] / n0;
                if (!std::isfinite(r) || std::fabs(r - 1.0) > 1e-3) {
                    char buf[256];
                    std::snprintf(buf, sizeof buf,
                                  "norm check failed (member %d, state %d, step %d: ||psi||^2/||psi0||^2 = %.6g); "
                                  "is the spectrum inside [-rescale, rescale]?",
                                  i, s, k, r);
                    return fail(TBPM_E_DIVERGED, buf);
                }
            }
        }
    }
    return TBPM_OK;
}

tbpm_status Engine::apply_series(const std::vector<double> &a_in, double f, int32_t log2s, const void *src, void *dst,
                                 void *w0, void *w1, hipStream_t st, void *w2, void *w3) {
    // Clenshaw for sum_{k<K} a_k T_k(x), x = H/f (zero-padded to K >= 3):
    //   b_{K-2} = a_{K-2} v + 2 a_{K-1} x v                       (FIRST)
    //   b_{K-3} = (a_{K-3} - a_{K-1}) v + 2 x b_{K-2}             (NOB2)
    //   b_k     = a_k v + 2 x b_{k+1} - b_{k+2},  k = K-4 .. 1   (MID)
    //   out     = a_0 v + x b_1 - b_2                              (MID with beta = 1/f)
    // and for K = 3: b_1 by FIRST, out = (a_0 - a_2) v + x b_1 (NOB2).
    std::vector<double> a(a_in);
    if (a.size() < 3) a.resize(3, 0.0);
    const int32_t K = (int32_t)a.size();
    struct Launch {
        int kind;
        const void *x, *b2;
        void *out;
        PassCoef c;
    };
    std::vector<Launch> seq;
    void *w[2] = {w0, w1};
    if (K == 3) {
        seq.push_back({kPassFirst, src, nullptr, w[0], {a[1], 0, 2.0 * a[2] / f, 0}});
        seq.push_back({kPassNoB2, w[0], nullptr, dst, {a[0] - a[2], 0, 1.0 / f, 0}});
    } else {
        seq.push_back({kPassFirst, src, nullptr, w[0], {a[K - 2], 0, 2.0 * a[K - 1] / f, 0}});
        seq.push_back({kPassNoB2, w[0], nullptr, w[1], {a[K - 3] - a[K - 1], 0, 2.0 / f, 0}});
        int cur = 1;  // b_{k+1} in w[cur], b_{k+2} in w[1 - cur]; MID writes over b_{k+2}
        for (int32_t k = K - 4; k >= 1; --k) {
            seq.push_back({kPassMid, w[cur], w[1 - cur], w[1 - cur], {a[k], 0, 2.0 / f, 0}});
            cur = 1 - cur;
        }
        seq.push_back({kPassMid, w[cur], w[1 - cur], dst, {a[0], 0, 1.0 / f, 0}});
    }
    // With the fused shape configured (and two more work blocks), the orders
    // run two per launch: (K-2, K-3) from the input, then (k, k-1) pairs over
    // four rotating blocks (a pair's outputs go to the two blocks it does not
    // read), the last pair writing the result; an order left over runs alone.
    const int32_t s_pad = 1 << log2s;
    bool pairs = w2 && w3 && K >= 4 && cfgs[0].fused > 0;
    int32_t pvs = 1, log2pvs = 0;
    while (pvs < cfgs[0].vec && pvs < s_pad && pvs < 4) {
        pvs <<= 1;
        ++log2pvs;
    }
    if (pairs && build_fused_tiles(s_pad, log2s - log2pvs, 16 * pvs, cfgs[0].fused) != TBPM_OK) pairs = false;
    if (!pairs && (!tiles.ptr || tiles_s == 0)) {
        tbpm_status s = build_tiles(s_pad, cfg.wg_chunks, 1);
        if (s != TBPM_OK) return s;
    }
    const size_t cb = sizeof(PassCoef) * seq.size();
    TRY_HIP(coef.ensure(cb), "alloc series coefficients");
    TRY_HIP(hipEventSynchronize(staging_done), "wait for staging");
    TRY_HIP(staging.ensure(cb), "alloc staging");
    PassCoef *hc = (PassCoef *)staging.ptr;
    for (size_t i = 0; i < seq.size(); ++i) hc[i] = seq[i].c;
    TRY_HIP(hipMemcpyAsync(coef.ptr, hc, cb, hipMemcpyHostToDevice, st), "upload series coefficients");
    TRY_HIP(hipEventRecord(staging_done, st), "record staging");
    PassParams pp{};
    pp.tiles = (const TileDesc *)tiles.ptr;
    pp.n_tiles = (int32_t)h_tiles.size();
    pp.xcd_remap = cfg.xcd_remap;
    pp.log2s = log2s;
    pp.col = mat.col;
    pp.val = mat.val64;
    pp.slice_off = mat.slice_off;
    pp.onsite = mat.onsite64;
    pp.counter = (int32_t *)counter.ptr;
    pp.s_user = 1 << log2s;
    pp.v = src;
    if (pairs) {
        // seq holds the orders K-2, K-3, ..., 0 in evaluation order with
        // their coefficients; only the coefficients are taken from it here
        const bool nt = cfgs[0].nontemporal != 0;
        FusedParams fp{};
        fp.tiles = (const TileDesc *)tiles.ptr;
        fp.n_tiles = (int32_t)h_tiles.size();
        fp.xcd_remap = cfg.xcd_remap;
        fp.log2s = log2s;
        fp.col = mat.col;
        fp.val = mat.val64;
        fp.slice_off = mat.slice_off;
        fp.onsite = mat.onsite64;
        fp.counter = (int32_t *)counter.ptr;
        fp.uoff = (const int32_t *)st_uoff.ptr;
        fp.n1 = (const int32_t *)fu_n1.ptr;
        fp.ucol = (const int32_t *)st_ucol.ptr;
        fp.lidx = (const uint16_t *)st_lidx.ptr;
        fp.hoff = (const int32_t *)fu_hoff.ptr;
        fp.hw = (const int32_t *)fu_hw.ptr;
        fp.hidx = (const uint16_t *)fu_hidx.ptr;
        fp.lds_units = (int32_t)(fu_max_rows << (log2s - log2pvs));
        fp.uniform_w = mat.uniform_w;
        fp.v = src;
        void *wb[4] = {w0, w1, w2, w3};
        const PassCoef *cf = (const PassCoef *)coef.ptr;
        const size_t n_ord = seq.size();  // K - 1 orders, the last one the result
        // (K-2, K-3) from the input into wb[0], wb[1]
        fp.x = src;
        fp.b2 = nullptr;
        fp.out1 = wb[0];
        fp.out2 = n_ord == 2 ? dst : wb[1];
        fp.coef1 = cf;
        fp.coef2 = cf + 1;
        // consecutive launches walk the tiles in opposite directions
        int32_t walk = 0;
        fp.reverse = walk;
        walk ^= 1;
        hipError_t e = launch_pair(kPairFirst, false, mat.is_complex, nt, pvs, fp, st);
        int x = 1, b2 = 0;  // b_{k+1} in wb[x], b_{k+2} in wb[b2]
        size_t i = 2;
        for (; e == hipSuccess && i + 1 < n_ord; i += 2) {
            int free_[2], nf = 0;
            for (int q = 0; q < 4 && nf < 2; ++q)
                if (q != x && q != b2) free_[nf++] = q;
            fp.x = wb[x];
            fp.b2 = wb[b2];
            fp.out1 = wb[free_[0]];
            fp.out2 = (i + 1 == n_ord - 1) ? dst : wb[free_[1]];
            fp.coef1 = cf + i;
            fp.coef2 = cf + i + 1;
            fp.reverse = walk;
            walk ^= 1;
            e = launch_pair(kPairMid, false, mat.is_complex, nt, pvs, fp, st);
            b2 = free_[0];
            x = free_[1];
        }
        if (e == hipSuccess && i < n_ord) {  // the result alone: out = a_0 v + H~ b_1 - b_2
            pp.x = wb[x];
            pp.b2 = wb[b2];
            pp.out = dst;
            pp.coef = cf + i;
            pp.reverse = walk;
            e = launch_pass(kPassMid, false, mat.is_complex, nt, 1, pvs, pp, st);
        }
        if (e != hipSuccess) return hip_fail(e, "launch series pair");
        return TBPM_OK;
    }
    for (size_t i = 0; i < seq.size(); ++i) {
        pp.x = seq[i].x;
        pp.b2 = seq[i].b2;
        pp.out = seq[i].out;
        pp.coef = (const PassCoef *)coef.ptr + i;
        pp.reverse = (int32_t)(i & 1);  // consecutive launches walk the tiles in opposite directions
        hipError_t e = launch_pass(seq[i].kind, false, mat.is_complex, false, 1, 1, pp, st);
        if (e != hipSuccess) return hip_fail(e, "launch series pass");
    }
    return TBPM_OK;
}

tbpm_status Engine::apply_ell(const double *jval, int32_t log2s, const void *src, void *dst, hipStream_t st) {
    if (!tiles.ptr || tiles_s == 0) {
        tbpm_status s = build_tiles(1 << log2s, cfg.wg_chunks, 1);
        if (s != TBPM_OK) return s;
    }
    TRY_HIP(ac_zero.ensure(sizeof(double) * (size_t)std::max<int64_t>(mat.n_rows, 1)), "alloc zero on-site");
    TRY_HIP(launch_fill_zero((double *)ac_zero.ptr, mat.n_rows, st), "clear zero on-site");
    TRY_HIP(coef.ensure(sizeof(PassCoef)), "alloc coefficient");
    TRY_HIP(hipEventSynchronize(staging_done), "wait for staging");
    TRY_HIP(staging.ensure(sizeof(PassCoef)), "alloc staging");
    PassCoef *hc = (PassCoef *)staging.ptr;
    hc[0] = PassCoef{0.0, 0.0, 1.0, 0.0};  // out = 0 * v + 1 * (J x)
    TRY_HIP(hipMemcpyAsync(coef.ptr, hc, sizeof(PassCoef), hipMemcpyHostToDevice, st), "upload coefficient");
    TRY_HIP(hipEventRecord(staging_done, st), "record staging");
    PassParams pp{};
    pp.tiles = (const TileDesc *)tiles.ptr;
    pp.n_tiles = (int32_t)h_tiles.size();
    pp.xcd_remap = cfg.xcd_remap;
    pp.log2s = log2s;
    pp.col = mat.col;
    pp.val = jval;
    pp.slice_off = mat.slice_off;
    pp.onsite = ac_zero.ptr;
    pp.x = src;
    pp.v = src;
    pp.out = dst;
    pp.coef = (const PassCoef *)coef.ptr;
    pp.counter = (int32_t *)counter.ptr;
    pp.s_user = 1 << log2s;
    hipError_t e = launch_pass(kPassFirst, false, true, false, 1, 1, pp, st);
    if (e != hipSuccess) return hip_fail(e, "launch current operator");
    return TBPM_OK;
}

tbpm_status Engine::bench_pass(int32_t s_user, bool fp32, int32_t n_launch, hipStream_t stream) {
    int32_t s_pad = 1, log2s = 0;
    while (s_pad < s_user) {
        s_pad <<= 1;
        ++log2s;
    }
    if (last_s_pad != s_pad || last_fp32 != (fp32 ? 1 : 0) || !v.ptr || tiles_s != s_pad)
        return fail(TBPM_E_ARG, "tbpm_bench_pass needs a prior tbpm_propagate with the same n_states and precision");
    cfg = cfgs[fp32 ? 1 : 0];
    PassParams pp{};
    pp.tiles = (const TileDesc *)tiles.ptr;
    pp.n_tiles = (int32_t)h_tiles.size();
    pp.xcd_remap = cfg.xcd_remap;
    pp.log2s = log2s;
    pp.bump_counter = 0;
    pp.col = mat.col;
    pp.val = fp32 ? mat.val32 : mat.val64;
    pp.slice_off = mat.slice_off;
    pp.onsite = fp32 ? (const void *)mat.onsite32 : (const void *)mat.onsite64;
    pp.x = ba.ptr;
    pp.v = v.ptr;
    pp.b2 = bb.ptr;
    pp.out = bb.ptr;
    pp.coef = (const PassCoef *)coef.ptr;  // the first pass's coefficients: finite, bounded
    pp.counter = (int32_t *)counter.ptr;
    pp.s_user = s_user;
    pp.uniform_w = last_staged == 1 ? 0 : mat.uniform_w;  // as run() sets it
    pp.uoff = (const int32_t *)st_uoff.ptr;
    pp.ucol = (const int32_t *)st_ucol.ptr;
    pp.lidx = (const uint16_t *)st_lidx.ptr;
    pp.stage_units = stage_units;
    pp.log2ub = last_log2ub;
    if (last_staged == 2) {
        // the interior launch of the fused shape: a MID pair (b_{j+1} in B,
        // b_{j+2} in A, outputs to C and D)
        FusedParams fp{};
        fp.tiles = pp.tiles;
        fp.n_tiles = pp.n_tiles;
        fp.xcd_remap = cfg.xcd_remap;
        fp.log2s = log2s;
        fp.col = mat.col;
        fp.val = pp.val;
        fp.slice_off = mat.slice_off;
        fp.onsite = pp.onsite;
        fp.x = bb.ptr;
        fp.v = v.ptr;
        fp.b2 = ba.ptr;
        fp.out1 = bc.ptr;
        fp.out2 = bd.ptr;
        fp.coef1 = fp.coef2 = pp.coef;
        fp.counter = pp.counter;
        fp.uoff = pp.uoff;
        fp.n1 = (const int32_t *)fu_n1.ptr;
        fp.ucol = pp.ucol;
        fp.lidx = pp.lidx;
        fp.hoff = (const int32_t *)fu_hoff.ptr;
        fp.hw = (const int32_t *)fu_hw.ptr;
        fp.hidx = (const uint16_t *)fu_hidx.ptr;
        fp.lds_units = fu_lds_units;
        fp.uniform_w = mat.uniform_w;
        // as in a time step: each launch reads the two outputs of the one
        // before and walks the tiles the other way
        for (int32_t i = 0; i < n_launch; ++i) {
            const bool odd = (i & 1) != 0;
            fp.x = odd ? bd.ptr : bb.ptr;
            fp.b2 = odd ? bc.ptr : ba.ptr;
            fp.out1 = odd ? ba.ptr : bc.ptr;
            fp.out2 = odd ? bb.ptr : bd.ptr;
            fp.reverse = odd ? 1 : 0;
            hipError_t e = launch_pair(kPairMid, fp32, mat.is_complex, cfg.nontemporal != 0, last_vs, fp, stream);
            if (e != hipSuccess) return hip_fail(e, "launch pair");
        }
        return TBPM_OK;
    }
    // as in a time step: the order just written is the next one's gathered
    // vector, and the tiles are walked the other way
    for (int32_t i = 0; i < n_launch; ++i) {
        const bool odd = (i & 1) != 0;
        pp.x = odd ? bb.ptr : ba.ptr;
        pp.b2 = pp.out = odd ? ba.ptr : bb.ptr;
        pp.reverse = odd ? 1 : 0;
        hipError_t e = last_staged
                           ? launch_pass_staged(kPassMid, fp32, mat.is_complex, cfg.nontemporal != 0, last_vs,
                                                mat.max_width > kStagedWide, pp, stream)
                           : launch_pass(kPassMid, fp32, mat.is_complex, cfg.nontemporal != 0, cfg.unroll, last_vs, pp,
                                         stream);
        if (e != hipSuccess) return hip_fail(e, "launch pass");
    }
    return TBPM_OK;
}

}  // namespace tbpm
