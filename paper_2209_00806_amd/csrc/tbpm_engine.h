// Internal engine of libtbpm: one block-diagonal device operator (a single
// Hamiltonian, or a batch of them concatenated) with its work buffers and
// the cached HIP graph of one time step.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "tbpm_internal.h"

namespace tbpm {

tbpm_status fail(tbpm_status st, const std::string &msg);
tbpm_status hip_fail(hipError_t e, const char *what);

// Merged host CSR (rows in order, columns ascending, no duplicates).
struct HostCsr {
    int64_t n = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<double> val;  // 2 * nnz
    std::vector<double> onsite;
    bool is_complex = false;
    double gershgorin = 0.0;
    // the device values were last replaced from device pointers: gershgorin
    // (and val, onsite) describe the last host values, not the device copy
    bool bound_stale = false;
    int64_t max_row = 0;
    int64_t nnz() const { return (int64_t)col.size(); }
};

tbpm_status canonical_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                          const double *onsite, HostCsr &out);
tbpm_status check_values(HostCsr &h, double &hmax);

// One pass of the Clenshaw schedule of a time step: kernel kind, buffer ids
// (0 = psi, 1 = A, 2 = B, -1 = none) and per-member (alpha, beta).
struct PassPlan {
    int kind;
    int x, v, b2, out;
    std::vector<PassCoef> coef;
};

// c_0 = J_0(z), c_m = 2 (-i)^m J_m(z) for m < M; returns M (or < 0)
int32_t cheb_coeffs(double z, double tol, std::vector<std::complex<double>> &c);
// schedule of one step (passes FIRST, NOB2, MID j = M-4..1, LAST; or FIRST,
// LAST_NOB2 when M = 3) for zero-padded coefficient sets c[i] and scales f[i]
std::vector<PassPlan> plan_step(const std::vector<std::vector<std::complex<double>>> &c,
                                const std::vector<double> &f, int mmax);

// Device buffer that only grows.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need);
    void release();
};

struct PinnedBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need);
    void release();
};

// Everything a time step's launches depend on; a cached graph is reused only
// if the key is equal.
struct GraphKey {
    int32_t s_pad = 0, s_user = 0, fp32 = 0, mmax = 0, n_inst = 0;
    int32_t chunks = 0, remap = 0, nt = 0, unroll = 0, staged = 0, vec = 0, fused = 0;
    // identity of the tile tables the launches were captured with
    int32_t n_tiles = 0, tiles_chunks = 0, tiles_unit = 0, lds_units = 0;
    int32_t n_steps = 0, n_qe = 0, jc_states = 0, steps = 0;
    const void *ckpt = nullptr;
    const void *bufs[22] = {};
    bool operator==(const GraphKey &o) const;
};

struct Engine {
    DevMatrix mat;
    std::vector<int64_t> inst_row0;  // [n_inst + 1]
    tbpm_launch_config cfgs[2] = {{2, 1, 1, 1, 0, 1, 0}, {4, 0, 1, 2, 0, 2, 0}};  // FP64, FP32-mixed
    tbpm_launch_config cfg{2, 1, 1, 1, 0, 1, 0};                                   // the one in use
    // host copy of the sliced ELL columns (for building staged tiles)
    std::vector<int64_t> h_slice_off;
    std::vector<int32_t> h_col;
    // staged tiles: external-row lists and per-slot local indices
    DevBuf st_uoff, st_ucol, st_lidx;
    int32_t stage_units = 0;
    size_t stage_max_rows = 0;  // most staged rows of a tile (units = rows << log2u)
    // two-hop tiles of the fused launch shape, and its two extra work vectors
    DevBuf fu_n1, fu_hoff, fu_hw, fu_hidx, bc, bd;
    int32_t fu_lds_units = 0;
    size_t fu_max_rows = 0;
    int device = -1;

    // work buffers
    DevBuf v, ba, bb, phi0, partials, counter, coef, norm2_all, tiles, inst_tile0, ptr_tab, inst_row0_dev;
    // per-step slot of the stored states (checkpoints or snapshots), and a
    // correlation buffer for calls that do not ask for one
    DevBuf ckpt_slot, corr_scratch;
    // quasi-eigenstates: coefficient table, accumulators, partials, norms
    DevBuf qe_coef, qe_acc, qe_part, qe_norm2;
    // optical conductivity: J_alpha / J_beta in ELL layout, their CSR upload,
    // a zero on-site vector, preparation vectors, the packed block, and the
    // correlation's pointer table and norm scratch
    DevBuf ac_ja, ac_jb, ac_csr, ac_zero, ac_vec, ac_block, jc_tab, jc_norm;
    // Haydock recursion: two Lanczos vectors, the product vector, per-state scalars
    DevBuf hay_u, hay_y, hay_s;
    // kernel-polynomial moments: the L store, a block of R, Chebyshev vectors,
    // per-chunk partial products; the product's workgroup tiling (kpm_product_shape)
    DevBuf kp_store, kp_rblk, kp_vec, kp_parts;
    int32_t kpm_shape = 0;
    // adjoint: segment store, four adjoint vectors, gradient accumulators,
    // and the transposed-slot table of the two-order adjoint (built on first use)
    DevBuf bwd_store, bwd_adj, bwd_gacc, bwd_gdiag, bwd_coef, bwd_partner;
    bool partner_ready = false;
    PinnedBuf staging;
    hipEvent_t staging_done = nullptr;
    hipStream_t capture_stream = nullptr;

    // tile tables (host) for the current (S, chunks)
    // tiles_chunks < 0: staged or two-hop tiles of at most -chunks rows
    // (tiles_unit = unit bytes*64 + log2u, or the two-hop key);
    // else plain tiles of chunks*256 units of tiles_unit = -vs states
    int32_t tiles_s = 0, tiles_chunks = 0, tiles_unit = 0;
    std::vector<TileDesc> h_tiles;
    std::vector<int32_t> h_inst_tile0;

    // cached graphs: several time steps, and one step for the remainder
    hipGraphExec_t graph_exec = nullptr, graph_exec1 = nullptr;
    GraphKey graph_key, graph_key1;

    int32_t n_inst() const { return (int32_t)inst_row0.size() - 1; }

    // row order of each member (empty: the caller's order); mode for new
    // uploads: -1 automatic, 0 the caller's order, 1 bisection order
    std::vector<std::vector<int32_t>> member_perm;
    int32_t row_order = -1;
    // orders: per-member row orders to use instead of choosing them (or null)
    tbpm_status upload(const HostCsr *const *members, int32_t n, const std::vector<int32_t> *const *orders = nullptr);
    void release();

    // the propagation driver (shared by single and batched entry points)
    struct RunArgs;
    struct RunArgs {
        const double *const *psi0;  // n_inst device pointers
        int32_t s_user;
        int32_t n_steps;
        const double *dt;       // n_inst
        const double *rescale;  // n_inst, already resolved (> 0)
        double tol;
        bool fp32;
        double *const *corr;   // n_inst device pointers
        double *const *norm2;  // n_inst device pointers (entries may be null) or null
        int32_t ckpt_every;
        double *ckpt;
        // snapshots of psi(k dt) for the listed steps (k > 0; step 0 is the
        // caller's psi0 and is copied by the caller of run) into ckpt slots;
        // used instead of ckpt_every when n_snap > 0
        const int32_t *snap_steps;
        int32_t n_snap;
        // quasi-eigenstate accumulation: after the initial state and after
        // every step, qe_acc[j] += qe_coef[k][j] psi(k dt) (qe_coef host,
        // complex [n_steps][n_qe]; qe_acc device, [n_qe][rows][S padded])
        const double *qe_coef;
        int32_t n_qe;
        double *qe_acc;
        // optical-conductivity correlation: after the initial state and every
        // step, jc_corr[k][s] = <block[:, S+s]| J |block[:, s]> for s < jc_states
        // (the block holds psi1 in columns 0..S-1 and psi2 in S..2S-1; J as
        // complex128 values in the sliced-ELL layout of H)
        const double *jc_val;
        int32_t jc_states;
        double *jc_corr;
        uint32_t flags;
        hipStream_t stream;
    };
    tbpm_status run(const RunArgs &a);
    // dst = sum_k a[k] T_k(H/f) src on [rows][2^log2s] FP64 internal blocks
    // (Clenshaw; w0, w1 work blocks, and w2, w3 for two orders per launch
    // when the fused shape is configured; src kept)
    tbpm_status apply_series(const std::vector<double> &a, double f, int32_t log2s, const void *src, void *dst,
                             void *w0, void *w1, hipStream_t st, void *w2 = nullptr, void *w3 = nullptr);
    // dst = J src for J given as complex128 values in the ELL layout of H
    tbpm_status apply_ell(const double *jval, int32_t log2s, const void *src, void *dst, hipStream_t st);
    // Haydock (Lanczos) recursion of every column of psi0 (device, caller's
    // order, [rows][s_user] complex128): a_out, b_out device [n_iter][s_user]
    tbpm_status haydock(const double *psi0, int32_t s_user, int32_t n_iter, double thr, double *a_out, double *b_out,
                        uint32_t flags, hipStream_t st);
    // mu[n][m] (complex128, m contiguous) = (1/S) sum_s <r_s| v_a T_m(H/f) v_b T_n(H/f) |r_s>
    // for m, n < n_mom; ja, jb: complex128 values in the ELL layout of H
    struct KpmTiming {
        float l_ms = 0, r_ms = 0, gemm_ms = 0;
        int32_t n_parts = 0;
    };
    tbpm_status kpm_moments(const double *ja, const double *jb, const double *psi0, int32_t s_user, int32_t n_mom,
                            double f, double *mu, hipStream_t st, KpmTiming *timing);
    // back-to-back launches of the interior pass on the current buffers
    tbpm_status bench_pass(int32_t s_user, bool fp32, int32_t n_launch, hipStream_t stream);
    int32_t last_s_pad = 0, last_fp32 = -1, last_staged = 0, last_vs = 1, last_log2ub = 0;

    tbpm_status build_tiles(int32_t s_pad, int32_t chunks, int32_t vs);
    // staged tiles for s_pad states of unit_bytes per VS states (log2u units per row);
    // TBPM_E_ARG if no tile size fits the LDS budget
    tbpm_status build_staged_tiles(int32_t s_pad, int32_t log2u, int32_t unit_bytes, int32_t tier);
    // two-hop tiles for the fused launch shape with the LDS budget of a tier
    // (tiles_chunks = -R, tiles_unit = 2^24 + 16 * row bytes + tier)
    tbpm_status build_fused_tiles(int32_t s_pad, int32_t log2u, int32_t unit_bytes, int32_t tier);
};

}  // namespace tbpm

struct tbpm_hamiltonian {
    tbpm::HostCsr csr;
    tbpm::Engine eng;
};

struct tbpm_batch {
    std::vector<tbpm_hamiltonian *> members;
    tbpm::Engine eng;
};

namespace tbpm {
// tbpm_propagate in the plain launch shape with every work buffer in a fixed
// per-device scratch array (noalloc.hip): enqueues kernels only, no norm check
tbpm_status propagate_noalloc(tbpm_hamiltonian *H, const double *psi0, int32_t s_user, int32_t n_steps, double dt,
                              double f, double tol, bool fp32, double *corr, double *norm2, hipStream_t st);
size_t noalloc_scratch_bytes();
}  // namespace tbpm
