// Internal declarations shared by the host side of libtbpm and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/tbpm.h"
#include "kernel_params.h"

namespace tbpm {

// Device image of the Hamiltonian (sliced ELL, described in kernel_params.h).
struct DevMatrix {
    int64_t n_rows = 0;      // total rows (sum over batch members)
    int64_t n_slices = 0;
    int64_t ell_size = 0;    // slots incl. padding
    int32_t max_width = 0;   // stored elements per row of the widest slice
    int32_t uniform_w = 0;   // that width when every slice has it, else 0
    bool is_complex = false;
    uint32_t *slice_off = nullptr; // [n_slices + 1]
    int32_t *col = nullptr;        // [ell_size]
    void *val64 = nullptr;         // double or double2 [ell_size]
    void *val32 = nullptr;         // float or float2 [ell_size]
    double *onsite64 = nullptr;    // [n_rows]
    float *onsite32 = nullptr;     // [n_rows]
    int64_t *ell_csr = nullptr;    // [ell_size] merged-CSR position of each slot, -1 for padding
    // [n_rows] for each internal row, its row in the caller's order (local to
    // its member); null when every member keeps the caller's order
    int32_t *perm = nullptr;
};

// Host-side image of the sliced ELL build (also used by tests of the layout).
struct HostEll {
    std::vector<int64_t> slice_off;
    std::vector<int32_t> col;
    std::vector<int64_t> csr_pos;
};

// launchers (kernels.hip)
// vs = states per thread (1, 2 or 4; at most the padded state count)
hipError_t launch_pass(int kind, bool fp32, bool cplx, bool nontemporal, int ne, int vs, const PassParams &p,
                       hipStream_t st);
// wide: the matrix has slices wider than kStagedWide stored elements per row
// (the staged pass then walks a row's elements in batches of 12, else of 4)
constexpr int32_t kStagedWide = 8;
// widest state row the staged shape propagates at once (bytes per row)
constexpr int32_t kStagedRowBytes = 128;
hipError_t launch_pass_staged(int kind, bool fp32, bool cplx, bool nontemporal, int vs, bool wide,
                              const PassParams &p, hipStream_t st);
hipError_t launch_init(bool fp32, const InitParams &p, hipStream_t st);
hipError_t launch_reduce(int n_inst, int s_pad, const ReduceParams &p, hipStream_t st);
hipError_t launch_dos(const double *corr, int32_t n_steps, int32_t n_states, double dt, int window,
                      double *energies, double *dos, hipStream_t st);
hipError_t launch_dos_backward(const double *gdos, int32_t n_steps, int32_t n_states, double dt,
                               int window, double *gcorr, hipStream_t st);
hipError_t launch_convert_values(const DevMatrix &m, const double *csr_val, const double *csr_onsite,
                                 int64_t n_rows, hipStream_t st);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st);

// ---------------------------------------------------------------------------
// Adjoint (backward) pass: alpha_{j+1} = 2 H~ alpha_j - alpha_{j-1}
// (alpha_1 = H~ alpha_0), lam_acc += conj(c_{j+1}) alpha_{j+1}, and the
// gradient G_pq += gw * alpha_j[p] * conj(bscale * b_{j+1}[q]) on every stored
// entry and the diagonal, summed over the states.
// ---------------------------------------------------------------------------
enum AdjKind : int {
    kAdjFirst = 0,  // j = 0: no alpha_{j-1}; lam_acc = conj(c_0) alpha_0 + conj(c_1) alpha_1
    kAdjMid = 1,    // 0 < j < M-2
    kAdjFinal = 2   // j = M-2: lam_new = lam_acc + conj(c_{M-1}) alpha_{M-1} + g_l phi0
};

struct AdjParams {
    const TileDesc *tiles;
    int32_t n_tiles;
    int32_t xcd_remap;
    int32_t reverse;  // walk the tiles last to first (see tile_of_block)
    int32_t log2s;
    int32_t s_user;
    const int32_t *col;
    const void *val;        // double or double2 (FP64)
    const uint32_t *slice_off;
    const double *onsite;
    double inv_f;           // 1/f
    const double *a_cur;    // alpha_j (gathered), complex [rows][S]
    const double *a_prev;   // alpha_{j-1} (streamed)
    double *a_next;         // alpha_{j+1} (written; unused by the final pass)
    double *lam_acc;        // complex [rows][S], read-modify-write
    const double *bq;       // b_{j+1} (gathered), complex [rows][S]
    double bs_re, bs_im;    // b_{j+1} = bscale * bq
    double gw;              // gradient weight (1 for j = 0, else 2)
    double cc0_re, cc0_im;  // conj(c_0)   (first pass)
    double ccn_re, ccn_im;  // conj(c_{j+1})
    void *gacc;             // per ELL slot: double (real H) or double2
    double *gdiag;          // [rows] real part of the diagonal gradient
    const double *phi0;     // complex [rows][S] (final pass)
    const double *gcorr_l;  // complex [s_user]: dL/dC at this step (final pass)
    // per ELL slot of (q, p), the slot of (p, q), -1 for padding (the
    // gradient of (p, q) is formed by row q and written there)
    const int32_t *partner;
    int32_t uniform_w;      // stored elements per row when every slice has that width, else 0
};

// Two adjoint orders per launch (backward.hip), on the two-hop tiles of the
// fused shape with single-state units: alpha_j staged, alpha_{j+1} on own and
// 1-hop rows, alpha_{j+2} on own rows, both orders' gradient contributions
// and lambda terms in one read-modify-write.
enum AdjPairKind : int {
    kAdjPairFirst = 0,  // orders 0, 1: alpha_1 = H~ alpha_0, lambda initialised
    kAdjPairMid = 1     // orders j, j+1 (1 <= j, j+2 <= M-2)
};

struct AdjPairParams {
    const TileDesc *tiles;
    int32_t n_tiles;
    int32_t xcd_remap;
    int32_t reverse;  // walk the tiles last to first (see tile_of_block)
    int32_t log2s;
    const int32_t *col;
    const void *val;        // double or double2 (FP64)
    const uint32_t *slice_off;
    const double *onsite;
    double inv_f;
    const double *x;        // alpha_j, complex [rows][S], staged
    const double *a_prev;   // alpha_{j-1} (own and 1-hop rows; null for the first pair)
    double *out1;           // alpha_{j+1}, own rows
    double *out2;           // alpha_{j+2}, own rows
    double *lam_acc;        // lambda accumulator (written by the first pair, else read-modify-write)
    const double *bq1;      // b_{j+1} (gathered)
    const double *bq2;      // b_{j+2} (gathered)
    double w1, w2;          // gradient weights of orders j and j+1
    double cc0_re, cc0_im;  // conj(c_0) (first pair)
    double cc1_re, cc1_im;  // conj(c_{j+1})
    double cc2_re, cc2_im;  // conj(c_{j+2})
    void *gacc;             // per ELL slot: double (real H) or double2
    double *gdiag;          // [rows]
    // per ELL slot of (q, p), the slot of (p, q), -1 for padding: the
    // gradient of (p, q) is formed by own row q from alpha at p (staged) and
    // b at q (own), and written to that slot
    const int32_t *partner;
    // two-hop tile tables (as FusedParams)
    const int32_t *uoff;
    const int32_t *n1;
    const int32_t *ucol;
    const uint16_t *lidx;
    const int32_t *hoff;
    const int32_t *hw;
    const uint16_t *hidx;
    int32_t lds_units;
    int32_t uniform_w;      // stored elements per row when every slice has that width, else 0
};
// vs: states per thread (1, 2 or 4; at most the padded state count);
// lds_units counts units of vs states
hipError_t launch_adjoint_pair(int kind, bool cplx, int vs, const AdjPairParams &p, hipStream_t st);

hipError_t launch_pair(int kind, bool fp32, bool cplx, bool nontemporal, int vs, const FusedParams &p,
                       hipStream_t st);

// quasi-eigenstate launchers (quasi.hip)
// acc[j][e] += coef[k][j] * state[e] for j < n_e, k = *counter (state at R precision)
hipError_t launch_qe_accum(bool fp32, const void *state, double *acc, int64_t n_el, const double *coef, int32_t n_e,
                           const int32_t *counter, hipStream_t st);
int32_t qe_partial_blocks(int64_t n_rows);  // partials need n_e * S * 3 * blocks doubles
// norm2[j][s] = ||acc[j][:, s]||^2 and out[j][perm[r]][s] = acc[j][r][s] / sqrt(norm2[j][s]), s < s_user
hipError_t launch_qe_finalize(const double *acc, int64_t n_rows, int32_t log2s, int32_t s_user, int32_t n_e,
                              const int32_t *perm, double *partials, double *norm2, double *out, hipStream_t st);

// optical-conductivity launchers (ac.hip)
hipError_t launch_gather_values(const int64_t *ell_csr, int64_t ell_size, const double *csr_val, double *ell_val,
                                hipStream_t st);
hipError_t launch_join(const double *jpsi, const double *psi, int64_t n_rows, int32_t log2s, int32_t log2s2,
                       int32_t S, double *out, hipStream_t st);
hipError_t launch_pack(const double *blk, const double *fblk, int64_t n_rows, int32_t log2s2, int32_t S,
                       const int32_t *perm, double *out, hipStream_t st);
hipError_t launch_jcorr(bool fp32, const TileDesc *tiles, int32_t n_tiles, int32_t log2sp, int32_t S, int32_t log2s2,
                        const void *state, const uint32_t *slice_off, const int32_t *col, const double *jval,
                        double *partials, hipStream_t st);
hipError_t launch_ac_cond(const double *corr, int32_t n_steps, int32_t n_states, double dt, double beta, double area,
                          int window, double *omegas, double *sigma, hipStream_t st);
// im[k] = Kramers-Kronig transform of re[0 .. n) on a uniform grid from 0
hipError_t launch_ac_kk(const double *re, int32_t n, double *im, hipStream_t st);
// Chebyshev coefficients a_k of the Fermi-Dirac operator f(H) = sum_k a_k
// T_k(H/rescale) (host); empty if they do not converge below tol
std::vector<double> fermi_cheb_coeffs(double beta, double mu, double rescale, double tol);

// backward launchers (backward.hip)
// Haydock recursion launchers (haydock.hip); mode: 0 a_i, 1 b_{i+1}, 2 initial norm
// uniform_w as in PassParams
hipError_t launch_hay_spmv(bool cplx, const TileDesc *tiles, int32_t n_tiles, int32_t xcd_remap, int32_t log2s,
                           const int32_t *col, const void *val, const uint32_t *slice_off, int32_t uniform_w,
                           const double *onsite, const double *u, const double *uprev, double *y, const double *hs,
                           int32_t *counter, double *partials, hipStream_t st);
hipError_t launch_hay_axpy(const TileDesc *tiles, int32_t n_tiles, int32_t xcd_remap, int32_t reverse, int32_t log2s,
                           const double *y, const double *u, double *unext, const double *hs, double *partials,
                           hipStream_t st);
// Per-state sum of the tile partials and the scalar update of `mode`; above
// 4 kWG tiles the sum runs in two stages through `fold`, which must hold
// hay_fold_count(n_tiles) * s_pad doubles (0: unused).
int32_t hay_fold_count(int32_t n_tiles);
hipError_t launch_hay_reduce(const double *partials, int32_t n_tiles, int32_t s_pad, int32_t s_user, int32_t mode,
                             double thr, double *hs, int32_t *counter, int32_t n_iter, double *a_out, double *b_out,
                             double *fold, hipStream_t st);
hipError_t launch_hay_ldos(const double *a, const double *b, int32_t n_iter, int32_t n_states, const double *energies,
                           int64_t n_e, double eps, double *out, hipStream_t st);

// kernel-polynomial method (kpm.hip)
int32_t kpm_max_moments_lds();
// Moment product parts[c][n][m] = sum over chunk c of conj(L_m) R_n (complex128)
// for L [n_mom], R [cnt] complex128 vectors of ld doubles (even) whose rows
// are stride doubles apart (even, >= ld), chunks of kchunk doubles (a
// multiple of 32), n_chunks = ceil(ld / kchunk).
// shape selects the workgroup tiling (kpm_product_shape): 0 is the default.
struct KpmProductShape {
    int tm, tn, wm;  // 16x16 tiles per wave along m and n; waves along m (of 4)
    int prefetch;    // 1: the next step's operands are loaded before the current products
};
KpmProductShape kpm_product_shape(int32_t shape);
hipError_t launch_kpm_product(int32_t shape, const double *L, const double *R, int64_t stride, int64_t ld,
                              int32_t n_mom, int32_t cnt, int64_t kchunk, int32_t n_chunks, double *parts,
                              hipStream_t st);
// out[i] = scale sum_{p < n_parts} parts[p * part_stride + i] (complex128), p in order
hipError_t launch_kpm_sum_parts(const double *parts, int64_t n_el, int32_t n_parts, int64_t part_stride, double scale,
                                double *out, hipStream_t st);
hipError_t launch_kubo_bastin(const double *mu, int32_t n_mom, double rescale, double th_lo, double dth,
                              int32_t n_energy, const double *mus, int32_t n_mu, double beta, double scale,
                              double *energies, double *weight, double *sigma, hipStream_t st);

hipError_t launch_adjoint_pass(int kind, bool cplx, const AdjParams &p, hipStream_t st);
// dst[r][s] = src[perm[r]][s] (src[r][s] if perm is null), zero for s >= s_user
hipError_t launch_expand_states(const double *src, const int32_t *perm, int32_t s_user, double *dst, int32_t log2s,
                                int64_t n_rows,
                                hipStream_t st);
hipError_t launch_lam_init(double *lam, const double *phi0, const double *gcorr_last, int32_t s_user,
                           int32_t log2s, int64_t n_rows, hipStream_t st);
hipError_t launch_fill_zero(double *p, int64_t n, hipStream_t st);
hipError_t launch_grad_scatter(const void *gacc, const double *gdiag, const int64_t *ell_csr, int64_t ell_size,
                               bool cplx, double inv_f, double *grad_val, double *grad_onsite, const int32_t *perm,
                               int64_t n_rows,
                               hipStream_t st);

// ---------------------------------------------------------------------------
// Host helpers (host.cpp)
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
const std::string &last_error();
int32_t num_terms(double z, double tol);
void bessel_j(double z, int32_t M, double *J);
HostEll build_sliced_ell(int64_t n_rows, const int64_t *row_ptr, const int32_t *col);
// per sliced-ELL slot of element (r, c), the slot of (c, r); -1 for padding;
// empty if some element has no transposed partner
std::vector<int32_t> ell_partner_slots(int64_t n_rows, const std::vector<int64_t> &slice_off,
                                       const std::vector<int32_t> &col);

// Tiles of the fused launch shape: runs of at most R consecutive rows of one
// member (R chosen for the least staged traffic; a run whose staged rows do
// not fit the budget is halved until they do); staged
// rows are the tile's own rows, then its 1-hop rows (neighbours outside the
// tile, sorted), then its 2-hop rows (neighbours of the 1-hop rows outside
// both, sorted).  lidx holds, for each ELL slot of a row, the local index of
// its column in the numbering of that row's tile; hidx holds, per tile, hw
// local indices for each 1-hop row (slot order, zero past the row's width).
struct TwoHopTables {
    int64_t R = 0;                // target rows per tile
    size_t max_x = 0, max_y = 0;  // most staged rows / most rows of b_j in a tile
    size_t max_xy = 0;            // most LDS rows of a tile: staged rows + b_j rows
    std::vector<TileDesc> tiles;
    std::vector<int32_t> inst_tile0, uoff, ucol, n1, hoff, hw;
    std::vector<uint16_t> lidx, hidx;
};
// LDS budget of a fused-shape tile for tier t = 1 .. 6: 1/(t+2) of a CU's
// 160 KiB, i.e. room for t+2 resident workgroups per CU
constexpr int kFusedTiers = 6;
inline size_t fused_lds_budget(int tier) { return (size_t)(160 * 1024 / (tier + 2)) & ~(size_t)255; }

// Host threads for a pass over `work` items (up to 16 from 2^20 items on,
// else one), and f(chunk, lo, hi) run on that many contiguous chunks of
// [0, n), each on its own thread; an exception in a chunk is rethrown as
// std::bad_alloc once every chunk has ended.
int host_threads(int64_t work);
void run_chunks(int64_t n, int threads, const std::function<void(int, int64_t, int64_t)> &f);

// Row order with locality at every scale, without coordinates: recursive
// bisection of the row graph; each part is split at the median of
// d(u, r) - d(v, r) for two pseudo-peripheral rows u, v (graph distances), a
// cut across the middle of the part; parts of at most 'leaf' rows keep the
// breadth-first order from u.  perm[new row] = old row.  The parts of one
// level are processed by up to max_threads host threads (0: up to 16 for
// graphs of at least 2^16 rows, else one); the order does not depend on the
// thread count.
std::vector<int32_t> bisection_order(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t leaf,
                                     int32_t max_threads = 0);
// false if no R fits the LDS budget of budget bytes (units of unit_bytes,
// 2^log2u units per row)
bool two_hop_tables(const std::vector<int64_t> &slice_off, const std::vector<int32_t> &col,
                    const std::vector<int64_t> &inst_row0, int32_t log2u, int32_t unit_bytes, size_t budget,
                    TwoHopTables &t);

}  // namespace tbpm
