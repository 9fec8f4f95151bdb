// Internal declarations shared by the host side of libtbpm and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tbpm.h"

namespace tbpm {

// ---------------------------------------------------------------------------
// Device layout
// ---------------------------------------------------------------------------
// Off-diagonal part of H in sliced ELL: slices of kSliceRows consecutive
// rows; slice q holds width_q = (slice_off[q+1]-slice_off[q])/kSliceRows
// entries per row, stored column-major inside the slice, i.e. entry k of
// row r lives at slice_off[q] + k*kSliceRows + (r % kSliceRows).  Rows
// shorter than width_q are padded with (col = row, value = 0).
constexpr int kSliceRows = 32;
// Threads per workgroup of every streaming kernel (4 wave64s).
constexpr int kWG = 256;

// One workgroup's share of a Chebyshev pass: 'rows' consecutive rows of a
// single batch member 'inst', starting at global row 'row0'.
struct TileDesc {
    int64_t row0;
    int32_t rows;
    int32_t inst;
};

// Per-member coefficients of one pass: out = alpha*v + beta*(H x) - b2.
struct PassCoef {
    double ar, ai, br, bi;
};

struct DevMatrix {
    int64_t n_rows = 0;      // total rows (sum over batch members)
    int64_t n_slices = 0;
    int64_t ell_size = 0;    // slots incl. padding
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

// ---------------------------------------------------------------------------
// Kernel launch parameters
// ---------------------------------------------------------------------------
enum PassKind : int {
    kPassFirst = 0,   // x = v, no b2 buffer
    kPassNoB2 = 1,    // no b2 buffer
    kPassMid = 2,     // b2 buffer
    kPassLast = 3,    // b2 buffer, fused correlation
    kPassLastNoB2 = 4 // no b2 buffer, fused correlation
};

struct PassParams {
    const TileDesc *tiles;
    int32_t n_tiles;
    int32_t xcd_remap;
    int32_t log2s;  // log2 of the (padded) number of states
    int32_t bump_counter;
    const int32_t *col;
    const void *val;
    const uint32_t *slice_off;
    const void *onsite;
    const void *x;   // gathered vector (b_{j+1}, or v for the first pass)
    const void *v;   // psi_k
    const void *b2;  // b_{j+2}
    void *out;       // b_j or psi_{k+1}; may alias b2 or v element-wise
    const PassCoef *coef;  // [n_inst] of this pass
    int32_t *counter;      // device step counter
    // fused correlation (last pass)
    const double *phi0;    // complex128 [rows][S]
    int64_t phi0_ld;       // states per row of phi0 (>= S padded or the caller's S)
    double *partials;      // [S][3][n_tiles]
    // stored states (last pass): checkpoints or snapshots of psi(k dt)
    double *ckpt;              // complex128 [n_slots][rows][s_user], rows in the caller's order
    const int32_t *ckpt_slot;  // [n_steps]: slot of psi(k dt) in ckpt, or -1; null: none stored
    const int32_t *perm;       // internal row -> caller's row (single member), or null
    int64_t ckpt_stride;       // complex elements per slot (rows * s_user)
    int32_t s_user;
    // LDS staging (staged launch shape): tile t reads its own rows and the
    // external rows ucol[uoff[t] .. uoff[t+1]); lidx[slot] is the local row of
    // each ELL slot in that staged set
    const int32_t *uoff;
    const int32_t *ucol;
    const uint16_t *lidx;
    int32_t stage_units;   // LDS capacity in units (VS states)
};

// Two Clenshaw orders per launch (fused.hip).
enum PairKind : int {
    kPairFirst = 0,  // b_{M-2}, b_{M-3} from psi (x = psi, no b_{j+2})
    kPairMid = 1     // b_j, b_{j-1} from b_{j+1} (x) and b_{j+2}
};

struct FusedParams {
    const TileDesc *tiles;
    int32_t n_tiles;
    int32_t xcd_remap;
    int32_t log2s;
    int32_t bump_counter;
    const int32_t *col;
    const void *val;
    const uint32_t *slice_off;
    const void *onsite;
    const void *x;     // b_{j+1} (or psi for kPairFirst), staged
    const void *v;     // psi
    const void *b2;    // b_{j+2} (kPairMid)
    void *out1;        // b_j on own rows
    void *out2;        // b_{j-1} on own rows
    const PassCoef *coef1, *coef2;  // [n_inst] for orders j and j-1
    int32_t *counter;
    // 2-hop tiles: staged rows are own, then 1-hop (n1 of them), then 2-hop
    const int32_t *uoff;   // [n_tiles + 1] offsets into ucol
    const int32_t *n1;     // [n_tiles]
    const int32_t *ucol;   // 1-hop then 2-hop global rows of every tile
    const uint16_t *lidx;  // per ELL slot of an own row: local index (own or 1-hop)
    const int32_t *hoff;   // [n_tiles] offset of the tile's 1-hop index block in hidx
    const int32_t *hw;     // [n_tiles] entries per 1-hop row in that block
    const uint16_t *hidx;  // local indices of the stored elements of the 1-hop rows
    int32_t lds_units;     // LDS capacity in units: max over tiles of n_x + n_y
};

struct InitParams {
    const TileDesc *tiles;
    int32_t n_tiles;
    int32_t log2s;
    int32_t s_user;
    const double *const *psi0;   // per member, [N_i][s_user] complex128
    const int64_t *inst_row0;    // per member, first global row
    void *v;                     // state buffer [rows][S] (R precision)
    double *phi0;                // padded FP64 copy [rows][S], or null
    double *partials;            // [S][3][n_tiles]
    int32_t *counter;
    const int32_t *perm;         // internal row -> caller's row in its member, or null
};

struct ReduceParams {
    const double *partials;      // [S][3][n_tiles]
    int32_t n_tiles;
    const int32_t *inst_tile0;   // [n_inst + 1]
    int32_t log2s;
    int32_t s_user;
    int32_t n_steps;
    const int32_t *counter;
    double *const *corr;          // per member [n_steps][s_user] complex128
    double *const *norm2;         // per member, entries may be null
    double *norm2_all;            // [n_inst][n_steps][s_user]
};

// launchers (kernels.hip)
// vs = states per thread (1, 2 or 4; at most the padded state count)
hipError_t launch_pass(int kind, bool fp32, bool cplx, bool nontemporal, int ne, int vs, const PassParams &p,
                       hipStream_t st);
hipError_t launch_pass_staged(int kind, bool fp32, bool cplx, bool nontemporal, int vs, const PassParams &p,
                              hipStream_t st);
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
};

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
// Chebyshev coefficients a_k of the Fermi-Dirac operator f(H) = sum_k a_k
// T_k(H/rescale) (host); empty if they do not converge below tol
std::vector<double> fermi_cheb_coeffs(double beta, double mu, double rescale, double tol);

// backward launchers (backward.hip)
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

// Row order with locality at every scale, without coordinates: recursive
// bisection of the row graph, each part split at the middle of a
// breadth-first order started from a pseudo-peripheral row; parts of at most
// 'leaf' rows keep that breadth-first order.  perm[new row] = old row.
std::vector<int32_t> bisection_order(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t leaf);
// false if no R fits the LDS budget of budget bytes (units of unit_bytes,
// 2^log2u units per row)
bool two_hop_tables(const std::vector<int64_t> &slice_off, const std::vector<int32_t> &col,
                    const std::vector<int64_t> &inst_row0, int32_t log2u, int32_t unit_bytes, size_t budget,
                    TwoHopTables &t);

}  // namespace tbpm
