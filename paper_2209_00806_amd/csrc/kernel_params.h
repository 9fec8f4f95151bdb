// Launch parameters and layout constants of the propagation kernels (the
// Clenshaw passes, the fused two-order pass, initialisation and the
// correlation reduction): everything these kernels see besides their own
// source and device_util.h.
#pragma once

#include <cstdint>

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
    int32_t uniform_w;     // stored elements per row when every slice has that width, else 0
    int32_t reverse;  // walk the tiles last to first (see tile_of_block)
    // staged launch shape: log2 of the units of one state block of a row (at
    // most log2s - log2 VS); with several blocks, one workgroup per (tile,
    // block) stages and evaluates the tile's rows of that block, so the LDS
    // holds rows of one block
    int32_t log2ub;
};

// Two Clenshaw orders per launch (fused.hip).
enum PairKind : int {
    kPairFirst = 0,  // b_{M-2}, b_{M-3} from psi (x = psi, no b_{j+2})
    kPairMid = 1,    // b_j, b_{j-1} from b_{j+1} (x) and b_{j+2}
    kPairLast = 2,   // b_1 (kept in LDS only) and psi_{k+1} from b_2 (x) and b_3,
                     // with the fused correlation of psi_{k+1}
    kPairSecond = 3  // b_{M-3} (b_{M-1} folded into alpha1, no b_{j+2}) and
                     // b_{M-4} from b_{M-2} (x), after the first order ran alone
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
    void *out1;        // b_j on own rows (not written by kPairLast)
    void *out2;        // b_{j-1} on own rows; never a buffer the launch reads
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
    int32_t uniform_w;     // stored elements per row when every slice has that width, else 0
    int32_t reverse;       // walk the tiles last to first (see tile_of_block)
    // fused correlation (kPairLast): as in PassParams
    const double *phi0;
    int64_t phi0_ld;
    double *partials;
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
    double *norm2_all;            // [n_inst][n_steps][s_user], or null
};

}  // namespace tbpm
