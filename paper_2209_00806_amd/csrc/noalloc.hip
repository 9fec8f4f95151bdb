// Propagation and correlation (paper, Eq. (eq:psi_t) and Eq. (eq:corr_dos))
// with no device allocation, for callers that cannot allocate (code under
// HIP graph capture, serving loops).  Every work buffer of the Clenshaw
// schedule -- the coefficient and pointer tables, the tile table, the
// correlation partials, the three state-sized work vectors and the padded
// copy of psi0 -- lives in one file-scope device array of fixed size.  The
// kernels are the ones tbpm_propagate launches in its plain shape (one
// Clenshaw order per launch); only the small tables are written here, by a
// set-up kernel that takes them as arguments, so the call enqueues kernels
// only: no allocation, no host copy, no memset, no synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <mutex>
#include <string>
#include <vector>

#include "tbpm_engine.h"

namespace tbpm {
namespace {

// Scratch of the no-allocation entry point: 64 MiB per device, held until
// the process ends.  Every call on a device shares it; overlapping calls on
// one device race.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxPasses = 64;  // series of at most 65 terms
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// byte offsets of the small tables at the start of the scratch
constexpr size_t kOffCoef = 0;       // PassCoef [n_passes]
constexpr size_t kOffPtr = 2048;     // {psi0, corr, norm2}
constexpr size_t kOffRow0 = 2304;    // int64 {0, n_rows}
constexpr size_t kOffTile0 = 2560;   // int32 {0, n_tiles}
constexpr size_t kOffCounter = 2816; // int32 step counter (+ padding)
constexpr size_t kHeadBytes = 4096;  // tiles, partials and vectors follow
static_assert(kOffPtr >= kMaxPasses * sizeof(PassCoef), "coefficient table overlaps the pointer table");

std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device

struct SetupArgs {
    PassCoef coef[kMaxPasses];
    const double *psi0;
    double *corr;
    double *norm2;
    int64_t n_rows;
    int32_t rows_per_tile;
    int32_t n_tiles;
    int32_t n_passes;
};

__global__ __launch_bounds__(kWG) void k_noalloc_setup(const SetupArgs a, unsigned char *base, TileDesc *tiles) {
    if (blockIdx.x == 0) {
        if ((int)threadIdx.x < a.n_passes) ((PassCoef *)(base + kOffCoef))[threadIdx.x] = a.coef[threadIdx.x];
        if (threadIdx.x == 0) {
            const void **pt = (const void **)(base + kOffPtr);
            pt[0] = a.psi0;
            pt[1] = a.corr;
            pt[2] = a.norm2;
            int64_t *r0 = (int64_t *)(base + kOffRow0);
            r0[0] = 0;
            r0[1] = a.n_rows;
            int32_t *t0 = (int32_t *)(base + kOffTile0);
            t0[0] = 0;
            t0[1] = a.n_tiles;
        }
    }
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < a.n_tiles; i += stride) {
        TileDesc d;
        d.row0 = i * a.rows_per_tile;
        const int64_t left = a.n_rows - d.row0;
        d.rows = (int32_t)(left < a.rows_per_tile ? left : a.rows_per_tile);
        d.inst = 0;
        tiles[i] = d;
    }
}

// The device address of `scratch` on device `dev` (which must be current),
// looked up once per device.  In host code `scratch` names a host-side
// stand-in, never the device memory itself.
tbpm_status scratch_base(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(TBPM_E_DEVICE, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(TBPM_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = p;
    }
    *out = (unsigned char *)g_scratch[dev];
    return TBPM_OK;
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

tbpm_status propagate_noalloc(tbpm_hamiltonian *H, const double *psi0, int32_t s_user, int32_t n_steps, double dt,
                              double f, double tol, bool fp32, double *corr, double *norm2, hipStream_t st) {
    Engine &eng = H->eng;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != eng.device) return fail(TBPM_E_ARG, "handle was created on another device");
    if (eng.n_inst() != 1) return fail(TBPM_E_ARG, "the no-allocation entry point takes one Hamiltonian");

    std::vector<std::complex<double>> c;
    const int32_t M = cheb_coeffs(f * dt, tol, c);
    if (M < 0) return fail(TBPM_E_ARG, "Bessel series does not converge for z = " + std::to_string(f * dt));
    if (M - 1 > kMaxPasses)
        return fail(TBPM_E_ARG, "the series has " + std::to_string(M) + " terms; the no-allocation entry point takes " +
                                    std::to_string(kMaxPasses + 1) + " at most");
    const std::vector<PassPlan> plan = plan_step({c}, {f}, M);
    const int32_t n_passes = (int32_t)plan.size();

    const tbpm_launch_config &cf = eng.cfgs[fp32 ? 1 : 0];
    int32_t s_pad = 1, log2s = 0;
    while (s_pad < s_user) {
        s_pad <<= 1;
        ++log2s;
    }
    const int32_t vs = std::min(cf.vec, s_pad);
    const int64_t n = eng.mat.n_rows;
    const int64_t rows_per_tile = std::max<int64_t>(1, (int64_t)kWG * cf.wg_chunks * vs / s_pad);
    const int64_t n_tiles = (n + rows_per_tile - 1) / rows_per_tile;
    const size_t esize = fp32 ? 8 : 16;
    const int64_t n_el = n * s_pad;

    // scratch layout after the small tables, 256-byte aligned pieces
    size_t off = kHeadBytes;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_tiles = take(sizeof(TileDesc) * (size_t)n_tiles);
    const size_t o_part = take(sizeof(double) * 3 * (size_t)n_tiles * s_pad);
    const size_t o_v = take(esize * (size_t)n_el);
    const size_t o_a = take(esize * (size_t)n_el);
    const size_t o_b = take(esize * (size_t)n_el);
    const size_t o_phi0 = take(16 * (size_t)n_el);
    if (off > kScratchBytes)
        return fail(TBPM_E_ARG, "n_orb = " + std::to_string(n) + " with " + std::to_string(s_pad) +
                                    " padded states needs " + std::to_string(off) +
                                    " bytes of work memory; the no-allocation entry point has " +
                                    std::to_string(kScratchBytes) + " (use tbpm_propagate)");

    unsigned char *base = nullptr;
    if (tbpm_status s = scratch_base(dev, &base); s != TBPM_OK) return s;
    TileDesc *tiles = (TileDesc *)(base + o_tiles);
    double *partials = (double *)(base + o_part);
    int32_t *counter = (int32_t *)(base + kOffCounter);
    const PassCoef *coef = (const PassCoef *)(base + kOffCoef);
    const void **ptab = (const void **)(base + kOffPtr);
    void *buf[3] = {base + o_v, base + o_a, base + o_b};
    double *phi0 = (double *)(base + o_phi0);

    SetupArgs sa{};
    for (int32_t p = 0; p < n_passes; ++p) sa.coef[p] = plan[p].coef[0];
    sa.psi0 = psi0;
    sa.corr = corr;
    sa.norm2 = norm2;
    sa.n_rows = n;
    sa.rows_per_tile = (int32_t)rows_per_tile;
    sa.n_tiles = (int32_t)n_tiles;
    sa.n_passes = n_passes;
    const int64_t sblocks = std::min<int64_t>(1024, std::max<int64_t>(1, (n_tiles + kWG - 1) / kWG));
    hipLaunchKernelGGL(k_noalloc_setup, dim3((unsigned)sblocks), dim3(kWG), 0, st, sa, base, tiles);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "launch no-allocation set-up");

    InitParams ip{};
    ip.tiles = tiles;
    ip.n_tiles = (int32_t)n_tiles;
    ip.log2s = log2s;
    ip.s_user = s_user;
    ip.psi0 = (const double *const *)ptab;
    ip.inst_row0 = (const int64_t *)(base + kOffRow0);
    ip.v = buf[0];
    ip.phi0 = phi0;
    ip.partials = partials;
    ip.counter = counter;
    ip.perm = eng.mat.perm;
    e = launch_init(fp32, ip, st);
    if (e != hipSuccess) return hip_fail(e, "launch init");
    ReduceParams rp{};
    rp.partials = partials;
    rp.n_tiles = (int32_t)n_tiles;
    rp.inst_tile0 = (const int32_t *)(base + kOffTile0);
    rp.log2s = log2s;
    rp.s_user = s_user;
    rp.n_steps = n_steps;
    rp.counter = counter;
    rp.corr = (double *const *)(ptab + 1);
    rp.norm2 = (double *const *)(ptab + 2);
    rp.norm2_all = nullptr;
    e = launch_reduce(1, s_pad, rp, st);
    if (e != hipSuccess) return hip_fail(e, "launch reduce");

    const DevMatrix &m = eng.mat;
    for (int32_t k = 1; k < n_steps; ++k) {
        for (int32_t p = 0; p < n_passes; ++p) {
            const PassPlan &pl = plan[p];
            PassParams pp{};
            pp.tiles = tiles;
            pp.n_tiles = (int32_t)n_tiles;
            pp.xcd_remap = cf.xcd_remap;
            pp.log2s = log2s;
            pp.bump_counter = (p == 0);
            pp.col = m.col;
            pp.val = fp32 ? m.val32 : m.val64;
            pp.slice_off = m.slice_off;
            pp.onsite = fp32 ? (const void *)m.onsite32 : (const void *)m.onsite64;
            pp.x = buf[pl.x];
            pp.v = buf[pl.v];
            pp.b2 = pl.b2 >= 0 ? buf[pl.b2] : nullptr;
            pp.out = buf[pl.out];
            pp.coef = coef + p;
            pp.counter = counter;
            pp.phi0 = phi0;
            pp.phi0_ld = s_pad;
            pp.partials = partials;
            pp.s_user = s_user;
            pp.uniform_w = m.uniform_w;
            // consecutive launches walk the tiles in opposite directions
            pp.reverse = (int32_t)(((int64_t)k * n_passes + p) & 1);
            e = launch_pass(pl.kind, fp32, m.is_complex, cf.nontemporal != 0, cf.unroll, vs, pp, st);
            if (e != hipSuccess) return hip_fail(e, "launch pass");
        }
        e = launch_reduce(1, s_pad, rp, st);
        if (e != hipSuccess) return hip_fail(e, "launch reduce");
    }
    return TBPM_OK;
}

}  // namespace tbpm
