// C ABI of libtbpm (declared in include/tbpm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tbpm_engine.h"
#include "tbpm_internal.h"

using namespace tbpm;

namespace tbpm {
tbpm_status backward_impl(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_steps, double dt,
                          double rescale, double tol, const double *grad_corr, int32_t ckpt_every,
                          const double *ckpt, double *grad_val, double *grad_onsite, hipStream_t stream);
tbpm_status autotune_impl(Engine &eng, const std::vector<double> &rescale, int32_t n_states, bool fp32,
                          tbpm_launch_config *best, double *best_ms, hipStream_t stream);
}  // namespace tbpm

namespace {

bool valid_cfg(const tbpm_launch_config &c) {
    const int ok[] = {1, 2, 4, 8, 16, 32};
    return std::find(std::begin(ok), std::end(ok), c.wg_chunks) != std::end(ok) && (c.xcd_remap >= 0 && c.xcd_remap <= 6) &&
           (c.nontemporal == 0 || c.nontemporal == 1) && (c.unroll == 1 || c.unroll == 2) &&
           (c.staged >= 0 && c.staged <= kFusedTiers) && (c.vec == 1 || c.vec == 2 || c.vec == 4) &&
           (c.fused >= 0 && c.fused <= kFusedTiers);
}

double resolve_rescale(const HostCsr &h, double rescale) {
    if (rescale > 0) return rescale;
    return h.gershgorin > 0 ? h.gershgorin : 1.0;
}

// rescale <= 0 selects the Gershgorin bound, which is only known for values
// given on the host: after a device-pointer set_values the caller must pass f
tbpm_status pick_rescale(const HostCsr &h, double rescale, double *f) {
    if (!std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be finite");
    if (rescale <= 0 && h.bound_stale)
        return fail(TBPM_E_ARG,
                    "rescale <= 0 selects the Gershgorin bound, which is not known after values were set from "
                    "device pointers: pass rescale > 0");
    *f = resolve_rescale(h, rescale);
    return TBPM_OK;
}

tbpm_status check_prop_args(int32_t n_states, int32_t n_steps, double dt, double tol, tbpm_precision prec) {
    if (n_states < 1 || n_states > 64) return fail(TBPM_E_ARG, "n_states must be in [1, 64]");
    if (n_steps < 1) return fail(TBPM_E_ARG, "n_steps must be >= 1");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TBPM_E_ARG, "dt must be positive and finite");
    if (!(tol > 0.0 && tol < 1.0)) return fail(TBPM_E_ARG, "bessel_tol must be in (0, 1)");
    if (prec != TBPM_FP64 && prec != TBPM_FP32_MIXED) return fail(TBPM_E_ARG, "unknown precision");
    return TBPM_OK;
}

}  // namespace

// every call on a handle runs on the device the handle was created on
tbpm_status check_device(const Engine &eng) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != eng.device) return fail(TBPM_E_ARG, "handle was created on another device");
    return TBPM_OK;
}

namespace {

// memory of the current device (hipMalloc'd, or a view into it)
bool on_current_device(const void *p) {
    if (!p) return false;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice && a.device == dev;
}

// The CSR arrays given as device pointers, read into host memory: row_ptr
// first (its last entry sizes the rest), checked before the other reads.
tbpm_status read_device_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                            const double *onsite, std::vector<int64_t> &rp, std::vector<int32_t> &ci,
                            std::vector<double> &va, std::vector<double> &on) {
    if (n < 1 || n >= (int64_t)INT32_MAX) return fail(TBPM_E_ARG, "n_orb must be in [1, 2^31)");
    if (!on_current_device(row_ptr) || !on_current_device(onsite))
        return fail(TBPM_E_ARG, "TBPM_FLAG_DEVICE_PTRS: row_ptr and onsite must be device memory of the current device");
    rp.resize(n + 1);
    on.resize(n);
    hipError_t e = hipMemcpy(rp.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(on.data(), onsite, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read device CSR");
    if (rp[0] != 0) return fail(TBPM_E_CSR, "row_ptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(TBPM_E_CSR, "row_ptr must be non-decreasing");
    const int64_t nnz = rp[n];
    ci.resize(nnz);
    va.resize(2 * nnz);
    if (nnz > 0) {
        if (!on_current_device(col) || !on_current_device(val))
            return fail(TBPM_E_ARG, "TBPM_FLAG_DEVICE_PTRS: col_idx and val must be device memory of the current device");
        e = hipMemcpy(ci.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(va.data(), val, sizeof(double) * 2 * nnz, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "read device CSR");
    }
    return TBPM_OK;
}

}  // namespace

extern "C" {

const char *tbpm_version(void) { return "libtbpm 0.1 (gfx950)"; }

tbpm_status tbpm_hamiltonian_create(int64_t n_orb, const int64_t *row_ptr, const int32_t *col_idx,
                                    const double *val, const double *onsite, uint32_t flags,
                                    tbpm_hamiltonian **out) {
    if (!out) return fail(TBPM_E_ARG, "out must not be NULL");
    *out = nullptr;
    if (flags & ~TBPM_FLAG_DEVICE_PTRS) return fail(TBPM_E_ARG, "unknown flags");
    tbpm_hamiltonian *H = new (std::nothrow) tbpm_hamiltonian();
    if (!H) return fail(TBPM_E_OOM, "host allocation failed");
    tbpm_status st;
    try {
        if (flags & TBPM_FLAG_DEVICE_PTRS) {
            std::vector<int64_t> rp;
            std::vector<int32_t> ci;
            std::vector<double> va, on;
            st = read_device_csr(n_orb, row_ptr, col_idx, val, onsite, rp, ci, va, on);
            if (st == TBPM_OK)
                st = canonical_csr(n_orb, rp.data(), ci.data(), va.data(), on.data(), H->csr);
        } else {
            st = canonical_csr(n_orb, row_ptr, col_idx, val, onsite, H->csr);
        }
    } catch (const std::bad_alloc &) {
        st = fail(TBPM_E_OOM, "host allocation failed");
    }
    if (st != TBPM_OK) {
        delete H;
        return st;
    }
    const HostCsr *m = &H->csr;
    try {
        st = H->eng.upload(&m, 1);
    } catch (const std::bad_alloc &) {
        st = fail(TBPM_E_OOM, "host allocation failed");
    }
    if (st != TBPM_OK) {
        H->eng.release();
        delete H;
        return st;
    }
    *out = H;
    return TBPM_OK;
}

tbpm_status tbpm_hamiltonian_set_values(tbpm_hamiltonian *H, const double *val, const double *onsite,
                                        uint32_t flags, void *stream) {
    if (!H) return fail(TBPM_E_ARG, "H must not be NULL");
    const int64_t nnz = H->csr.nnz(), n = H->csr.n;
    if ((nnz > 0 && !val) || !onsite) return fail(TBPM_E_ARG, "val and onsite must not be NULL");
    if (tbpm_status d = check_device(H->eng); d != TBPM_OK) return d;
    hipStream_t st = (hipStream_t)stream;
    if (flags & TBPM_FLAG_DEVICE_PTRS) {
        hipError_t e = launch_convert_values(H->eng.mat, val, onsite, n, st);
        if (e != hipSuccess) return hip_fail(e, "launch value conversion");
        H->csr.bound_stale = true;
        return TBPM_OK;
    }
    HostCsr copy = H->csr;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(onsite[i])) return fail(TBPM_E_ARG, "non-finite on-site energy");
    for (int64_t p = 0; p < 2 * nnz; ++p)
        if (!std::isfinite(val[p])) return fail(TBPM_E_ARG, "non-finite matrix element");
    std::memcpy(copy.val.data(), val, sizeof(double) * 2 * nnz);
    if (!H->csr.is_complex)
        for (int64_t p = 0; p < nnz; ++p) copy.val[2 * p + 1] = 0.0;
    std::memcpy(copy.onsite.data(), onsite, sizeof(double) * n);
    double hmax = 0;
    const bool was_complex = H->csr.is_complex;
    tbpm_status s = check_values(copy, hmax);
    if (s != TBPM_OK) return s;
    copy.is_complex = was_complex;
    copy.bound_stale = false;
    // stage through device scratch and convert with the device path
    double *dval = nullptr, *dons = nullptr;
    hipError_t e = hipMalloc(&dval, sizeof(double) * std::max<int64_t>(2 * nnz, 1));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    e = hipMalloc(&dons, sizeof(double) * n);
    if (e != hipSuccess) {
        (void)hipFree(dval);
        return hip_fail(e, "hipMalloc");
    }
    e = hipMemcpy(dval, copy.val.data(), sizeof(double) * 2 * nnz, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dons, copy.onsite.data(), sizeof(double) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = launch_convert_values(H->eng.mat, dval, dons, n, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dval);
    (void)hipFree(dons);
    if (e != hipSuccess) return hip_fail(e, "set_values");
    H->csr = std::move(copy);
    return TBPM_OK;
}

tbpm_status tbpm_hamiltonian_set_row_order(tbpm_hamiltonian *H, int32_t order) {
    if (!H) return fail(TBPM_E_ARG, "H must not be NULL");
    if (order < -1 || order > 1) return fail(TBPM_E_ARG, "order must be -1, 0 or 1");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != H->eng.device) return fail(TBPM_E_ARG, "handle was created on another device");
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronize before re-upload");
    H->eng.release();
    H->eng.row_order = order;
    H->csr.bound_stale = false;  // the device copy is rebuilt from the host values
    const HostCsr *m = &H->csr;
    try {
        return H->eng.upload(&m, 1);
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
}

tbpm_status tbpm_hamiltonian_get_row_order(const tbpm_hamiltonian *H, int32_t *order) {
    if (!H || !order) return fail(TBPM_E_ARG, "NULL argument");
    *order = (!H->eng.member_perm.empty() && !H->eng.member_perm[0].empty()) ? 1 : 0;
    return TBPM_OK;
}

tbpm_status tbpm_hamiltonian_info(const tbpm_hamiltonian *H, int64_t *n_orb, int64_t *nnz, double *gershgorin,
                                  int32_t *is_complex, int32_t *max_row) {
    if (!H) return fail(TBPM_E_ARG, "H must not be NULL");
    if (n_orb) *n_orb = H->csr.n;
    if (nnz) *nnz = H->csr.nnz();
    if (gershgorin) *gershgorin = H->csr.gershgorin;
    if (is_complex) *is_complex = H->csr.is_complex ? 1 : 0;
    if (max_row) *max_row = (int32_t)H->csr.max_row;
    return TBPM_OK;
}

tbpm_status tbpm_hamiltonian_pattern(const tbpm_hamiltonian *H, int64_t *row_ptr, int32_t *col_idx) {
    if (!H || !row_ptr || (!col_idx && H->csr.nnz() > 0)) return fail(TBPM_E_ARG, "NULL argument");
    std::memcpy(row_ptr, H->csr.row_ptr.data(), sizeof(int64_t) * (H->csr.n + 1));
    if (H->csr.nnz() > 0) std::memcpy(col_idx, H->csr.col.data(), sizeof(int32_t) * H->csr.nnz());
    return TBPM_OK;
}

tbpm_status tbpm_hamiltonian_destroy(tbpm_hamiltonian *H) {
    if (!H) return TBPM_OK;
    H->eng.release();
    delete H;
    return TBPM_OK;
}

tbpm_status tbpm_num_terms(double z, double tol, int32_t *M) {
    if (!M) return fail(TBPM_E_ARG, "M must not be NULL");
    if (!std::isfinite(z) || std::fabs(z) > 1e4) return fail(TBPM_E_ARG, "|z| must be finite and <= 1e4");
    if (!(tol > 0.0 && tol < 1.0)) return fail(TBPM_E_ARG, "tol must be in (0, 1)");
    const int32_t m = num_terms(z, tol);
    if (m < 0) return fail(TBPM_E_ARG, "series does not reach tol");
    *M = m;
    return TBPM_OK;
}

tbpm_status tbpm_bessel_j(double z, int32_t M, double *J) {
    if (!J || M < 1) return fail(TBPM_E_ARG, "J must not be NULL and M >= 1");
    if (!std::isfinite(z) || std::fabs(z) > 1e4) return fail(TBPM_E_ARG, "|z| must be finite and <= 1e4");
    bessel_j(z, M, J);
    return TBPM_OK;
}

tbpm_status tbpm_propagate(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_steps, double dt,
                           double rescale, double bessel_tol, tbpm_precision prec, double *corr, double *norm2,
                           int32_t ckpt_every, double *ckpt, uint32_t flags, void *stream) {
    if (!H || !psi0 || !corr) return fail(TBPM_E_ARG, "H, psi0 and corr must not be NULL");
    tbpm_status st = check_prop_args(n_states, n_steps, dt, bessel_tol, prec);
    if (st != TBPM_OK) return st;
    if (ckpt_every < 0 || (ckpt_every > 0 && !ckpt && n_steps > ckpt_every + 1))
        return fail(TBPM_E_ARG, "ckpt_every must be >= 0 and ckpt non-NULL when checkpoints are due");
    if (ckpt_every > 0 && prec != TBPM_FP64) return fail(TBPM_E_ARG, "checkpoints require TBPM_FP64");
    if (!std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be finite");
    double f = 0.0;
    if (tbpm_status rs = pick_rescale(H->csr, rescale, &f); rs != TBPM_OK) return rs;
    const double *p0 = psi0;
    double *c0 = corr;
    double *n0 = norm2;
    Engine::RunArgs a{};
    a.psi0 = &p0;
    a.s_user = n_states;
    a.n_steps = n_steps;
    a.dt = &dt;
    a.rescale = &f;
    a.tol = bessel_tol;
    a.fp32 = prec == TBPM_FP32_MIXED;
    a.corr = &c0;
    a.norm2 = &n0;
    a.ckpt_every = ckpt_every;
    a.ckpt = ckpt_every > 0 ? ckpt : nullptr;
    a.flags = flags;
    a.stream = (hipStream_t)stream;
    try {
        return H->eng.run(a);
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
}

tbpm_status tbpm_propagate_noalloc(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_steps,
                                   double dt, double rescale, double bessel_tol, tbpm_precision prec, double *corr,
                                   double *norm2, void *stream) {
    if (!H || !psi0 || !corr) return fail(TBPM_E_ARG, "H, psi0 and corr must not be NULL");
    tbpm_status st = check_prop_args(n_states, n_steps, dt, bessel_tol, prec);
    if (st != TBPM_OK) return st;
    if (!std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be finite");
    double f = 0.0;
    if (tbpm_status rs = pick_rescale(H->csr, rescale, &f); rs != TBPM_OK) return rs;
    try {
        return propagate_noalloc(H, psi0, n_states, n_steps, dt, f, bessel_tol, prec == TBPM_FP32_MIXED, corr, norm2,
                                 (hipStream_t)stream);
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
}

tbpm_status tbpm_propagate_snapshots(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, const int32_t *steps,
                                     int32_t n_snap, double dt, double rescale, double bessel_tol,
                                     tbpm_precision prec, double *snaps, double *corr, uint32_t flags,
                                     void *stream) {
    if (!H || !psi0 || !steps || !snaps) return fail(TBPM_E_ARG, "H, psi0, steps and snaps must not be NULL");
    if (n_snap < 1) return fail(TBPM_E_ARG, "n_snap must be >= 1");
    int32_t last = 0;
    std::vector<int32_t> sorted(steps, steps + n_snap);
    std::sort(sorted.begin(), sorted.end());
    if (sorted.front() < 0) return fail(TBPM_E_ARG, "snapshot steps must be >= 0");
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(TBPM_E_ARG, "snapshot steps must be distinct");
    last = sorted.back();
    if (last >= (1 << 28)) return fail(TBPM_E_ARG, "snapshot step too large");
    const int32_t n_steps = last + 1;
    tbpm_status st = check_prop_args(n_states, n_steps, dt, bessel_tol, prec);
    if (st != TBPM_OK) return st;
    if (!std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be finite");
    if (tbpm_status d = check_device(H->eng); d != TBPM_OK) return d;
    double f = 0.0;
    if (tbpm_status rs = pick_rescale(H->csr, rescale, &f); rs != TBPM_OK) return rs;
    hipStream_t hs = (hipStream_t)stream;
    // psi(0) is the caller's state itself
    const size_t snap_bytes = sizeof(double) * 2 * (size_t)H->csr.n * n_states;
    for (int32_t q = 0; q < n_snap; ++q)
        if (steps[q] == 0) {
            hipError_t e = hipMemcpyAsync(snaps + 2 * (size_t)q * H->csr.n * n_states, psi0, snap_bytes,
                                          hipMemcpyDeviceToDevice, hs);
            if (e != hipSuccess) return hip_fail(e, "copy snapshot 0");
        }
    double *c0 = corr;
    if (!c0) {
        hipError_t e = H->eng.corr_scratch.ensure(sizeof(double) * 2 * (size_t)n_steps * n_states);
        if (e != hipSuccess) return hip_fail(e, "alloc correlation scratch");
        c0 = (double *)H->eng.corr_scratch.ptr;
    }
    const double *p0 = psi0;
    double *n0 = nullptr;
    Engine::RunArgs a{};
    a.psi0 = &p0;
    a.s_user = n_states;
    a.n_steps = n_steps;
    a.dt = &dt;
    a.rescale = &f;
    a.tol = bessel_tol;
    a.fp32 = prec == TBPM_FP32_MIXED;
    a.corr = &c0;
    a.norm2 = &n0;
    a.ckpt = snaps;
    a.snap_steps = steps;
    a.n_snap = n_snap;
    a.flags = flags;
    a.stream = hs;
    try {
        return H->eng.run(a);
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
}

tbpm_status tbpm_quasi_eigenstates(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_steps,
                                   double dt, double rescale, double bessel_tol, tbpm_precision prec,
                                   const double *energies, int32_t n_energies, tbpm_window win, double *states,
                                   double *norm2, uint32_t flags, void *stream) {
    if (!H || !psi0 || !energies || !states) return fail(TBPM_E_ARG, "H, psi0, energies and states must not be NULL");
    tbpm_status st = check_prop_args(n_states, n_steps, dt, bessel_tol, prec);
    if (st != TBPM_OK) return st;
    if (n_energies < 1 || n_energies > 256) return fail(TBPM_E_ARG, "n_energies must be in [1, 256]");
    for (int32_t j = 0; j < n_energies; ++j)
        if (!std::isfinite(energies[j])) return fail(TBPM_E_ARG, "energies must be finite");
    if (win != TBPM_WIN_HANN && win != TBPM_WIN_NONE) return fail(TBPM_E_ARG, "unknown window");
    if (!std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be finite");
    double f = 0.0;
    if (tbpm_status rs = pick_rescale(H->csr, rescale, &f); rs != TBPM_OK) return rs;
    Engine &eng = H->eng;
    int32_t s_pad = 1, log2s = 0;
    while (s_pad < n_states) {
        s_pad <<= 1;
        ++log2s;
    }
    const int64_t n_rows = H->csr.n;
    if (tbpm_status d = check_device(eng); d != TBPM_OK) return d;
    hipStream_t hs = (hipStream_t)stream;
    const size_t acc_doubles = 2 * (size_t)n_energies * n_rows * s_pad;
    hipError_t e = eng.qe_acc.ensure(sizeof(double) * acc_doubles);
    if (e == hipSuccess) e = eng.qe_part.ensure(sizeof(double) * 3 * (size_t)n_energies * s_pad *
                                                qe_partial_blocks(n_rows));
    if (e == hipSuccess) e = eng.qe_norm2.ensure(sizeof(double) * (size_t)n_energies * n_states);
    if (e == hipSuccess) e = eng.corr_scratch.ensure(sizeof(double) * 2 * (size_t)n_steps * n_states);
    if (e != hipSuccess) return hip_fail(e, "alloc quasi-eigenstate buffers");
    e = launch_fill_zero((double *)eng.qe_acc.ptr, (int64_t)acc_doubles, hs);
    if (e != hipSuccess) return hip_fail(e, "clear accumulators");
    // coef[k][j] = w_k e^{i E_j t_k} for t_k = +k dt, then -k dt (k = 0 counted once)
    std::vector<double> coef(2 * (size_t)n_steps * n_energies);
    for (int pass = 0; pass < 2; ++pass) {
        const double sgn = pass == 0 ? 1.0 : -1.0;
        for (int32_t k = 0; k < n_steps; ++k) {
            const double w = win == TBPM_WIN_HANN ? 0.5 * (1.0 + std::cos(M_PI * k / n_steps)) : 1.0;
            for (int32_t j = 0; j < n_energies; ++j) {
                const double ph = energies[j] * sgn * k * dt;
                const bool skip = pass == 1 && k == 0;
                coef[2 * ((size_t)k * n_energies + j)] = skip ? 0.0 : w * std::cos(ph);
                coef[2 * ((size_t)k * n_energies + j) + 1] = skip ? 0.0 : w * std::sin(ph);
            }
        }
        const double *p0 = psi0;
        double *c0 = (double *)eng.corr_scratch.ptr;
        double *n0 = nullptr;
        const double dt_run = sgn * dt;
        Engine::RunArgs a{};
        a.psi0 = &p0;
        a.s_user = n_states;
        a.n_steps = n_steps;
        a.dt = &dt_run;
        a.rescale = &f;
        a.tol = bessel_tol;
        a.fp32 = prec == TBPM_FP32_MIXED;
        a.corr = &c0;
        a.norm2 = &n0;
        a.qe_coef = coef.data();
        a.n_qe = n_energies;
        a.qe_acc = (double *)eng.qe_acc.ptr;
        a.flags = flags & ~(uint32_t)TBPM_FLAG_ASYNC;  // the coefficient table is rewritten for the second run
        a.stream = hs;
        try {
            st = eng.run(a);
        } catch (const std::bad_alloc &) {
            st = fail(TBPM_E_OOM, "host allocation failed");
        }
        if (st != TBPM_OK) return st;
    }
    double *n2 = norm2 ? norm2 : (double *)eng.qe_norm2.ptr;
    e = launch_qe_finalize((const double *)eng.qe_acc.ptr, n_rows, log2s, n_states, n_energies, eng.mat.perm,
                           (double *)eng.qe_part.ptr, n2, states, hs);
    if (e != hipSuccess) return hip_fail(e, "launch quasi-eigenstate normalisation");
    if (flags & TBPM_FLAG_ASYNC) return TBPM_OK;
    e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    return TBPM_OK;
}

// j_alpha, j_beta (host, complex128 on H's merged pattern) -> eng.ac_ja,
// eng.ac_jb in the ELL layout of H
static tbpm_status upload_currents(tbpm_hamiltonian *H, const double *j_alpha, const double *j_beta, hipStream_t hs) {
    Engine &eng = H->eng;
    const int64_t nnz = H->csr.nnz();
    for (int64_t p = 0; p < 2 * nnz; ++p)
        if (!std::isfinite(j_alpha[p]) || !std::isfinite(j_beta[p])) return fail(TBPM_E_ARG, "non-finite current value");
    const size_t ell = sizeof(double) * 2 * (size_t)std::max<int64_t>(eng.mat.ell_size, 1);
    hipError_t e = eng.ac_csr.ensure(sizeof(double) * 2 * (size_t)std::max<int64_t>(nnz, 1));
    if (e == hipSuccess) e = eng.ac_ja.ensure(ell);
    if (e == hipSuccess) e = eng.ac_jb.ensure(ell);
    if (e != hipSuccess) return hip_fail(e, "alloc current operators");
    const double *jv[2] = {j_alpha, j_beta};
    DevBuf *jd[2] = {&eng.ac_ja, &eng.ac_jb};
    for (int q = 0; q < 2; ++q) {
        e = hipStreamSynchronize(hs);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpy(eng.ac_csr.ptr, jv[q], sizeof(double) * 2 * (size_t)nnz, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_gather_values(eng.mat.ell_csr, eng.mat.ell_size, (const double *)eng.ac_csr.ptr,
                                     (double *)jd[q]->ptr, hs);
        if (e != hipSuccess) return hip_fail(e, "upload current operator");
    }
    return TBPM_OK;
}

tbpm_status tbpm_ac_corr(tbpm_hamiltonian *H, const double *j_alpha, const double *j_beta, const double *psi0,
                         int32_t n_states, int32_t n_steps, double dt, double rescale, double bessel_tol, double beta,
                         double mu, double fermi_tol, tbpm_precision prec, double *corr, uint32_t flags,
                         void *stream) {
    if (!H || !j_alpha || !j_beta || !psi0 || !corr) return fail(TBPM_E_ARG, "NULL argument");
    if (n_states < 1 || n_states > 32) return fail(TBPM_E_ARG, "n_states must be in [1, 32]");
    tbpm_status st = check_prop_args(2 * n_states, n_steps, dt, bessel_tol, prec);
    if (st != TBPM_OK) return st;
    if (!(beta > 0.0) || !std::isfinite(beta)) return fail(TBPM_E_ARG, "beta must be positive and finite");
    if (!std::isfinite(mu)) return fail(TBPM_E_ARG, "mu must be finite");
    if (!(fermi_tol > 0.0 && fermi_tol < 1e-2)) return fail(TBPM_E_ARG, "fermi_tol must be in (0, 1e-2)");
    if (!std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be finite");
    const int64_t n = H->csr.n;
    if (tbpm_status d = check_device(H->eng); d != TBPM_OK) return d;
    double f = 0.0;
    if (tbpm_status rs = pick_rescale(H->csr, rescale, &f); rs != TBPM_OK) return rs;
    const std::vector<double> a = fermi_cheb_coeffs(beta, mu, f, fermi_tol);
    if (a.empty()) return fail(TBPM_E_ARG, "the Fermi-Dirac expansion needs more than 2^19 terms (beta * rescale too large)");
    Engine &eng = H->eng;
    int32_t s_pad = 1, log2s = 0;
    while (s_pad < n_states) {
        s_pad <<= 1;
        ++log2s;
    }
    const int32_t log2s2 = log2s + 1;  // the joined block [J psi0 | psi0]
    hipStream_t hs = (hipStream_t)stream;
    const size_t vec = sizeof(double) * 2 * (size_t)n * s_pad;
    const size_t vec2 = 2 * vec;
    hipError_t e = eng.ac_vec.ensure(2 * vec + 6 * vec2);
    if (e == hipSuccess) e = eng.ac_block.ensure(sizeof(double) * 4 * (size_t)n * n_states);
    if (e == hipSuccess) e = eng.corr_scratch.ensure(sizeof(double) * 4 * (size_t)n_steps * n_states);
    if (e != hipSuccess) return hip_fail(e, "alloc optical-conductivity buffers");
    st = upload_currents(H, j_alpha, j_beta, hs);
    if (st != TBPM_OK) return st;
    char *vb = (char *)eng.ac_vec.ptr;
    void *src = vb, *jpsi = vb + vec, *blk = vb + 2 * vec, *w0 = vb + 2 * vec + vec2, *w1 = vb + 2 * vec + 2 * vec2,
         *fblk = vb + 2 * vec + 3 * vec2, *w2 = vb + 2 * vec + 4 * vec2, *w3 = vb + 2 * vec + 5 * vec2;
    e = launch_expand_states(psi0, eng.mat.perm, n_states, (double *)src, log2s, n, hs);
    if (e != hipSuccess) return hip_fail(e, "load states");
    try {
        // one series over [J_beta psi0 | psi0]: psi1 = J_beta psi0 - f(H) J_beta psi0,
        // psi2 = f(H) psi0
        st = eng.apply_ell((const double *)eng.ac_jb.ptr, log2s, src, jpsi, hs);
        if (st != TBPM_OK) return st;
        e = launch_join((const double *)jpsi, (const double *)src, n, log2s, log2s2, n_states, (double *)blk, hs);
        if (e != hipSuccess) return hip_fail(e, "join states");
        st = eng.apply_series(a, f, log2s2, blk, fblk, w0, w1, hs, w2, w3);
        if (st != TBPM_OK) return st;
        e = launch_pack((const double *)blk, (const double *)fblk, n, log2s2, n_states, eng.mat.perm,
                        (double *)eng.ac_block.ptr, hs);
        if (e != hipSuccess) return hip_fail(e, "pack states");
        const double *p0 = (const double *)eng.ac_block.ptr;
        double *c0 = (double *)eng.corr_scratch.ptr;
        double *n0 = nullptr;
        Engine::RunArgs r{};
        r.psi0 = &p0;
        r.s_user = 2 * n_states;
        r.n_steps = n_steps;
        r.dt = &dt;
        r.rescale = &f;
        r.tol = bessel_tol;
        r.fp32 = prec == TBPM_FP32_MIXED;
        r.corr = &c0;
        r.norm2 = &n0;
        r.jc_val = (const double *)eng.ac_ja.ptr;
        r.jc_states = n_states;
        r.jc_corr = corr;
        r.flags = flags;
        r.stream = hs;
        return eng.run(r);
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
}

tbpm_status tbpm_kpm_moments(tbpm_hamiltonian *H, const double *v_alpha, const double *v_beta, const double *psi0,
                             int32_t n_states, int32_t n_moments, double rescale, double *mu, double *timing_ms,
                             void *stream) {
    if (!H || !v_alpha || !v_beta || !psi0 || !mu) return fail(TBPM_E_ARG, "NULL argument");
    if (n_states < 1 || n_states > 64) return fail(TBPM_E_ARG, "n_states must be in [1, 64]");
    if (n_moments < 2 || n_moments > 16384) return fail(TBPM_E_ARG, "n_moments must be in [2, 16384]");
    if (!std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be finite");
    if ((int64_t)H->csr.n * 64 >= ((int64_t)1 << 31)) return fail(TBPM_E_ARG, "rows * 64 states must be below 2^31");
    double f = 0.0;
    if (tbpm_status rs = pick_rescale(H->csr, rescale, &f); rs != TBPM_OK) return rs;
    if (tbpm_status d = check_device(H->eng); d != TBPM_OK) return d;
    hipStream_t hs = (hipStream_t)stream;
    try {
        tbpm_status st = upload_currents(H, v_alpha, v_beta, hs);
        if (st != TBPM_OK) return st;
        Engine::KpmTiming t;
        st = H->eng.kpm_moments((const double *)H->eng.ac_ja.ptr, (const double *)H->eng.ac_jb.ptr, psi0, n_states,
                                n_moments, f, mu, hs, timing_ms ? &t : nullptr);
        if (st == TBPM_OK && timing_ms) {
            timing_ms[0] = t.l_ms;
            timing_ms[1] = t.r_ms;
            timing_ms[2] = t.gemm_ms;
            timing_ms[3] = t.n_parts;
        }
        return st;
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
}

tbpm_status tbpm_kubo_bastin(const double *mu, int32_t n_moments, double rescale, double e_lo, double e_hi,
                             int32_t n_energy, double beta, const double *mus, int32_t n_mu, double area,
                             double *energies, double *weight, double *sigma, void *stream) {
    if (!mu || !mus || !energies || !weight || !sigma) return fail(TBPM_E_ARG, "NULL argument");
    if (n_moments < 2 || n_moments > kpm_max_moments_lds())
        return fail(TBPM_E_ARG, "n_moments must be in [2, " + std::to_string(kpm_max_moments_lds()) + "]");
    if (!(rescale > 0.0) || !std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be positive and finite");
    if (!(e_lo > -rescale && e_lo < e_hi && e_hi < rescale))
        return fail(TBPM_E_ARG, "need -rescale < e_lo < e_hi < rescale");
    if (n_energy < 1 || n_mu < 1) return fail(TBPM_E_ARG, "n_energy and n_mu must be positive");
    if (!(beta > 0.0) || !std::isfinite(beta)) return fail(TBPM_E_ARG, "beta must be positive and finite");
    if (!(area > 0.0) || !std::isfinite(area)) return fail(TBPM_E_ARG, "area must be positive and finite");
    const double th_lo = std::acos(e_hi / rescale), th_hi = std::acos(e_lo / rescale);
    const double dth = (th_hi - th_lo) / n_energy;
    const double scale = 4.0 / (M_PI * area * rescale * rescale);
    hipError_t e = launch_kubo_bastin(mu, n_moments, rescale, th_lo, dth, n_energy, mus, n_mu, beta, scale, energies,
                                      weight, sigma, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch Kubo-Bastin integral");
    return TBPM_OK;
}

tbpm_status tbpm_haydock(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_iter, double *a,
                         double *b, uint32_t flags, void *stream) {
    if (!H || !psi0 || !a || !b) return fail(TBPM_E_ARG, "NULL argument");
    if (n_states < 1 || n_states > 64) return fail(TBPM_E_ARG, "n_states must be in [1, 64]");
    if (n_iter < 1 || n_iter > (1 << 24)) return fail(TBPM_E_ARG, "n_iter must be in [1, 2^24]");
    if ((int64_t)H->csr.n * 64 >= ((int64_t)1 << 31)) return fail(TBPM_E_ARG, "rows * 64 states must be below 2^31");
    const double thr = 1e-11 * H->csr.gershgorin;
    if (tbpm_status d = check_device(H->eng); d != TBPM_OK) return d;
    try {
        return H->eng.haydock(psi0, n_states, n_iter, thr, a, b, flags, (hipStream_t)stream);
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
}

tbpm_status tbpm_haydock_ldos(const double *a, const double *b, int32_t n_iter, int32_t n_states,
                              const double *energies, int64_t n_e, double eps, double *ldos, void *stream) {
    if (!a || !b || !energies || !ldos) return fail(TBPM_E_ARG, "NULL argument");
    if (n_iter < 1 || n_states < 1 || n_e < 1 || n_e * n_states > ((int64_t)1 << 31))
        return fail(TBPM_E_ARG, "bad n_iter, n_states or n_e");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(TBPM_E_ARG, "eps must be positive and finite");
    hipError_t e = launch_hay_ldos(a, b, n_iter, n_states, energies, n_e, eps, ldos, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch continued fraction");
    return TBPM_OK;
}

tbpm_status tbpm_fermi_cheb(double beta, double mu, double rescale, double tol, double *a, int32_t cap,
                            int32_t *K) {
    if (!K || (cap > 0 && !a) || cap < 0) return fail(TBPM_E_ARG, "NULL argument or negative capacity");
    if (!(beta > 0.0) || !std::isfinite(beta)) return fail(TBPM_E_ARG, "beta must be positive and finite");
    if (!std::isfinite(mu)) return fail(TBPM_E_ARG, "mu must be finite");
    if (!(rescale > 0.0) || !std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be positive and finite");
    if (!(tol > 0.0 && tol < 1e-2)) return fail(TBPM_E_ARG, "tol must be in (0, 1e-2)");
    try {
        const std::vector<double> c = fermi_cheb_coeffs(beta, mu, rescale, tol);
        if (c.empty()) return fail(TBPM_E_ARG, "the Fermi-Dirac expansion needs more than 2^19 terms");
        *K = (int32_t)c.size();
        std::memcpy(a, c.data(), sizeof(double) * (size_t)std::min<int64_t>(cap, (int64_t)c.size()));
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
    return TBPM_OK;
}

tbpm_status tbpm_ac_cond(const double *corr, int32_t n_steps, int32_t n_states, double dt, double beta, double area,
                         tbpm_window win, double *omegas, double *sigma, void *stream) {
    if (!corr || !omegas || !sigma) return fail(TBPM_E_ARG, "NULL argument");
    if (n_steps < 1 || n_states < 1 || n_steps > (1 << 28)) return fail(TBPM_E_ARG, "bad n_steps or n_states");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TBPM_E_ARG, "dt must be positive and finite");
    if (!(beta > 0.0) || !std::isfinite(beta)) return fail(TBPM_E_ARG, "beta must be positive and finite");
    if (!(area > 0.0) || !std::isfinite(area)) return fail(TBPM_E_ARG, "area must be positive and finite");
    if (win != TBPM_WIN_HANN && win != TBPM_WIN_NONE) return fail(TBPM_E_ARG, "unknown window");
    hipError_t e = launch_ac_cond(corr, n_steps, n_states, dt, beta, area, (int)win, omegas, sigma, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch optical conductivity");
    return TBPM_OK;
}

tbpm_status tbpm_ac_cond_imag(const double *re_sigma, int32_t n, double *im_sigma, void *stream) {
    if (!re_sigma || !im_sigma) return fail(TBPM_E_ARG, "NULL argument");
    if (n < 1 || n > (1 << 17)) return fail(TBPM_E_ARG, "n must be in [1, 2^17] (the transform is a direct O(n^2) sum)");
    if (re_sigma == im_sigma) return fail(TBPM_E_ARG, "re_sigma and im_sigma must not be the same array");
    hipError_t e = launch_ac_kk(re_sigma, n, im_sigma, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch Kramers-Kronig transform");
    return TBPM_OK;
}

tbpm_status tbpm_dos(const double *corr, int32_t n_steps, int32_t n_states, double dt, tbpm_window win,
                     double *energies, double *dos, void *stream) {
    if (!corr || !energies || !dos) return fail(TBPM_E_ARG, "NULL argument");
    if (n_steps < 1 || n_states < 1) return fail(TBPM_E_ARG, "n_steps and n_states must be >= 1");
    if (n_steps > (1 << 28)) return fail(TBPM_E_ARG, "n_steps too large");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TBPM_E_ARG, "dt must be positive and finite");
    if (win != TBPM_WIN_HANN && win != TBPM_WIN_NONE) return fail(TBPM_E_ARG, "unknown window");
    hipError_t e = launch_dos(corr, n_steps, n_states, dt, (int)win, energies, dos, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch dos");
    return TBPM_OK;
}

tbpm_status tbpm_dos_backward(const double *grad_dos, int32_t n_steps, int32_t n_states, double dt,
                              tbpm_window win, double *grad_corr, void *stream) {
    if (!grad_dos || !grad_corr) return fail(TBPM_E_ARG, "NULL argument");
    if (n_steps < 1 || n_states < 1) return fail(TBPM_E_ARG, "n_steps and n_states must be >= 1");
    if (n_steps > (1 << 28)) return fail(TBPM_E_ARG, "n_steps too large");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TBPM_E_ARG, "dt must be positive and finite");
    if (win != TBPM_WIN_HANN && win != TBPM_WIN_NONE) return fail(TBPM_E_ARG, "unknown window");
    hipError_t e = launch_dos_backward(grad_dos, n_steps, n_states, dt, (int)win, grad_corr, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch dos backward");
    return TBPM_OK;
}

tbpm_status tbpm_backward(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_steps, double dt,
                          double rescale, double bessel_tol, const double *grad_corr, int32_t ckpt_every,
                          const double *ckpt, double *grad_val, double *grad_onsite, void *stream) {
    if (!H || !psi0 || !grad_corr || !grad_val || !grad_onsite)
        return fail(TBPM_E_ARG, "NULL argument");
    tbpm_status st = check_prop_args(n_states, n_steps, dt, bessel_tol, TBPM_FP64);
    if (st != TBPM_OK) return st;
    if (ckpt_every < 1) return fail(TBPM_E_ARG, "ckpt_every must be >= 1");
    if (!ckpt && n_steps > ckpt_every + 1) return fail(TBPM_E_ARG, "ckpt must not be NULL");
    if (!std::isfinite(rescale)) return fail(TBPM_E_ARG, "rescale must be finite");
    double f = 0.0;
    if (tbpm_status rs = pick_rescale(H->csr, rescale, &f); rs != TBPM_OK) return rs;
    try {
        return backward_impl(H, psi0, n_states, n_steps, dt, f, bessel_tol, grad_corr, ckpt_every, ckpt, grad_val,
                             grad_onsite, (hipStream_t)stream);
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
}

tbpm_status tbpm_batch_create(tbpm_hamiltonian *const *Hs, int32_t n_ham, tbpm_batch **out) {
    if (!out) return fail(TBPM_E_ARG, "out must not be NULL");
    *out = nullptr;
    if (!Hs || n_ham < 1) return fail(TBPM_E_ARG, "need at least one Hamiltonian");
    std::vector<const HostCsr *> m(n_ham);
    std::vector<const std::vector<int32_t> *> orders(n_ham);
    for (int32_t i = 0; i < n_ham; ++i) {
        if (!Hs[i]) return fail(TBPM_E_ARG, "NULL Hamiltonian in batch");
        m[i] = &Hs[i]->csr;
        // each member keeps the row order of its own handle
        orders[i] = Hs[i]->eng.member_perm.empty() ? nullptr : &Hs[i]->eng.member_perm[0];
    }
    static const std::vector<int32_t> keep;
    for (auto &o : orders)
        if (!o) o = &keep;
    tbpm_batch *B = new (std::nothrow) tbpm_batch();
    if (!B) return fail(TBPM_E_OOM, "host allocation failed");
    B->members.assign(Hs, Hs + n_ham);
    tbpm_status st;
    try {
        st = B->eng.upload(m.data(), n_ham, orders.data());
    } catch (const std::bad_alloc &) {
        st = fail(TBPM_E_OOM, "host allocation failed");
    }
    if (st != TBPM_OK) {
        B->eng.release();
        delete B;
        return st;
    }
    *out = B;
    return TBPM_OK;
}

tbpm_status tbpm_batch_destroy(tbpm_batch *B) {
    if (!B) return TBPM_OK;
    B->eng.release();
    delete B;
    return TBPM_OK;
}

tbpm_status tbpm_propagate_batched(tbpm_batch *B, const double *const *psi0, int32_t n_states, int32_t n_steps,
                                   const double *dt, const double *rescale, double bessel_tol, tbpm_precision prec,
                                   double *const *corr, double *const *norm2, uint32_t flags, void *stream) {
    if (!B || !psi0 || !corr || !dt || !rescale) return fail(TBPM_E_ARG, "NULL argument");
    const int32_t n = (int32_t)B->members.size();
    for (int32_t i = 0; i < n; ++i) {
        if (!psi0[i] || !corr[i]) return fail(TBPM_E_ARG, "NULL psi0/corr entry in batch");
        tbpm_status st = check_prop_args(n_states, n_steps, dt[i], bessel_tol, prec);
        if (st != TBPM_OK) return st;
        if (!std::isfinite(rescale[i])) return fail(TBPM_E_ARG, "rescale must be finite");
    }
    std::vector<double> f(n);
    // the batch holds each member's host values as of tbpm_batch_create, whose bound is known
    for (int32_t i = 0; i < n; ++i) f[i] = resolve_rescale(B->members[i]->csr, rescale[i]);
    Engine::RunArgs a{};
    a.psi0 = psi0;
    a.s_user = n_states;
    a.n_steps = n_steps;
    a.dt = dt;
    a.rescale = f.data();
    a.tol = bessel_tol;
    a.fp32 = prec == TBPM_FP32_MIXED;
    a.corr = corr;
    a.norm2 = norm2;
    a.ckpt_every = 0;
    a.ckpt = nullptr;
    a.flags = flags;
    a.stream = (hipStream_t)stream;
    try {
        return B->eng.run(a);
    } catch (const std::bad_alloc &) {
        return fail(TBPM_E_OOM, "host allocation failed");
    }
}

static bool valid_prec(tbpm_precision p) { return p == TBPM_FP64 || p == TBPM_FP32_MIXED; }

tbpm_status tbpm_get_launch_config(const tbpm_hamiltonian *H, tbpm_precision prec, tbpm_launch_config *cfg) {
    if (!H || !cfg || !valid_prec(prec)) return fail(TBPM_E_ARG, "bad argument");
    *cfg = H->eng.cfgs[prec];
    return TBPM_OK;
}

tbpm_status tbpm_set_launch_config(tbpm_hamiltonian *H, tbpm_precision prec, const tbpm_launch_config *cfg) {
    if (!H || !cfg || !valid_prec(prec)) return fail(TBPM_E_ARG, "bad argument");
    if (!valid_cfg(*cfg)) return fail(TBPM_E_ARG, "invalid launch configuration");
    H->eng.cfgs[prec] = *cfg;
    return TBPM_OK;
}

tbpm_status tbpm_batch_get_launch_config(const tbpm_batch *B, tbpm_precision prec, tbpm_launch_config *cfg) {
    if (!B || !cfg || !valid_prec(prec)) return fail(TBPM_E_ARG, "bad argument");
    *cfg = B->eng.cfgs[prec];
    return TBPM_OK;
}

tbpm_status tbpm_batch_set_launch_config(tbpm_batch *B, tbpm_precision prec, const tbpm_launch_config *cfg) {
    if (!B || !cfg || !valid_prec(prec)) return fail(TBPM_E_ARG, "bad argument");
    if (!valid_cfg(*cfg)) return fail(TBPM_E_ARG, "invalid launch configuration");
    B->eng.cfgs[prec] = *cfg;
    return TBPM_OK;
}

tbpm_status tbpm_autotune(tbpm_hamiltonian *H, int32_t n_states, tbpm_precision prec, tbpm_launch_config *best,
                          double *best_ms, void *stream) {
    if (!H) return fail(TBPM_E_ARG, "H must not be NULL");
    if (n_states < 1 || n_states > 64) return fail(TBPM_E_ARG, "n_states must be in [1, 64]");
    if (tbpm_status d = check_device(H->eng); d != TBPM_OK) return d;
    std::vector<double> f{resolve_rescale(H->csr, 0.0)};
    return autotune_impl(H->eng, f, n_states, prec == TBPM_FP32_MIXED, best, best_ms, (hipStream_t)stream);
}

tbpm_status tbpm_batch_autotune(tbpm_batch *B, int32_t n_states, tbpm_precision prec, tbpm_launch_config *best,
                                double *best_ms, void *stream) {
    if (!B) return fail(TBPM_E_ARG, "B must not be NULL");
    if (n_states < 1 || n_states > 64) return fail(TBPM_E_ARG, "n_states must be in [1, 64]");
    if (tbpm_status d = check_device(B->eng); d != TBPM_OK) return d;
    std::vector<double> f;
    for (auto *h : B->members) f.push_back(resolve_rescale(h->csr, 0.0));
    return autotune_impl(B->eng, f, n_states, prec == TBPM_FP32_MIXED, best, best_ms, (hipStream_t)stream);
}

tbpm_status tbpm_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst || bytes % 16 != 0) return fail(TBPM_E_ARG, "src/dst NULL or bytes not a multiple of 16");
    hipError_t e = launch_copy(src, dst, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch copy");
    return TBPM_OK;
}

tbpm_status tbpm_bench_pass(tbpm_hamiltonian *H, int32_t n_states, tbpm_precision prec, int32_t n_launch,
                            void *stream) {
    if (!H || n_launch < 0) return fail(TBPM_E_ARG, "bad argument");
    if (tbpm_status d = check_device(H->eng); d != TBPM_OK) return d;
    return H->eng.bench_pass(n_states, prec == TBPM_FP32_MIXED, n_launch, (hipStream_t)stream);
}

const char *tbpm_last_error(void) { return tbpm::last_error().c_str(); }

}  // extern "C"
