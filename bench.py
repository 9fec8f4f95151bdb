#!/usr/bin/env python3
"""TBPM propagation benchmark on one MI355X.

Workload (one "step" = one pass of the whole TBPM DOS path over one batch):
disordered periodic graphene, 1024 x 1024 cells (2,097,152 orbitals), Anderson
disorder W = 1 eV, 8 random-phase states propagated together, 2048
correlation samples at f = 9 eV, dt = pi/f, Chebyshev terms until
|J_m| < 1e-12 (18 terms, 17 sparse passes per time step), FP64, then the
Hann-windowed DOS on 4096 energies.  Inputs are resident in HBM before the
timed region.

Metric: nnz-updates/s = (stored off-diagonal nnz + N) * S * (M - 1) * (N_t - 1)
per step / step time.  Extra fields report the FP32-mixed form of the same
workload (speed and DOS error against FP64), the dominant kernel against the
HBM roofline, and the CPU oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
KERNEL_SOURCES = ["paper_2209_00806_amd/csrc/kernels.hip", "paper_2209_00806_amd/csrc/device_util.h",
                  "paper_2209_00806_amd/csrc/kernel_params.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_pass_mid_graphene1024_s8_fp64.json")
PAIR_SOURCES = ["paper_2209_00806_amd/csrc/fused.hip", "paper_2209_00806_amd/csrc/device_util.h",
                "paper_2209_00806_amd/csrc/kernel_params.h"]
PAIR_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_pair_mid_graphene1024_s8_fp64.json")


T_START = time.time()


def log(msg):
    print(f"[bench {time.time() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def kernel_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def nnz_updates(n_orb: int, nnz: int, S: int, M: int, nt: int) -> int:
    """Work of a run in the metric's unit: one stored element (off-diagonal or
    on-site) x one state x one sparse pass, over M-1 passes per time step and
    nt-1 time steps."""
    return (nnz + n_orb) * S * (M - 1) * (nt - 1)


def pass_bytes(n_orb: int, nnz: int, S: int, b: int, v: int) -> int:
    """Algorithmic HBM bytes of one Clenshaw pass: 4 state streams (read the
    gathered b_{j+1}, b_{j+2} and psi once, write b_j), the sliced-ELL matrix
    (4-byte column + v-byte value per stored element) and the on-site vector."""
    return 4 * b * n_orb * S + nnz * (4 + v) + n_orb * v


def pair_bytes(n_orb: int, nnz: int, S: int, b: int, v: int) -> int:
    """Bytes one fused launch (two Clenshaw orders) must move at least: 5 state
    streams (read b_{j+1}, b_{j+2} and psi once, write b_j and b_{j-1}) and the
    matrix and on-site vector once."""
    return 5 * b * n_orb * S + nnz * (4 + v) + n_orb * v


def step_bytes(M: int, n_orb: int, nnz: int, S: int, b: int, v: int) -> int:
    """Algorithmic bytes of one time step, independent of the launch schedule:
    M-1 passes of pass_bytes plus the FP64 phi0 stream of the correlation."""
    return (M - 1) * pass_bytes(n_orb, nnz, S, b, v) + 16 * n_orb * S


def hay_iter_bytes(n_orb: int, nnz: int, S: int, b: int, v: int) -> int:
    """Algorithmic bytes of one Haydock iteration over S chains: the product
    pass reads u_i (gathered) and u_{i-1} and writes y, the update reads y and
    u_i and writes u_{i+1} (6 state vectors), plus the matrix and on-site
    energies once."""
    return 6 * b * n_orb * S + nnz * (4 + v) + n_orb * v


def schedule_bytes(M: int, fused: bool, n_orb: int, nnz: int, S: int, b: int, v: int) -> int:
    """Bytes one time step of a plain propagation (no stored states) must move
    at least with the launch schedule in use, plus the phi0 stream: M-1
    passes; or (fused) the last middle order and LAST as one launch (read
    b_2, b_3 and psi, write psi') after the other middle orders in pairs
    (read three vectors, write two), led by FIRST+NOB2 as one launch (read
    psi, write two) when the number of middle orders is odd, else by FIRST
    alone (read psi, write one) and NOB2 with the first middle order (read
    two, write two); with M = 4 (no middle order) FIRST+NOB2, then LAST
    alone."""
    mat = nnz * (4 + v) + n_orb * v
    vec = b * n_orb * S
    phi0 = 16 * n_orb * S
    if not fused or M < 4:
        return (M - 1) * (4 * vec + mat) + phi0
    n_mid = M - 4
    if n_mid == 0:
        return (3 * vec + mat) + (4 * vec + mat) + phi0
    if n_mid % 2:
        lead, rest = (3 * vec + mat), n_mid - 1
    else:
        lead, rest = (2 * vec + mat) + (4 * vec + mat), n_mid - 2
    return lead + (rest // 2) * (5 * vec + mat) + (4 * vec + mat) + phi0


ORACLE_PREFIX = 24  # correlation samples of a member / state the cpu_baseline leg checks against the oracle


def bench_batched(args, log, stash=None):
    """Uneven batch: square/graphene lattices of 1e4..1e6 orbitals with Anderson
    disorder, 4 states each, propagated in one launch sequence (FP64 and FP32).
    The prefixes of state 0 of the smallest, median and largest member go to
    ``stash`` for the oracle check of the cpu_baseline leg."""
    import numpy as np
    import torch

    from paper_2209_00806_amd import inputs, tbpm

    t0 = time.time()
    lats, states = inputs.workload_batch(args.batch_members)
    hams = [tbpm.Hamiltonian.from_lattice(l) for l in lats]
    fs = [h.info()["gershgorin"] for h in hams]
    dts = [math.pi / f for f in fs]
    B = tbpm.Batch(hams)
    psis = [torch.from_numpy(s).cuda() for s in states]
    S = states[0].shape[1]
    nt = args.batch_nt
    tuned = {}
    if not args.no_autotune:
        for prec in ("fp64", "fp32"):
            log(f"batch: autotuning {prec}")
            cfg, ms = B.autotune(S, prec)
            tuned[prec] = cfg
            log(f"batch autotuned {prec}: {cfg} ({ms:.3f} ms per time step)")
    n_orb = sum(l.n_orb for l in lats)
    log(f"batch built: {len(lats)} members, {n_orb} orbitals in {time.time() - t0:.1f}s")
    out = {"members": len(lats), "n_orb_total": n_orb, "n_states": S, "n_steps": nt,
           "sizes_min_max": [min(l.n_orb for l in lats), max(l.n_orb for l in lats)]}
    updates = 0
    alg64 = alg32 = 0
    # every member runs the schedule of the longest series (zero-padded coefficients)
    m_max = max(tbpm.num_terms(f * dt, 1e-12) for f, dt in zip(fs, dts))
    for l, f, dt in zip(lats, fs, dts):
        M = tbpm.num_terms(f * dt, 1e-12)
        updates += (l.nnz + l.n_orb) * S * (M - 1) * (nt - 1)
        alg64 += step_bytes(m_max, l.n_orb, l.nnz, S, 16, 8) * (nt - 1)
        alg32 += step_bytes(m_max, l.n_orb, l.nnz, S, 8, 4) * (nt - 1)
    stream = torch.cuda.current_stream()
    res = {}
    for prec in ("fp64", "fp32"):
        B.propagate(psis, 8, dts, fs, precision=prec)  # warm-up
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        corrs = B.propagate(psis, nt, dts, fs, precision=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[prec] = [c.cpu().numpy() for c in corrs]
        out[prec] = {"ms": round(ms, 1), "nnz_updates_per_s": updates / (ms / 1e3),
                     "alg_GBps": round((alg64 if prec == "fp64" else alg32) / (ms / 1e3) / 1e9, 1)}
        log(f"batched {prec}: {ms:.1f} ms, {updates / (ms / 1e3):.3e} nnz-updates/s")
    errs = []
    for c64, c32, dt in zip(res["fp64"], res["fp32"], dts):
        _, d64 = tbpm.dos(torch.from_numpy(c64).cuda(), dt)
        _, d32 = tbpm.dos(torch.from_numpy(c32).cuda(), dt)
        d64 = d64.cpu().numpy()
        d32 = d32.cpu().numpy()
        errs.append(float(np.sum(np.abs(d32 - d64)) / np.sum(np.abs(d64))))
    out["fp32_dos_l1_rel_err_max_vs_gpu_fp64"] = max(errs)
    out["fp32_speedup_vs_fp64"] = round(out["fp64"]["ms"] / out["fp32"]["ms"], 3)
    if stash is not None:
        order = sorted(range(len(lats)), key=lambda i: lats[i].n_orb)
        picks = [order[0], order[len(order) // 2], order[-1]]
        stash["batch"] = [{"member": i, "lat": lats[i], "psi0": states[i][:, :1].copy(), "dt": dts[i], "f": fs[i],
                           "fp64": res["fp64"][i][:ORACLE_PREFIX, 0].copy(),
                           "fp32": res["fp32"][i][:ORACLE_PREFIX, 0].copy()} for i in picks]
    out["launch"] = tuned or {"fp64": B.launch_config("fp64"), "fp32": B.launch_config("fp32")}
    B.close()
    for h in hams:
        h.close()
    torch.cuda.empty_cache()
    return out


def bench_ldos_psi_t(args, log, cfg64=None):
    """The legs beyond the DOS, all FP64 on 1024^2 graphene: LDOS by
    propagation (8 unit-vector states on the disordered lattice of the
    headline), wave-function snapshots (a Gaussian packet in the pristine
    lattice, 1 state, snapshots at steps 0, 16, 32, 64, 128 as in the
    usage-section example), quasi-eigenstates, the optical conductivity,
    the Haydock LDOS and the Kubo-Bastin conductivity (one random-phase state
    or the 8 orbitals on the disordered lattice)."""
    import numpy as np
    import torch

    from paper_2209_00806_amd import inputs, tbpm

    out = {}
    stream = torch.cuda.current_stream()
    f = 9.0
    dt = math.pi / f
    M = tbpm.num_terms(f * dt, 1e-12)
    lat, _ = inputs.workload_disordered_graphene(args.cells, 1)
    H = tbpm.Hamiltonian.from_lattice(lat)
    if cfg64:  # the headline's autotuned shape (same operator and state count)
        H.set_launch_config(precision="fp64", **cfg64)
    orbs = np.linspace(0, lat.n_orb - 1, 8).astype(np.int64)
    nt = args.ldos_nt
    tbpm.ldos(H, orbs, 8, dt, f)  # warm-up (tiles, graph)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    _, D = tbpm.ldos(H, orbs, nt, dt, f)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    upd = (lat.nnz + lat.n_orb) * len(orbs) * (M - 1) * (nt - 1)
    out["ldos"] = {"orbitals": len(orbs), "n_steps": nt, "ms": round(ms, 1), "nnz_updates_per_s": upd / (ms / 1e3),
                   "alg_GBps": round(step_bytes(M, lat.n_orb, lat.nnz, len(orbs), 16, 8) * (nt - 1) / (ms / 1e3) / 1e9,
                                     1),
                   "ldos_integral": float(D.sum().item() * (2 * f / (2 * nt)))}
    log(f"ldos: 8 orbitals, {nt} samples, {ms:.1f} ms, {upd / (ms / 1e3):.3e} nnz-updates/s")
    H.close()
    del H
    lat = inputs.graphene(args.cells, args.cells)
    pos = inputs.graphene_positions(args.cells, args.cells)
    psi0 = torch.from_numpy(inputs.gaussian_packet(pos, pos[:, :2].mean(axis=0), sigma=5.0)).cuda()
    H = tbpm.Hamiltonian.from_lattice(lat)
    if cfg64:
        H.set_launch_config(precision="fp64", **cfg64)
    steps = [0, 16, 32, 64, 128]
    tbpm.propagate_snapshots(H, psi0, [0, 4], dt, f)  # warm-up
    torch.cuda.synchronize()
    e0.record(stream)
    snaps = tbpm.propagate_snapshots(H, psi0, steps, dt, f)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    upd = (lat.nnz + lat.n_orb) * (M - 1) * max(steps)
    norms = [float(torch.linalg.norm(snaps[q]).item()) for q in range(len(steps))]
    out["psi_t"] = {"n_orb": lat.n_orb, "steps": steps, "ms": round(ms, 2), "nnz_updates_per_s": upd / (ms / 1e3),
                    "alg_GBps": round(step_bytes(M, lat.n_orb, lat.nnz, 1, 16, 8) * max(steps) / (ms / 1e3) / 1e9, 1),
                    "max_norm_dev": max(abs(x - 1) for x in norms)}
    log(f"psi_t: {len(steps)} snapshots over {max(steps)} steps, {ms:.1f} ms, {upd / (ms / 1e3):.3e} nnz-updates/s")
    H.close()
    # quasi-eigenstates: 8 energies, one random-phase state on the disordered
    # lattice, 256 samples forward and backward
    lat, psi_np = inputs.workload_disordered_graphene(args.cells, 1)
    H = tbpm.Hamiltonian.from_lattice(lat)
    if cfg64:
        H.set_launch_config(precision="fp64", **cfg64)
    psi = torch.from_numpy(psi_np).cuda()
    en = [-6.0, -4.0, -2.7, -1.0, 0.3, 1.0, 2.7, 5.0]
    nq = 256
    tbpm.quasi_eigenstates(H, psi, en, 8, dt, f)  # warm-up
    torch.cuda.synchronize()
    e0.record(stream)
    qs, qn2 = tbpm.quasi_eigenstates(H, psi, en, nq, dt, f, return_norm=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_q = e0.elapsed_time(e1)
    e0.record(stream)
    tbpm.propagate(H, psi, nq, dt, f)
    tbpm.propagate(H, psi, nq, dt, f)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1)
    acc_bytes = (16 + 32 * len(en)) * lat.n_orb * 2 * (nq - 1)
    out["quasi_eigenstates"] = {"energies": len(en), "n_steps": nq, "ms": round(ms_q, 1),
                                "ms_propagation_only": round(ms_p, 1),
                                "accumulation_GBps": round(acc_bytes / max(ms_q - ms_p, 1e-3) / 1e6, 1),
                                "norm2_min_max": [float(qn2.min()), float(qn2.max())]}
    log(f"quasi-eigenstates: {len(en)} energies, 2 x {nq} samples, {ms_q:.1f} ms ({ms_p:.1f} ms propagation alone)")
    # optical conductivity sigma_xx at 300 K, mu = 0, one random-phase state on
    # the same disordered lattice: the Fermi-Dirac series over the joined
    # block [J psi0 | psi0], then both states propagated together
    jx = inputs.current_values(lat, 0)
    beta, mu = 38.68, 0.0
    na = args.ac_nt
    K = len(tbpm.fermi_coeffs(beta, mu, f, 1e-12))
    tbpm.ac_corr(H, jx, jx, psi, 8, dt, beta, mu, rescale=f)  # warm-up
    torch.cuda.synchronize()
    e0.record(stream)
    corr = tbpm.ac_corr(H, jx, jx, psi, na, dt, beta, mu, rescale=f)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_a = e0.elapsed_time(e1)
    psi2 = psi.repeat(1, 2).contiguous()
    tbpm.propagate(H, psi2, 8, dt, f)
    torch.cuda.synchronize()
    e0.record(stream)
    tbpm.propagate(H, psi2, na, dt, f)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_p2 = e0.elapsed_time(e1)
    om, sg = tbpm.ac_cond(corr, dt, beta, lat.area / lat.n_orb)
    im_sg = tbpm.ac_cond_imag(sg).cpu().numpy()
    om = om.cpu().numpy()
    sg = sg.cpu().numpy()
    band = (om > 0.9) & (om < 2.1)
    series_bytes = (K - 1) * pass_bytes(lat.n_orb, lat.nnz, 2, 16, 8)
    out["optical_conductivity"] = {
        "n_steps": na, "beta_per_eV": beta, "fermi_terms": K, "ms": round(ms_a, 1),
        "ms_propagation_only": round(ms_p2, 1),
        "series_alg_GBps": round(series_bytes / max(ms_a - ms_p2, 1e-3) / 1e6, 1),
        "sigma_xx_over_e2_8hbar_0.9_2.1eV": round(float(np.mean(sg[band]) / 0.125), 3),
        "im_sigma_xx_over_e2_8hbar_at_1_2_eV": [round(float(np.interp(w, om, im_sg)) / 0.125, 3) for w in (1.0, 2.0)]}
    log(f"optical conductivity: {K} Fermi terms, {na} steps, {ms_a:.1f} ms ({ms_p2:.1f} ms propagation alone), "
        f"sigma_xx/(e^2/8hbar) = {np.mean(sg[band]) / 0.125:.3f} at 0.9-2.1 eV")
    # LDOS by the Haydock recursion: the 8 orbitals of the LDOS leg, one
    # Lanczos chain each, advanced together
    st = torch.zeros((lat.n_orb, len(orbs)), dtype=torch.complex128, device="cuda")
    st[torch.as_tensor(orbs, device="cuda"), torch.arange(len(orbs), device="cuda")] = 1.0
    nh = args.hay_iter
    tbpm.haydock(H, st, 8)  # warm-up (tiles, buffers)
    torch.cuda.synchronize()
    e0.record(stream)
    ha, hb = tbpm.haydock(H, st, nh)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_h = e0.elapsed_time(e1)
    en_h = torch.linspace(-10.0, 10.0, 4001, dtype=torch.float64, device="cuda")
    dh = tbpm.haydock_ldos(ha, hb, en_h, 0.02).mean(dim=1)
    hay_bytes = hay_iter_bytes(lat.n_orb, lat.nnz, len(orbs), 16, 8) * nh
    out["haydock"] = {"orbitals": len(orbs), "iterations": nh, "ms": round(ms_h, 1),
                      "us_per_iteration": round(1e3 * ms_h / nh, 1),
                      "alg_GBps": round(hay_bytes / (ms_h / 1e3) / 1e9, 1),
                      "ldos_integral_pm10eV": round(float(dh.sum().item() * 20.0 / 4000), 4)}
    log(f"haydock: 8 orbitals, {nh} iterations, {ms_h:.1f} ms, {hay_bytes / (ms_h / 1e3) / 1e9:.0f} GB/s")
    # Kubo-Bastin sigma_xx by the kernel polynomial method: one random-phase
    # state on the disordered lattice, M moments; the moment product L^H R is
    # the library's own complex FP64 product kernel on the matrix cores
    # (k_kpm_product)
    nm = args.kpm_moments
    tbpm.kpm_moments(H, jx, jx, psi, 16, f)  # warm-up (handle, tiles)
    torch.cuda.synchronize()
    e0.record(stream)
    mu_k, tk = tbpm.kpm_moments(H, jx, jx, psi, nm, f, return_timing=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_k = e0.elapsed_time(e1)
    mus_k = [-2.0, -1.0, -0.5, 0.0, 0.5, 1.0, 2.0]
    sk, _, _ = tbpm.kubo_bastin(mu_k, f, -0.98 * f, 0.98 * f, 2 * nm, 38.68, mus_k, lat.area / lat.n_orb)
    product_flops = 8.0 * nm * nm * lat.n_orb
    # a Chebyshev order reads the gathered T_m and T_{m-1} and writes T_{m+1}
    # (3 streams); the current operator reads its input and writes its output
    # (2 streams) with complex values
    cheb_b = 3 * 16 * lat.n_orb + lat.nnz * 12 + lat.n_orb * 8
    cur_b = 2 * 16 * lat.n_orb + lat.nnz * 20 + lat.n_orb * 8
    pass_b = nm * cheb_b * 2 + nm * cur_b
    out["kubo_bastin"] = {
        "moments": nm, "states": 1, "ms": round(ms_k, 1), "l_recursion_ms": round(tk["l_ms"], 1),
        "r_recursion_ms": round(tk["r_ms"], 1), "product_ms": round(tk["product_ms"], 1), "product_chunks": tk["chunks"],
        "product_kernel": "k_kpm_product (library's own FP64 MFMA kernel)",
        "product_TFLOPs": round(product_flops / (tk["product_ms"] / 1e3) / 1e12, 2),
        "product_frac_of_fp64_mfma_peak": round(product_flops / (tk["product_ms"] / 1e3) / 78.6e12, 3),
        "recursion_alg_GBps": round(pass_b / ((tk["l_ms"] + tk["r_ms"]) / 1e3) / 1e9, 1),
        "sigma_xx_e2_over_h": {str(m): round(float(v) * 2 * math.pi, 4) for m, v in zip(mus_k, sk.cpu().numpy())}}
    log(f"kubo-bastin: {nm} moments, {ms_k:.1f} ms (recursions {tk['l_ms'] + tk['r_ms']:.1f} ms, product "
        f"{tk['product_ms']:.1f} ms = {product_flops / (tk['product_ms'] / 1e3) / 1e12:.1f} TFLOP/s)")
    del mu_k
    H.close()
    return out


def bench_tbg(args, log, stash=None):
    """Twisted bilayer flake (two 1024^2-cell layers, 1.05 deg, ~19 stored elements per
    row, irregular rows, open boundaries): 16 states, 1024 steps, FP32-mixed, with a
    full FP64 run of the same states for the DOS error."""
    import numpy as np
    import torch

    from paper_2209_00806_amd import inputs, tbpm

    t0 = time.time()
    lat, psi0_np = inputs.workload_twisted_bilayer(args.tbg_cells, 16)
    H = tbpm.Hamiltonian.from_lattice(lat)
    f = H.info()["gershgorin"]
    dt = math.pi / f
    nt = args.tbg_nt
    M = tbpm.num_terms(f * dt, 1e-12)
    psi0 = torch.from_numpy(psi0_np).cuda()
    psi0_s0 = psi0_np[:, :1].copy()
    del psi0_np
    log(f"twisted bilayer built: N={lat.n_orb}, nnz={lat.nnz} ({lat.nnz / lat.n_orb:.1f}/row), "
        f"f={f:.3f} eV in {time.time() - t0:.1f}s")
    updates = nnz_updates(lat.n_orb, lat.nnz, 16, M, nt)
    stream = torch.cuda.current_stream()
    out = {"n_orb": lat.n_orb, "nnz_offdiag": lat.nnz, "nnz_per_row": round(lat.nnz / lat.n_orb, 2),
           "max_row": H.info()["max_row"], "n_states": 16, "n_steps": nt, "rescale_eV": f}
    res = {}
    prefix = {}
    for prec in ("fp32", "fp64"):
        log(f"tbg {prec}: autotuning")
        cfg, ms_t, _ = tbpm.autotune_cached(H, 16, prec, args.tune_cache)
        tbpm.propagate(H, psi0, 4, dt, f, precision=prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        corr = tbpm.propagate(H, psi0, nt, dt, f, precision=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        b, v = (8, 4) if prec == "fp32" else (16, 8)
        alg = step_bytes(M, lat.n_orb, lat.nnz, 16, b, v) * (nt - 1)
        _, D = tbpm.dos(corr, dt)
        res[prec] = D.cpu().numpy()
        prefix[prec] = corr[:TBG_PREFIX, 0].cpu().numpy()
        out[prec] = {"ms": round(ms, 1), "nnz_updates_per_s": updates / (ms / 1e3),
                     "alg_GBps": round(alg / (ms / 1e3) / 1e9, 1), "launch": cfg}
        log(f"tbg {prec}: {ms:.1f} ms, {updates / (ms / 1e3):.3e} nnz-updates/s, {alg / (ms / 1e3) / 1e9:.0f} GB/s")
    out["fp32_dos_l1_rel_err_vs_gpu_fp64"] = float(np.sum(np.abs(res["fp32"] - res["fp64"]))
                                                  / np.sum(np.abs(res["fp64"])))
    out["fp32_speedup_vs_fp64"] = round(out["fp64"]["ms"] / out["fp32"]["ms"], 3)
    if stash is not None:
        stash["tbg"] = {"lat": lat, "psi0": psi0_s0, "dt": dt, "f": f, **prefix}
    H.close()
    torch.cuda.empty_cache()
    return out


TBG_PREFIX = 8  # correlation samples of state 0 of the twisted bilayer checked against the oracle


def bench_backward(args, log):
    """Differentiable DOS: graphene with per-bond hoppings, loss = sum over 256
    energies of (D(E) - target)^2; forward and backward (adjoint) timed."""
    import numpy as np
    import torch

    from paper_2209_00806_amd import autograd as ag
    from paper_2209_00806_amd import inputs, tbpm

    t0 = time.time()
    lat, target_lat, psi0_np = inputs.workload_bond_graphene(args.bwd_cells, 4)
    f = 9.0
    dt = math.pi / f
    nt = args.bwd_nt
    K = 64
    psi0 = torch.from_numpy(psi0_np).cuda()
    Ht = tbpm.Hamiltonian.from_lattice(target_lat)
    _, target = tbpm.dos(tbpm.propagate(Ht, psi0, nt, dt, f), dt)
    Ht.close()
    H = tbpm.Hamiltonian.from_lattice(lat)
    slot_ij = torch.from_numpy(lat.slot_ij).cuda()
    slot_ji = torch.from_numpy(lat.slot_ji).cuda()
    sel = torch.arange(0, 2 * nt, 8, device="cuda")  # 256 energies
    t_param = torch.from_numpy(lat.bond_t.copy()).cuda().requires_grad_(True)
    e_param = torch.zeros(lat.n_orb, dtype=torch.float64, device="cuda", requires_grad=True)
    log(f"backward workload built: N={lat.n_orb}, {lat.bond_t.shape[0]} bonds in {time.time() - t0:.1f}s")

    def forward(n=nt):
        val = ag.bond_values(lat.nnz, slot_ij, slot_ji, t_param)
        _, D = ag.tbpm_dos(H, val, e_param, psi0, n, dt, f, ckpt_every=K)
        if n != nt:
            return torch.sum(D ** 2)
        return torch.sum((D[sel] - target[sel]) ** 2)

    # one launch shape serves the forward, the segment replay and the adjoint.
    # The autotuner times the forward alone, where the plain and the fused
    # shapes can tie on this cache-resident lattice while the backward runs
    # much faster fused (two adjoint orders per launch), so the shape is
    # chosen on a short forward + backward among the tuner's pick and the
    # fused shape at LDS tiers 2-4, with one contiguous range of tiles per XCD
    # or runs of 16 tiles dealt to the XCDs in turn
    cfg, _, _ = tbpm.autotune_cached(H, 4, "fp64", args.tune_cache)
    cands = [cfg]
    for tier in (2, 3, 4):
        for remap in (1, 4):
            c = {"wg_chunks": 2, "xcd_remap": remap, "nontemporal": 1, "unroll": 1, "staged": 0, "vec": 2,
                 "fused": tier}
            if all(c != d for d in cands):
                cands.append(c)
    trials = []
    for c in cands:
        H.set_launch_config(c["wg_chunks"], c["xcd_remap"], c["nontemporal"], c["unroll"], c.get("staged", 0),
                            c.get("vec"), precision="fp64", fused=c.get("fused", 0))
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            Lt = forward(256)
            Lt.backward()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - ta) * 1e3
            best = ms if best is None else min(best, ms)
        t_param.grad = None
        e_param.grad = None
        trials.append({"launch": c, "ms_forward_backward_256_steps": round(best, 2)})
    cfg = min(trials, key=lambda t: t["ms_forward_backward_256_steps"])["launch"]
    H.set_launch_config(cfg["wg_chunks"], cfg["xcd_remap"], cfg["nontemporal"], cfg["unroll"], cfg.get("staged", 0),
                        cfg.get("vec"), precision="fp64", fused=cfg.get("fused", 0))

    L = forward()  # warm-up
    L.backward()
    torch.cuda.synchronize()
    t_param.grad = None
    e_param.grad = None
    stream = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(stream)
    L = forward()
    e1.record(stream)
    L.backward()
    e2.record(stream)
    torch.cuda.synchronize()
    fwd = e0.elapsed_time(e1)
    bwd = e1.elapsed_time(e2)
    g = t_param.grad
    out = {"n_orb": lat.n_orb, "bond_params": int(lat.bond_t.shape[0]), "n_states": 4, "n_steps": nt,
           "ckpt_every": K, "launch": cfg, "launch_trials": trials, "loss": L.item(), "forward_ms": round(fwd, 2),
           "backward_ms": round(bwd, 2),
           "backward_over_forward": round(bwd / fwd, 3), "grad_norm": float(torch.linalg.norm(g).item())}
    log(f"backward: fwd {fwd:.1f} ms, bwd {bwd:.1f} ms, ratio {bwd / fwd:.2f}")
    H.close()
    torch.cuda.empty_cache()
    del np
    return out


def bench_small(args, log, stash=None):
    """Clean periodic graphene 64 x 64 cells (8192 orbitals), 1 random-phase
    state, 512 correlation samples, f = 9 eV, dt = pi/f, FP64, then the Hann
    DOS on 1024 energies.  Its vectors (131 KB) stay in the caches, so the run
    is bound by launch and latency, not by HBM: the figure is the time of a
    whole run and per time step."""
    import torch

    from paper_2209_00806_amd import inputs, tbpm

    lat, psi0_np = inputs.workload_graphene_dos(args.small_cells, 1)
    f = 9.0
    dt = math.pi / f
    nt = args.small_nt
    H = tbpm.Hamiltonian.from_lattice(lat)
    cfg, _, _ = tbpm.autotune_cached(H, 1, "fp64", args.tune_cache)
    psi0 = torch.from_numpy(psi0_np).cuda()
    M = tbpm.num_terms(f * dt, 1e-12)

    def run():
        corr = tbpm.propagate(H, psi0, nt, dt, f)
        _, D = tbpm.dos(corr, dt)
        return corr, D

    for _ in range(3):
        run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = args.small_reps
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        corr, D = run()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_wall) / reps * 1e3
    ms = e0.elapsed_time(e1) / reps
    fused = cfg.get("fused", 0) > 0 and M >= 4
    # launches of one time step: the passes (paired in the fused shape) and the correlation reduce
    launches = (1 + (M - 4) // 2 + (M - 4) % 2 + 1 if fused else M - 1) + 1
    updates = nnz_updates(lat.n_orb, lat.nnz, 1, M, nt)
    out = {"workload": f"clean periodic graphene {args.small_cells}x{args.small_cells} cells ({lat.n_orb} orbitals), "
                       f"1 random-phase state, {nt} correlation samples, f=9 eV, dt=pi/f, FP64, "
                       f"Hann DOS on {2 * nt} energies",
           "ms_per_run": round(ms, 3), "wall_ms_per_run": round(wall, 3),
           "us_per_time_step": round(1e3 * ms / (nt - 1), 2), "launches_per_time_step": launches,
           "us_per_launch": round(1e3 * ms / (nt - 1) / launches, 2),
           "nnz_updates_per_s": updates / (ms / 1e3),
           "alg_GBps_cache_resident": round(step_bytes(M, lat.n_orb, lat.nnz, 1, 16, 8) * (nt - 1)
                                            / (ms / 1e3) / 1e9, 1),
           "note": "working set ~0.5 MB, served by the caches: launch- and latency-bound, no roofline fraction",
           "launch": cfg, "runs_timed": reps}
    log(f"small graphene: {ms:.2f} ms per run ({1e3 * ms / (nt - 1):.1f} us per time step, wall {wall:.2f} ms)")
    if stash is not None:
        stash["small"] = {"lat": lat, "psi0": psi0_np, "dt": dt, "f": f, "corr": corr.cpu().numpy(),
                          "dos": D.cpu().numpy()}
    H.close()
    return out


def bench_hbm_resident(args, log, cfg64=None, cfg32=None, stash=None):
    """The FP32/batched-vs-FP64 comparison on a lattice whose vectors exceed
    the 256 MB Infinity Cache: disordered graphene 3072 x 3072 cells
    (18,874,368 orbitals, 302 MB per FP64 state vector), plain FP64 with one
    state, FP32-mixed with 8 states and FP64 with 8 states, each timed over
    the same number of time steps, against the byte model (B per row per
    pass per state: FP64 S=1 108, FP64 S=8 69.5, FP32 S=8 35.5)."""
    import torch

    from paper_2209_00806_amd import inputs, tbpm

    t0 = time.time()
    cells = args.hbm_cells
    lat, psi0_np = inputs.workload_disordered_graphene(cells, 8, seed_offset=5)
    H = tbpm.Hamiltonian.from_lattice(lat)
    f = 9.0
    dt = math.pi / f
    nt = args.hbm_nt
    M = tbpm.num_terms(f * dt, 1e-12)
    log(f"hbm-resident lattice built: N={lat.n_orb} in {time.time() - t0:.1f}s")
    psi8 = torch.from_numpy(psi0_np).cuda()
    psi1 = psi8[:, :1].contiguous()
    stream = torch.cuda.current_stream()
    out = {"workload": f"disordered graphene {cells}x{cells} cells ({lat.n_orb} orbitals, Anderson W=1 eV), "
                       f"{nt} correlation samples, f=9 eV",
           "fp64_vector_MB": round(16 * lat.n_orb / 1e6, 1)}
    corrs = {}
    for name, psi, prec, cfg in (("fp64_s1", psi1, "fp64", cfg64), ("fp32_s8", psi8, "fp32", cfg32),
                                 ("fp64_s8", psi8, "fp64", cfg64)):
        S = psi.shape[1]
        if cfg:
            c = dict(cfg)
            if S == 1:
                c["vec"] = 1
            H.set_launch_config(precision=prec, **c)
        tbpm.propagate(H, psi, 4, dt, f, precision=prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        corr = tbpm.propagate(H, psi, nt, dt, f, precision=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        b, v = (8, 4) if prec == "fp32" else (16, 8)
        upd = nnz_updates(lat.n_orb, lat.nnz, S, M, nt)
        out[name] = {"ms": round(ms, 1), "nnz_updates_per_s": upd / (ms / 1e3),
                     "alg_GBps": round(step_bytes(M, lat.n_orb, lat.nnz, S, b, v) * (nt - 1) / (ms / 1e3) / 1e9, 1),
                     "launch": H.launch_config(prec)}
        corrs[name] = corr[:, 0].cpu().numpy()
        log(f"hbm-resident {name}: {ms:.1f} ms, {upd / (ms / 1e3):.3e} nnz-updates/s")
    r1 = out["fp64_s1"]["nnz_updates_per_s"]
    out["fp32_s8_speedup_vs_fp64_s1"] = round(out["fp32_s8"]["nnz_updates_per_s"] / r1, 3)
    out["fp32_s8_speedup_model"] = round(108.0 / 35.5, 2)
    out["fp64_s8_speedup_vs_fp64_s1"] = round(out["fp64_s8"]["nnz_updates_per_s"] / r1, 3)
    out["fp64_s8_speedup_model"] = round(108.0 / 69.5, 2)
    if stash is not None:
        stash["hbm"] = {"lat": lat, "psi0": psi0_np[:, :1].copy(), "dt": dt, "f": f,
                        **{k: v[:TBG_PREFIX].copy() for k, v in corrs.items()}}
    H.close()
    del psi1, psi8
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(args, log, stash, extra, S, nt):
    """The oracle on the host: (1) the timed baseline, one state of the
    headline workload over a bounded prefix of steps; (2) from the same
    oracle, the error of every GPU result against it -- the headline's FP64
    and FP32-mixed runs over that prefix, the small graphene run at full
    length, and prefixes of the twisted bilayer, the batch members and the
    HBM-resident lattice.  Errors: max_k |dC_k| / max_k |C_k| over the
    prefix, and for FP32-mixed the L1-relative error of the prefix's DOS."""
    import numpy as np

    import oracle
    from paper_2209_00806_amd import tbpm

    def errs(gpu, ref, dt):
        gpu = np.asarray(gpu).reshape(-1)
        ref = np.asarray(ref).reshape(-1)
        n = min(gpu.shape[0], ref.shape[0])
        gpu, ref = gpu[:n], ref[:n]
        e = {"corr_max_rel_err": float(np.max(np.abs(gpu - ref)) / np.max(np.abs(ref)))}
        _, dg = oracle.dos(gpu.reshape(-1, 1), dt)
        _, dr = oracle.dos(ref.reshape(-1, 1), dt)
        e["dos_l1_rel_err"] = float(np.sum(np.abs(dg - dr)) / np.sum(np.abs(dr)))
        e["samples"] = int(ref.shape[0])
        return e

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    hl = stash["headline"]
    lat, f, dt = hl["lat"], hl["f"], hl["dt"]
    n_pass = tbpm.num_terms(f * dt, 1e-12) - 1
    one_state = hl["psi0"]
    # calibrate: 2 correlation samples = 1 time step
    tc = time.perf_counter()
    oracle.propagate(lat.row_ptr, lat.col, lat.val, lat.onsite, one_state, 2, dt, f)
    t1 = time.perf_counter() - tc
    n_cpu = min(max(2, int(args.cpu_seconds / max(t1, 1e-3))), nt - 1)
    tc = time.perf_counter()
    ref, _, _ = oracle.propagate(lat.row_ptr, lat.col, lat.val, lat.onsite, one_state, n_cpu + 1, dt, f)
    tcpu = time.perf_counter() - tc
    cpu_updates = (lat.nnz + lat.n_orb) * 1 * n_pass * n_cpu
    cpu = {"value": cpu_updates / tcpu, "unit": "nnz-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"1 of {S} states, {n_cpu} of {nt - 1} time steps of the same workload "
                     f"({tcpu:.1f} s on the host)", "cpu_model": cpu_model()}
    log(f"cpu oracle: {cpu['value']:.3e} nnz-updates/s on {threads} threads ({tcpu:.1f}s)")
    par = {}
    n = ref.shape[0]
    par["headline_fp64"] = errs(hl["fp64"][:n], ref[:, 0], dt)
    if "fp32" in hl:
        par["headline_fp32_mixed"] = errs(hl["fp32"][:n], ref[:, 0], dt)
        extra["fp32_mixed"]["vs_fp64_oracle"] = par["headline_fp32_mixed"]
    sm = stash.get("small")
    if sm:
        l = sm["lat"]
        r, _, _ = oracle.propagate(l.row_ptr, l.col, l.val, l.onsite, sm["psi0"], sm["corr"].shape[0], sm["dt"],
                                   sm["f"])
        _, dr = oracle.dos(r, sm["dt"])
        par["small_graphene_fp64"] = {"corr_max_rel_err": float(np.max(np.abs(sm["corr"] - r)) / np.max(np.abs(r))),
                                      "dos_max_rel_err": float(np.max(np.abs(sm["dos"] - dr)) / np.max(np.abs(dr))),
                                      "samples": int(r.shape[0])}
        extra["small_graphene"]["vs_fp64_oracle"] = par["small_graphene_fp64"]
    tb = stash.get("tbg")
    if tb:
        l = tb["lat"]
        r, _, _ = oracle.propagate(l.row_ptr, l.col, l.val, l.onsite, tb["psi0"], TBG_PREFIX, tb["dt"], tb["f"])
        for prec in ("fp64", "fp32"):
            par[f"twisted_bilayer_{prec}"] = errs(tb[prec], r[:, 0], tb["dt"])
            extra["twisted_bilayer"][prec]["vs_fp64_oracle"] = par[f"twisted_bilayer_{prec}"]
    bt = stash.get("batch")
    if bt:
        for prec in ("fp64", "fp32"):
            worst = None
            for m in bt:
                l = m["lat"]
                r, _, _ = oracle.propagate(l.row_ptr, l.col, l.val, l.onsite, m["psi0"], ORACLE_PREFIX, m["dt"], m["f"])
                e = errs(m[prec], r[:, 0], m["dt"])
                if worst is None or e["corr_max_rel_err"] > worst["corr_max_rel_err"]:
                    worst = dict(e, member=m["member"])
            par[f"batch_{prec}_worst_of_3_members"] = worst
            extra["batched"][prec]["vs_fp64_oracle_worst_of_3_members"] = worst
    hb = stash.get("hbm")
    if hb:
        l = hb["lat"]
        r, _, _ = oracle.propagate(l.row_ptr, l.col, l.val, l.onsite, hb["psi0"], TBG_PREFIX, hb["dt"], hb["f"])
        for k in ("fp64_s1", "fp32_s8", "fp64_s8"):
            par[f"hbm_resident_{k}"] = errs(hb[k], r[:, 0], hb["dt"])
            extra["hbm_resident"][k]["vs_fp64_oracle"] = par[f"hbm_resident_{k}"]
    log("oracle parity: " + ", ".join(f"{k} {v['corr_max_rel_err']:.1e}" for k, v in par.items()))
    return cpu, par


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=1024)
    ap.add_argument("--states", type=int, default=8)
    ap.add_argument("--nt", type=int, default=2048, help="correlation samples per step (2048 = the workload)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-cache", default=None, help="JSON file that stores/reuses autotuned launch shapes")
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the copy-bandwidth calibration")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--batch-members", type=int, default=64)
    ap.add_argument("--batch-nt", type=int, default=1024)
    ap.add_argument("--bwd-cells", type=int, default=512)
    ap.add_argument("--bwd-nt", type=int, default=1024)
    ap.add_argument("--no-tbg", action="store_true")
    ap.add_argument("--no-ldos", action="store_true", help="skip the LDOS, snapshot, quasi-eigenstate, optical-conductivity, Haydock and Kubo-Bastin legs")
    ap.add_argument("--ldos-nt", type=int, default=512)
    ap.add_argument("--ac-nt", type=int, default=256, help="time steps of the optical-conductivity leg")
    ap.add_argument("--hay-iter", type=int, default=1000, help="iterations of the Haydock leg")
    ap.add_argument("--kpm-moments", type=int, default=512, help="moments of the Kubo-Bastin leg")
    ap.add_argument("--tbg-cells", type=int, default=1024)
    ap.add_argument("--tbg-nt", type=int, default=1024)
    ap.add_argument("--small-cells", type=int, default=64, help="cells per side of the small graphene leg")
    ap.add_argument("--small-nt", type=int, default=512)
    ap.add_argument("--small-reps", type=int, default=20)
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--hbm-cells", type=int, default=3072, help="cells per side of the HBM-resident leg")
    ap.add_argument("--hbm-nt", type=int, default=64)
    ap.add_argument("--no-hbm", action="store_true")
    ap.add_argument("--only", choices=["small", "hbm", "backward", "next", "tbg", "batched"], default=None,
                    help="run one leg alone and print its record (for profiling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2209_00806_amd import inputs, tbpm

    if args.only == "small":
        print(json.dumps({"small_graphene": bench_small(args, log)}), flush=True)
        return
    if args.only == "hbm":
        print(json.dumps({"hbm_resident": bench_hbm_resident(args, log)}), flush=True)
        return
    if args.only == "backward":
        print(json.dumps({"backward": bench_backward(args, log)}), flush=True)
        return
    if args.only == "batched":
        print(json.dumps({"batched": bench_batched(args, log)}), flush=True)
        return
    if args.only == "tbg":
        print(json.dumps({"twisted_bilayer": bench_tbg(args, log)}), flush=True)
        return
    if args.only == "next":
        # the next-rows legs on the headline's FP64 launch shape (autotuned on
        # the headline operator, or read from --tune-cache)
        cfg64 = None
        if not args.no_autotune:
            lat, _ = inputs.workload_disordered_graphene(args.cells, args.states)
            H = tbpm.Hamiltonian.from_lattice(lat)
            cfg64, _, _ = tbpm.autotune_cached(H, args.states, "fp64", args.tune_cache)
            H.close()
            del H, lat
            torch.cuda.empty_cache()
        print(json.dumps(bench_ldos_psi_t(args, log, cfg64)), flush=True)
        return
    dev = torch.device("cuda:0")
    f = 9.0
    dt = math.pi / f
    S = args.states
    nt = args.nt
    t0 = time.time()
    lat, psi0_np = inputs.workload_disordered_graphene(args.cells, S)
    log(f"workload built: N={lat.n_orb} nnz={lat.nnz} in {time.time() - t0:.1f}s")
    H = tbpm.Hamiltonian.from_lattice(lat)
    psi0 = torch.from_numpy(psi0_np).to(dev)
    stash = {"headline": {"lat": lat, "psi0": psi0_np[:, :1].copy(), "dt": dt, "f": f}}
    del psi0_np
    M = tbpm.num_terms(f * dt, 1e-12)
    n_pass = M - 1
    stream = torch.cuda.current_stream()

    # copy calibration: a plain streaming copy of known size (1 GiB read + 1 GiB written)
    n_copy = args.copy_mib * 1024 * 1024 // 8
    csrc = torch.ones(n_copy, dtype=torch.float64, device=dev)
    cdst = torch.empty_like(csrc)
    tbpm.stream_copy(csrc, cdst)
    ca = torch.cuda.Event(enable_timing=True)
    cb = torch.cuda.Event(enable_timing=True)
    ca.record(stream)
    for _ in range(10):
        tbpm.stream_copy(csrc, cdst)
    cb.record(stream)
    torch.cuda.synchronize()
    copy_ms = ca.elapsed_time(cb) / 10
    copy_gbs = 2 * n_copy * 8 / (copy_ms / 1e3) / 1e9
    del csrc, cdst
    torch.cuda.empty_cache()
    log(f"copy calibration: {copy_gbs:.0f} GB/s (read + write of {args.copy_mib} MiB)")

    tuned = {}
    if not args.no_autotune:
        for prec in ("fp64", "fp32"):
            log(f"autotuning {prec}")
            cfg, ms, hit = tbpm.autotune_cached(H, S, prec, args.tune_cache)
            tuned[prec] = {"config": cfg, "ms_per_step": round(ms, 4), "cached": hit}
            log(f"autotuned {prec}: {cfg} ({ms:.3f} ms per time step{', cached' if hit else ''})")

    def one_step(precision="fp64"):
        corr = tbpm.propagate(H, psi0, nt, dt, f, precision=precision)
        E, D = tbpm.dos(corr, dt)
        return corr, E, D

    for w in range(args.warmup):
        one_step()
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        corr64, E, D64 = one_step()
        log(f"step {k + 1}/{args.steps} done")
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_per_step = ev0.elapsed_time(ev1) / max(args.steps, 1)
    updates = nnz_updates(lat.n_orb, lat.nnz, S, n_pass + 1, nt)
    value = updates / (ms_per_step / 1e3)
    fused64 = H.launch_config("fp64").get("fused", 0) > 0
    run_bytes = step_bytes(M, lat.n_orb, lat.nnz, S, 16, 8) * (nt - 1)
    sched_bytes = schedule_bytes(M, fused64, lat.n_orb, lat.nnz, S, 16, 8) * (nt - 1)
    log(f"fp64: {ms_per_step:.1f} ms/step (wall {t_wall / max(args.steps, 1) * 1e3:.1f}), "
        f"{value:.3e} nnz-updates/s, {run_bytes / (ms_per_step / 1e3) / 1e9:.0f} GB/s algorithmic")

    # dominant kernel: the interior launch (a Clenshaw pass, or a fused pair of
    # orders), timed in isolation on the same stream
    n_launch = 200
    tbpm.bench_pass(H, S, "fp64", 10)
    ka = torch.cuda.Event(enable_timing=True)
    kb = torch.cuda.Event(enable_timing=True)
    ka.record(stream)
    tbpm.bench_pass(H, S, "fp64", n_launch)
    kb.record(stream)
    torch.cuda.synchronize()
    pass_ms = ka.elapsed_time(kb) / n_launch
    # algorithmic bytes per launch = the per-pass figure B_pass x the passes one
    # launch performs (2 for a fused pair); the pair must move at least
    # pair_bytes, and the counters say what it moved
    units = 2 if fused64 else 1
    alg = units * pass_bytes(lat.n_orb, lat.nnz, S, 16, 8)
    if fused64:
        tfile, tsrc = PAIR_TRAFFIC_FILE, PAIR_SOURCES
        kname = "k_pair<double,real,MID> (two interior Clenshaw orders per launch)"
    else:
        tfile, tsrc = TRAFFIC_FILE, KERNEL_SOURCES
        kname = "k_pass<double,real,MID> (interior Clenshaw pass)"
    achieved = alg / (pass_ms / 1e3) / 1e9
    traffic = None
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tr = json.load(fh)
        if tr.get("kernel_hash") == kernel_hash(tsrc):
            traffic = tr.get("bytes_per_launch")
    min_bytes = pair_bytes(lat.n_orb, lat.nnz, S, 16, 8) if fused64 else alg
    drawn = max(traffic or 0, min_bytes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "achieved_is": "algorithmic bytes of the Clenshaw passes one launch performs (B_pass per pass, "
                               "2 for a fused pair) over the launch time: the unfused-equivalent rate",
                "hbm_frac_drawn": round(drawn / (pass_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "hbm_frac_drawn_is": "max(counted traffic, the bytes the launch must move) over the launch time "
                                     "/ peak: the rate actually drawn from HBM",
                "kernel": kname, "passes_per_launch": units,
                "kernel_avg_ms": round(pass_ms, 5), "algorithmic_bytes_per_launch": alg,
                "min_bytes_per_launch": min_bytes,
                "hbm_GBps_from_traffic": round(traffic / (pass_ms / 1e3) / 1e9, 1) if traffic else None,
                "copy_GBps": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}
    log(f"interior launch ({units} pass{'es' if units > 1 else ''}): {pass_ms * 1e3:.1f} us, {achieved:.0f} GB/s "
        f"algorithmic ({achieved / HBM_PEAK_GBS:.1%} of peak)")

    extra = {}
    c64 = corr64.cpu().numpy()
    d64 = D64.cpu().numpy()
    stash["headline"]["fp64"] = c64[:, 0].copy()
    # plain FP64 with a single state (the per-GPU share of an 8-way state split)
    psi1 = psi0[:, :1].contiguous()
    nt1 = min(nt, 256)
    tbpm.propagate(H, psi1, nt1, dt, f)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    tbpm.propagate(H, psi1, nt1, dt, f)
    e1.record(stream)
    torch.cuda.synchronize()
    ms1 = e0.elapsed_time(e1)
    rate_s1 = (lat.nnz + lat.n_orb) * n_pass * (nt1 - 1) / (ms1 / 1e3)
    alg_s1 = step_bytes(M, lat.n_orb, lat.nnz, 1, 16, 8) * (nt1 - 1) / (ms1 / 1e3) / 1e9
    extra["fp64_single_state"] = {"nnz_updates_per_s": rate_s1, "n_steps_timed": nt1,
                                  "alg_GBps": round(alg_s1, 1), "cache_resident": alg_s1 > HBM_PEAK_GBS,
                                  "note": "33.5 MB state vectors: a pass's working set (~134 MB) fits the 256 MB "
                                          "Infinity Cache; the HBM-resident comparison is extra.hbm_resident"}
    log(f"fp64 S=1: {rate_s1:.3e} nnz-updates/s")
    del psi1
    if not args.no_fp32:
        one_step("fp32")  # warm-up of the FP32 graph
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        corr32, _, D32 = one_step("fp32")
        e1.record(stream)
        torch.cuda.synchronize()
        ms32 = e0.elapsed_time(e1)
        d32 = D32.cpu().numpy()
        stash["headline"]["fp32"] = corr32[:, 0].cpu().numpy()
        l1 = float(np.sum(np.abs(d32 - d64)) / np.sum(np.abs(d64)))
        cerr = float(np.max(np.abs(corr32.cpu().numpy().mean(1) - c64.mean(1))) / np.max(np.abs(c64.mean(1))))
        extra["fp32_mixed"] = {"ms_per_step": round(ms32, 2), "nnz_updates_per_s": updates / (ms32 / 1e3),
                               "speedup_vs_fp64": round(ms_per_step / ms32, 3),
                               "dos_l1_rel_err_vs_gpu_fp64": l1, "corr_max_rel_err_vs_gpu_fp64": cerr,
                               "alg_GBps": round(step_bytes(M, lat.n_orb, lat.nnz, S, 8, 4) * (nt - 1)
                                                 / (ms32 / 1e3) / 1e9, 1)}
        extra["fp32_mixed"]["speedup_vs_fp64_single_state"] = round(updates / (ms32 / 1e3) / rate_s1, 3)
        log(f"fp32-mixed: {ms32:.1f} ms/step, speedup {ms_per_step / ms32:.2f}x, DOS L1 err {l1:.2e}")
    launch_cfg = {"fp64": H.launch_config("fp64"), "fp32": H.launch_config("fp32"), "autotuned": bool(tuned)}
    row_order = "bisection" if H.row_order() == 1 else "caller"
    H.close()
    del H
    torch.cuda.empty_cache()
    if not args.no_small:
        extra["small_graphene"] = bench_small(args, log, stash)
    if not args.no_hbm:
        extra["hbm_resident"] = bench_hbm_resident(args, log, launch_cfg["fp64"] if tuned else None,
                                                   launch_cfg["fp32"] if tuned else None, stash)
    if not args.no_batched:
        extra["batched"] = bench_batched(args, log, stash)
    if not args.no_backward:
        extra["backward"] = bench_backward(args, log)
    if not args.no_tbg:
        extra["twisted_bilayer"] = bench_tbg(args, log, stash)
    if not args.no_ldos:
        extra.update(bench_ldos_psi_t(args, log, launch_cfg["fp64"] if tuned else None))

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        cpu, parity = cpu_baseline_leg(args, log, stash, extra, S, nt)

    rec = {
        "metric": "TBPM propagation nnz-updates/s + HBM GB/s vs peak; FP32/batched vs FP64",
        "value": value,
        "unit": "nnz-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"disordered graphene {args.cells}x{args.cells} cells "
                               f"({lat.n_orb} orbitals, Anderson W=1 eV), {S} random-phase states, "
                               f"{nt} correlation samples, f=9 eV, dt=pi/f, {M} Chebyshev terms, "
                               f"Hann DOS on {2 * nt} energies",
                   "n_orb": lat.n_orb, "nnz_offdiag": lat.nnz, "n_states": S, "n_steps": nt,
                   "chebyshev_terms": M, "launch": launch_cfg},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "alg_GBps_step": round(run_bytes / (ms_per_step / 1e3) / 1e9, 1),
        "schedule_min_GBps_step": round(sched_bytes / (ms_per_step / 1e3) / 1e9, 1),
        "row_order": row_order,
        "oracle_parity": parity,
        "extra": extra,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
