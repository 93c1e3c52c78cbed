#!/usr/bin/env python3
"""Benchmark of the principal-cell lattice hot path on one MI355X.

One step = one pass of every hot-path stage over the workload (inputs already in HBM):
  DOF maps -> residual + energy + snapshots + plain operators -> greedy selection + RB
  coefficients -> principal operators -> ROM apply (the measured kernel) -> plain per-cell apply
  -> reverse mode (ROM apply adjoint, coefficient adjoint, residual adjoint) -> orthonormal basis
  stack -> reduced-precision ROM apply (bf16 slice products, reported beside the FP64 number).
`value` is the ROM apply's throughput, GDOF/s = (active local DOFs x right-hand sides) / (apply
kernel time), with the kernel timed by HIP events on the stream it runs on.

Workload: 32 x 32 cells of 32^2 Q1 quads with hole radius graded 0.20 -> 0.35 along x,
neo-Hookean mu = 1, lam = 10, 10% compression + seeded perturbation, 16 right-hand sides,
at most 32 principal cells (tolerance 1e-8).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD_INDEX = 1
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TF = 78.6
LOWP_REFINE = 2.0 ** -16       # bf16 slice products up to level 1 (two levels)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_apply2d_rw_hole2d_32x32_hbm_traffic.md")


def measured_traffic(workload):
    """HBM bytes per ROM-apply launch from the committed counter summary, or None when that
    summary was taken on another workload or on a different apply source than the one built."""
    if workload != "hole2d_32x32_n32_graded" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
    sha = re.search(r"apply source sha256: ([0-9a-f]{64})", text)
    val = re.search(r"rom_apply traffic bytes per launch: (\d+)", text)
    if not sha or not val or apply_source_sha() != sha.group(1):
        return None
    return int(val.group(1))


def apply_source_sha():
    """sha256 of the apply kernels' source and the internal header they include: any change to
    the code the counters were taken on makes the recorded traffic stale."""
    h = hashlib.sha256()
    for f in ("lat_apply.hip", "lat_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2603_10741_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Sets the OpenMP thread count of the oracle's runtime (libgomp) for the calls that follow."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


def _oracle_rate(fn, dofs_rhs, budget_s):
    reps, t0 = 0, time.perf_counter()
    while True:
        fn()
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return dofs_rhs * reps / el / 1e9, reps, el


def cpu_baseline(cfg, keep, mu, lam, u_bg, X, budget_s=12.0):
    """The FP64 oracle's ROM apply on the host cores, repeated for about `budget_s` seconds."""
    import numpy as np
    import oracle as O
    O.build(force=False)
    l2g, nact, g2bg = O.dofmap(cfg.dim, cfg.ncell, cfg.nel, keep)
    uloc = O.gather_local(u_bg[g2bg], l2g)
    T = O.cells_eval(cfg.dim, cfg.nel, keep, uloc, mu, lam, want_f=False, want_energy=False)["T"]
    g = O.greedy(T, cfg.tol, cfg.cap, keep_Z=False)
    Kp = np.ascontiguousarray(T[g["S"][:g["n_r"]]])
    del T
    dofs = int(nact.sum()) * cfg.dim * X.shape[-1]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    _omp_threads(threads)
    rate, reps, el = _oracle_rate(lambda: O.combo_apply(cfg.dim, cfg.nel, Kp, g["alpha"], l2g, X), dofs, budget_s)
    _omp_threads(1)
    rate1, reps1, el1 = _oracle_rate(lambda: O.combo_apply(cfg.dim, cfg.nel, Kp, g["alpha"], l2g, X), dofs,
                                     budget_s / 3)
    _omp_threads(threads)
    return {"value": rate, "unit": "GDOF/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "single_thread_value": rate1,
            "sample": f"full workload ({cfg.n_cells} cells, m={X.shape[-1]}), oracle ROM apply repeated "
                      f"{reps}x in {el:.1f} s on {threads} threads; {reps1}x in {el1:.1f} s on one thread"}, \
        {"S": g["S"], "n_r": g["n_r"]}



def adjoint_roof(nbytes, nflops, t):
    """Roofline of the adjoint stage against the nearer of its two roofs: HBM for its algorithmic
    bytes, the FP64 matrix cores for its dense contractions; the other fraction rides along."""
    f_hbm = nbytes / t / 1e9 / HBM_PEAK_GBS
    f_mfma = nflops / t / 1e12 / FP64_MFMA_PEAK_TF
    if f_mfma > f_hbm:
        return {"bound": "mfma", "achieved": round(nflops / t / 1e12, 2), "peak": FP64_MFMA_PEAK_TF, "unit": "TFLOP/s",
                "frac": round(f_mfma, 4), "algorithmic_flops": int(nflops), "hbm_frac": round(f_hbm, 4),
                "algorithmic_bytes": int(nbytes)}
    return {"bound": "hbm", "achieved": round(nbytes / t / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(f_hbm, 4), "algorithmic_bytes": int(nbytes), "mfma_frac": round(f_mfma, 4),
            "algorithmic_flops": int(nflops)}

def apply_stage(index, m=16, reps=10, cpu_budget=4.0, sample_n=12, seed=7):
    """Apply-stage record of one workload (outside the timed steps of the main line): after
    snapshots, greedy and principal tangents, the ROM apply in FP64 and with bf16 slices (two
    starting levels, FP64-measured refinement), the plain per-cell apply and the ROM apply's adjoint
    (Xbar, alpha_bar and the Lame parts), each timed with HIP events on its stream (mean of `reps`
    after two untimed calls); errors against the FP64 oracle on sampled cells; rooflines against
    the bound each form has; the oracle's ROM apply on a 4 x 4 x 4-cell slice as CPU baseline."""
    import numpy as np
    import torch

    import lattice as L
    import oracle as O
    from paper_2603_10741_amd import binding as B
    dev = torch.device("cuda:0")
    cfg = L.config(index)
    log("apply stage", cfg.name)
    keep = L.make_keep(cfg)
    mu, lam = L.make_material(cfg)
    u_bg = L.make_displacement(cfg)
    P = B.Plan(cfg.dim, cfg.ncell, cfg.nel, keep, cap=cfg.cap)
    _, nact, g2bg, _ = P.dofmap()
    lane_nodes = int(nact.sum().item())
    dofs_rhs = lane_nodes * cfg.dim * m
    ug = torch.from_numpy(u_bg).to(dev)[g2bg].contiguous()
    mu_t, lam_t = torch.from_numpy(mu).to(dev), torch.from_numpy(lam).to(dev)
    P.reset_status()
    r = P.residual_tangent(ug, mu_t, lam_t, f=True, energy=True, snap=True, plain=True)
    g = P.select_principal(r["snap"], cfg.tol, keep_Z=True)
    code, _ = P.check_status(allow_cap=True)
    n_r = int(g["n_r"].item())
    r_snap = r.pop("snap")
    ops = P.principal_ops(ug, mu_t, lam_t, g["S"], n_r, parts=True)
    bs = P.basis_stack(g["Z"], g["nu"], g["beta"], n_r)
    del g["Z"]
    torch.cuda.empty_cache()
    gen = torch.Generator(dev).manual_seed(seed)
    Xp = torch.randn(P.packed_size(m), dtype=torch.float64, device=dev, generator=gen)
    Ybp = torch.randn(P.packed_size(m), dtype=torch.float64, device=dev, generator=gen)
    Y64, Ylp, Ypl = (torch.empty_like(Xp) for _ in range(3))
    err_t = torch.zeros(1, dtype=torch.float64, device=dev)
    kw = dict(K_mu=ops["K_mu"], K_lam=ops["K_lam"], S=g["S"])
    calls = {
        "rom_f64": lambda: P.apply_combo(ops["K"], n_r, g["alpha"], Xp, m, out=Y64),
        "rom_bf16": lambda: P.apply_combo(bs["stack"], n_r, bs["coef"], Xp, m, prec=B.BF16, refine_tol=LOWP_REFINE,
                                          out=Ylp, err_est=err_t),
        "plain_f64": lambda: P.apply_plain(r["plain"], Xp, m, out=Ypl),
        "adjoint_f64": lambda: P.apply_combo_adjoint(ops["K"], n_r, g["alpha"], Xp, Ybp, m, **kw),
    }
    ms = {}
    s = torch.cuda.current_stream()
    for name, fn in calls.items():
        for _ in range(2):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(s)
            fn()
            b.record(s)
        torch.cuda.synchronize()
        ms[name] = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ad = calls["adjoint_f64"]()
    torch.cuda.synchronize()
    # residual + tangent (snapshots) and the residual alone, into the buffers of the first call
    # (the greedy is done with the snapshot matrix)
    r_out = {"snap": r_snap, "f": r["f"], "energy": r["energy"]}
    rt_calls = {"residual_tangent": lambda: P.residual_tangent(ug, mu_t, lam_t, f=True, energy=True, snap=True,
                                                               out=r_out),
                "residual_only": lambda: P.residual_tangent(ug, mu_t, lam_t, f=True, energy=True, snap=False,
                                                            out={"f": r["f"], "energy": r["energy"]})}
    for name, fn in rt_calls.items():
        fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for a_, b_ in ev:
            a_.record(s)
            fn()
            b_.record(s)
        torch.cuda.synchronize()
        ms[name] = float(np.mean([a_.elapsed_time(b_) for a_, b_ in ev]))
    P.check_status(allow_cap=True)
    del r_out, r_snap
    # oracle on sampled cells with the GPU's principal cells and coefficients
    O.build(force=False)
    l2g, _, g2bg_o = O.dofmap(cfg.dim, cfg.ncell, cfg.nel, keep)
    S = g["S"].cpu().numpy()[:n_r]
    rng = np.random.default_rng(seed)
    sample = np.unique(np.concatenate([rng.choice(cfg.n_cells, sample_n, replace=False), S[:2]]))
    cells = np.unique(np.concatenate([sample, S]))
    uloc = dict(zip(cells.tolist(), O.gather_local(u_bg[g2bg_o], l2g[cells])))
    Kp = np.stack([O.cell_eval(cfg.dim, cfg.nel, keep[c], uloc[c], mu[c], lam[c])["stencil"] for c in S])
    Ks = np.stack([O.cell_eval(cfg.dim, cfg.nel, keep[c], uloc[c], mu[c], lam[c])["stencil"] for c in sample])
    alpha = g["alpha"].cpu().numpy()
    idx = torch.from_numpy(sample).to(dev).long()

    def cells_of(packed):
        return P.unpack(packed, m)[idx].cpu().numpy()
    X, Yb = cells_of(Xp), cells_of(Ybp)
    Yo = O.combo_apply(cfg.dim, cfg.nel, Kp, alpha[sample], l2g[sample], X)
    Ypo = O.plain_apply(cfg.dim, cfg.nel, Ks, l2g[sample], X)
    Xbo = O.combo_apply(cfg.dim, cfg.nel, Kp, alpha[sample], l2g[sample], Yb, transpose=True)
    Go = O.combo_forms(cfg.dim, cfg.nel, Kp, P.cap, l2g[sample], X, Yb)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    err = {"rom_f64": rel(cells_of(Y64), Yo), "rom_bf16": rel(cells_of(Ylp), Yo), "plain_f64": rel(cells_of(Ypl), Ypo),
           "adjoint_f64_xbar": rel(cells_of(ad["Xbar"]), Xbo),
           "adjoint_f64_alpha_bar": rel(ad["alpha_bar"][idx].cpu().numpy(), Go)}
    rom_vs_plain = float(torch.linalg.norm(Y64 - Ypl) / torch.linalg.norm(Ypl))
    # rooflines: the FP64 combination against the FP64 matrix cores (2 E (N_r + m) flops per active
    # lane-node: combine, then apply), the other forms against HBM (16 B per DOF and RHS, plus the
    # stack and alpha; the plain apply its cells' stencils; the adjoint a third vector)
    E = P.E
    flops = 2.0 * E * (n_r + m) * lane_nodes
    stack_b = 8.0 * P.nloc * E * n_r + 8.0 * P.ncells * n_r
    b_rom = 16.0 * dofs_rhs + stack_b
    b_plain = 16.0 * dofs_rhs + 8.0 * E * lane_nodes
    b_adj = 24.0 * dofs_rhs + 3 * stack_b
    # the adjoint's dense work: the transposed apply's combination and application, the products
    # W = X * Ybar summed over the right-hand sides (2 m flops per snapshot entry of a cell) and the
    # three stacks' contractions of W (2 N_r flops per entry each)
    adj_flops = flops + 2.0 * E * m * lane_nodes + 3 * 2.0 * E * n_r * lane_nodes
    t = {k: v * 1e-3 for k, v in ms.items()}
    gd = {k: round(dofs_rhs / t[k] / 1e9, 3) for k in calls}
    roof = {
        "rom_f64": {"bound": "mfma", "achieved": round(flops / t["rom_f64"] / 1e12, 2), "peak": FP64_MFMA_PEAK_TF,
                    "unit": "TFLOP/s", "frac": round(flops / t["rom_f64"] / 1e12 / FP64_MFMA_PEAK_TF, 4),
                    "algorithmic_flops": int(flops)},
        "rom_bf16": {"bound": "hbm", "achieved": round(b_rom / t["rom_bf16"] / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(b_rom / t["rom_bf16"] / 1e9 / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes": int(b_rom)},
        "plain_f64": {"bound": "hbm", "achieved": round(b_plain / t["plain_f64"] / 1e9, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(b_plain / t["plain_f64"] / 1e9 / HBM_PEAK_GBS, 4),
                      "algorithmic_bytes": int(b_plain)},
        "adjoint_f64": adjoint_roof(b_adj, adj_flops, t["adjoint_f64"]),
        # the snapshot matrix written once (8 B per stencil entry per cell) is the tangent's floor
        "residual_tangent": {"bound": "hbm", "achieved": round(8.0 * P.nsnap * P.ncells / t["residual_tangent"] / 1e9, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(8.0 * P.nsnap * P.ncells / t["residual_tangent"] / 1e9 / HBM_PEAK_GBS, 4),
                             "algorithmic_bytes": int(8.0 * P.nsnap * P.ncells)},
    }
    # the oracle's ROM apply on the low 4 x 4 x 4 corner of the lattice, with the same S and alpha
    sub = cfg.with_sub(tuple(min(4, c) for c in cfg.ncell))
    sl_ids = np.array([c for c in range(cfg.n_cells)
                       if all((c // int(np.prod(cfg.ncell[:ax]))) % cfg.ncell[ax] < sub.ncell_eff[ax]
                              for ax in range(cfg.dim))])
    Xs = np.random.default_rng(seed).standard_normal((len(sl_ids), P.nloc, cfg.dim, m))
    sl_dofs = int((l2g[sl_ids] >= 0).sum()) * cfg.dim * m
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    fn = lambda: O.combo_apply(cfg.dim, cfg.nel, Kp, alpha[sl_ids], l2g[sl_ids], Xs)
    _omp_threads(threads)
    rate, reps_c, el = _oracle_rate(fn, sl_dofs, cpu_budget)
    # one thread on the first 8 cells of the corner
    s8 = sl_ids[:8]
    fn1 = lambda: O.combo_apply(cfg.dim, cfg.nel, Kp, alpha[s8], l2g[s8], Xs[:8])
    _omp_threads(1)
    rate1, reps1, el1 = _oracle_rate(fn1, int((l2g[s8] >= 0).sum()) * cfg.dim * m, cpu_budget / 2)
    _omp_threads(threads)
    out = {
        "workload": cfg.name, "cells": P.ncells, "elements_per_cell": f"{cfg.nel}^{cfg.dim}", "right_hand_sides": m,
        "principal_cap": cfg.cap, "tol": cfg.tol, "n_r": n_r, "capped": code == B.LAT_W_CAP,
        "active_local_dofs": lane_nodes * cfg.dim, "inputs": "snapshots at the seeded displacement; X, Ybar i.i.d. "
        "N(0,1) drawn on the device",
        "ms": {k: round(v, 4) for k, v in ms.items()}, "gdofs": gd,
        "rom_f64_over_plain": round(t["plain_f64"] / t["rom_f64"], 3),
        "rom_bf16_over_plain": round(t["plain_f64"] / t["rom_bf16"], 3),
        "bf16": {"refine_tol": LOWP_REFINE, "err_est": float(err_t.item())},
        "rel_err_vs_fp64_oracle": err, "rom_vs_plain_operator_rel_diff": rom_vs_plain,
        "oracle_sample_cells": len(sample), "roofline": roof,
        "cpu_baseline": {"value": rate, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
                         "cpu_model": cpu_model(), "single_thread_value": rate1,
                         "sample": f"oracle ROM apply on the {'x'.join(map(str, sub.ncell_eff))}-cell corner "
                                   f"({len(sl_ids)} cells, m={m}) of the lattice: {reps_c}x in {el:.1f} s on "
                                   f"{threads} threads; its first 8 cells {reps1}x in {el1:.1f} s on one thread"},
    }
    del P, r, g, ops, bs, Xp, Ybp, Y64, Ylp, Ypl, ad
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--workload", type=int, default=WORKLOAD_INDEX,
                    help="workload index (default: the 32x32 graded-hole lattice; the others are parity cases)")
    ap.add_argument("--no-3d", action="store_true", help="skip the apply-stage records of the 3D lattices")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run one plain device copy of this size (for counter calibration)")
    ap.add_argument("--newton", action="store_true",
                    help="time one load-stepped Newton-Raphson solve instead of the hot-path step")
    ap.add_argument("--strain", type=float, default=0.04, help="--newton: total compression")
    ap.add_argument("--shear", type=float, default=0.01, help="--newton: total shear of the top face")
    ap.add_argument("--n-inc", type=int, default=4, help="--newton: load increments")
    ap.add_argument("--rb-tol", type=float, default=3e-4, help="--newton: greedy tolerance")
    ap.add_argument("--cap", type=int, default=64, help="--newton: principal-cell cap")
    ap.add_argument("--max-newton", type=int, default=30, help="--newton: iterations per increment")
    ap.add_argument("--solve-tol", type=float, default=1e-8, help="--newton: tangent-solve tolerance")
    ap.add_argument("--solve-maxit", type=int, default=200000, help="--newton: tangent-solve iteration limit")
    ap.add_argument("--snap-rule", choices=["full", "reduced", "material", "sampled"], default="full",
                    help="--newton: snapshot data")
    ap.add_argument("--radius", type=float, default=None, help="--newton: one hole radius for every cell")
    ap.add_argument("--matvec", choices=["stencils", "rom"], default="stencils",
                    help="--newton: ROM tangent products from stencils formed once per iteration, or ROM applies")
    ap.add_argument("--precond", choices=["two-level", "diag", "feti"], default="two-level",
                    help="--newton: tangent solve (MINRES two-level / diagonal, or the inexact FETI-DP solve)")
    ap.add_argument("--feti", action="store_true",
                    help="time one FETI-DP tangent solve against MINRES (two levels) on the ROM tangent at the "
                         "affine state of half the --strain load, or after --feti-newton-steps Newton steps")
    ap.add_argument("--feti-newton-steps", type=int, default=0, help="--feti: Newton steps (MINRES) before the solve")
    ap.add_argument("--feti-inner", type=int, default=32, help="--feti: interface PCG steps (the cap with --feti-inner-tol)")
    ap.add_argument("--feti-inner-tol", type=float, default=1e-2,
                    help="--feti: relative reduction at which the interface PCG stops early (0: fixed steps)")
    ap.add_argument("--feti-enrich", type=int, default=0, help="--feti: enrichment level to start from")
    ap.add_argument("--feti-f32", action="store_true", help="--feti: FP32 local-solve blocks in the preconditioner")
    ap.add_argument("--feti-max-enrich", type=int, default=3, help="--feti: highest enrichment level")
    ap.add_argument("--feti-n-delta", type=int, default=0,
                    help="--newton --precond feti: principal cells the local models choose from (0 = all)")
    ap.add_argument("--tangent", choices=["rom", "full"], default="rom",
                    help="--newton: ROM tangent, or every cell's own tangent (the standard method)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.newton:
        newton_main(args)
        return
    if args.feti:
        feti_main(args)
        return

    import numpy as np
    import torch

    import lattice as L
    from paper_2603_10741_amd import binding as B
    from paper_2603_10741_amd.autograd import build_rom_state  # noqa: F401  (same pipeline, not timed here)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = L.config(args.workload)
    m = cfg.m
    log("workload", cfg.name)
    keep = L.make_keep(cfg)
    mu, lam = L.make_material(cfg)
    u_bg = L.make_displacement(cfg)
    X = L.make_rhs(cfg)
    Yb = L.make_rhs(cfg, stream=1)

    P = B.Plan(cfg.dim, cfg.ncell, cfg.nel, keep, cap=cfg.cap)
    l2g, nact, g2bg, perm = P.dofmap()
    active_dofs = int(nact.sum().item()) * cfg.dim
    ug = torch.from_numpy(u_bg).to(dev)[g2bg].contiguous()
    mu_t, lam_t = torch.from_numpy(mu).to(dev), torch.from_numpy(lam).to(dev)
    ones, zeros = torch.ones_like(mu_t), torch.zeros_like(mu_t)
    Xp = P.pack(torch.from_numpy(X).to(dev), m)
    Ybp = P.pack(torch.from_numpy(Yb).to(dev), m)
    rbar = torch.randn(P.nglobal, cfg.dim, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(5))
    w_cil = P.gather(rbar, cfg.dim)

    # persistent outputs (no allocation inside the timed steps)
    bufs = {
        "res": {"f": P._f64(P.nloc * P.dim * P.ld), "energy": P._f64(P.ncells), "snap": P._f64(P.nsnap * P.ld),
                "plain": P._f64(P.npacked * P.E * 64)},
        "snap_mu": {"snap": P._f64(P.nsnap * P.ld)},
        "snap_lam": {"snap": P._f64(P.nsnap * P.ld)},
        "ops": {k: P._f64(P.nloc * P.E * P.cap) for k in ("K", "K_mu", "K_lam")},
        "Y": P._f64(P.packed_size(m)), "Yp": P._f64(P.packed_size(m)), "Ylp": P._f64(P.packed_size(m)),
        "basis": {"stack": P._f64(P.nloc * P.E * P.cap), "coef": P._f64(P.ncells, P.cap)},
        "err": torch.zeros(1, dtype=torch.float64, device=dev),
    }
    greedy_out = {}
    stages = ["dofmap", "residual_tangent", "select_principal", "principal_ops", "rom_apply", "plain_apply",
              "adjoint", "basis_stack", "rom_apply_bf16"]
    ev = {s: [] for s in stages}
    state = {}

    def step(record):
        s = torch.cuda.current_stream()
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]  # stage i: marks[i]..marks[i+1]
        marks[0].record(s)
        P.dofmap()
        marks[1].record(s)
        P.residual_tangent(ug, mu_t, lam_t, f=True, energy=True, snap=True, plain=True, out=bufs["res"])
        P.residual_tangent(ug, ones, zeros, f=False, energy=False, snap=True, out=bufs["snap_mu"])
        P.residual_tangent(ug, zeros, ones, f=False, energy=False, snap=True, out=bufs["snap_lam"])
        marks[2].record(s)
        g = P.select_principal(bufs["res"]["snap"], cfg.tol, keep_Z=True, out=greedy_out or None)
        greedy_out.update(g)
        marks[3].record(s)
        if "n_r" not in state:
            state["n_r"] = int(g["n_r"].item())        # host copy of the count, read once
        n_r = state["n_r"]
        ops = P.principal_ops(ug, mu_t, lam_t, g["S"], n_r, parts=True, out=bufs["ops"])
        marks[4].record(s)
        P.apply_combo(ops["K"], n_r, g["alpha"], Xp, m, out=bufs["Y"])
        marks[5].record(s)
        P.apply_plain(bufs["res"]["plain"], Xp, m, out=bufs["Yp"])
        marks[6].record(s)
        ad = P.apply_combo_adjoint(ops["K"], n_r, g["alpha"], Xp, Ybp, m, K_mu=ops["K_mu"], K_lam=ops["K_lam"],
                                   S=g["S"])
        P.alpha_adjoint(bufs["res"]["snap"], g["Z"], g["R"], g["nu"], g["S"], n_r, g["alpha"], ad["alpha_bar"],
                        bufs["snap_mu"]["snap"], bufs["snap_lam"]["snap"], ad["mu_bar"], ad["lam_bar"])
        P.residual_adjoint(ug, mu_t, lam_t, w_cil)
        marks[7].record(s)
        # reduced-precision combo: orthonormal-basis form, bf16 slice products (2 levels)
        bs = P.basis_stack(g["Z"], g["nu"], g["beta"], n_r, out=bufs["basis"])
        marks[8].record(s)
        P.apply_combo(bs["stack"], n_r, bs["coef"], Xp, m, prec=B.BF16, refine_tol=LOWP_REFINE, out=bufs["Ylp"],
                      err_est=bufs["err"])
        marks[9].record(s)
        if record:
            for i, st in enumerate(stages):
                ev[st].append((marks[i], marks[i + 1]))

    P.reset_status()
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("warmup done; n_r =", state.get("n_r"))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    code, cell = P.check_status(allow_cap=True)
    ms_stage = {st: float(np.mean([a.elapsed_time(b) for a, b in ev[st]])) for st in stages}
    t_apply = ms_stage["rom_apply"] * 1e-3
    t_plain = ms_stage["plain_apply"] * 1e-3
    n_r = state["n_r"]
    dofs_rhs = active_dofs * m
    value = dofs_rhs / t_apply / 1e9
    alg_bytes = 16.0 * dofs_rhs + 8.0 * P.ncells * n_r + 8.0 * P.nloc * P.E * n_r
    achieved = alg_bytes / t_apply / 1e9
    traffic = measured_traffic(cfg.name)
    rom_roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": ("k_apply2d_rw<2,32,0,0>" if cfg.dim == 2 else "k_apply3d_mfma<NR,0,0>")
                + " (ROM apply; stage time includes the alpha interleave)", "traffic_unit": "bytes per launch",
                "algorithmic_bytes_per_launch": int(alg_bytes)}
    if cfg.dim == 3:
        # in 3D the FP64 combination (2 E (N_r + m) flops per active lane-node: combine, then apply;
        # 16 flop per byte, past the ridge) binds the apply to the FP64 matrix cores
        rom_flops = 2.0 * P.E * (n_r + m) * active_dofs / cfg.dim
        rom_roof.update(bound="mfma", achieved=round(rom_flops / t_apply / 1e12, 2), peak=FP64_MFMA_PEAK_TF,
                        unit="TFLOP/s", frac=round(rom_flops / t_apply / 1e12 / FP64_MFMA_PEAK_TF, 4),
                        algorithmic_flops_per_launch=int(rom_flops), hbm_frac=round(achieved / HBM_PEAK_GBS, 4))
    # the whole reverse-mode stage against the bytes the method has to move once: X and Ybar read
    # and Xbar written (24 B per active DOF and RHS), the three principal stacks and alpha, the
    # greedy's Delta and both snapshot parts (3 x 8 B per snapshot entry per cell) with Z, and the
    # residual adjoint's cotangent read and local result written
    t_adj = ms_stage["adjoint"] * 1e-3
    adj_bytes = (24.0 * dofs_rhs + 3 * 8.0 * P.nloc * P.E * n_r + 8.0 * P.ncells * n_r
                 + 3 * 8.0 * P.nsnap * P.ncells + 8.0 * n_r * P.nsnap + 2 * 8.0 * P.nloc * cfg.dim * P.ncells)
    # and its dense work over the active snapshot entries (E per active lane-node): the transposed
    # apply's combination and application, W = X * Ybar over the right-hand sides, the three stacks'
    # contractions of W and the coefficient adjoint's four row contractions (Z^T T^mu, Z^T T^lam,
    # Delta^T T^mu_S, Delta^T T^lam_S), 2 N_r flops per entry each
    adj_ent = P.E * active_dofs / cfg.dim
    adj_flops = 2.0 * adj_ent * (n_r + m) + 2.0 * adj_ent * m + 7 * 2.0 * adj_ent * n_r

    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mb} MiB read + {args.copy_probe_mb} MiB written")

    # accuracy of the ROM apply against the FP64 oracle, on a sample of cells, same S and alpha
    import oracle as O
    O.build(force=False)
    Y = P.unpack(bufs["Y"], m).cpu().numpy()
    Yp = P.unpack(bufs["Yp"], m).cpu().numpy()
    S = greedy_out["S"].cpu().numpy()[:n_r]
    alpha = greedy_out["alpha"].cpu().numpy()
    l2g_o, _, g2bg_o = O.dofmap(cfg.dim, cfg.ncell, cfg.nel, keep)
    uloc = O.gather_local(u_bg[g2bg_o], l2g_o)
    sample = np.unique(np.concatenate([np.arange(0, P.ncells, max(1, P.ncells // 24)), S]))
    Kp = np.stack([O.cell_eval(cfg.dim, cfg.nel, keep[s], uloc[s], mu[s], lam[s])["stencil"] for s in S])
    Yo = O.combo_apply(cfg.dim, cfg.nel, Kp, alpha[sample], l2g_o[sample], X[sample])
    err_rom = float(np.linalg.norm(Y[sample] - Yo) / np.linalg.norm(Yo))
    Kself = np.stack([O.cell_eval(cfg.dim, cfg.nel, keep[s], uloc[s], mu[s], lam[s])["stencil"] for s in sample])
    Ypo = O.plain_apply(cfg.dim, cfg.nel, Kself, l2g_o[sample], X[sample])
    err_plain = float(np.linalg.norm(Yp[sample] - Ypo) / np.linalg.norm(Ypo))
    Ylp = P.unpack(bufs["Ylp"], m).cpu().numpy()
    err_lp = float(np.linalg.norm(Ylp[sample] - Yo) / np.linalg.norm(Yo))
    t_lp = ms_stage["rom_apply_bf16"] * 1e-3
    lp_est = float(bufs["err"].item())
    rom_vs_plain = float(np.linalg.norm(Y - Yp) / np.linalg.norm(Yp))

    def snapshot_variant(rule, tol):
        """Snapshots with one quadrature rule, the greedy on them, then the ROM apply with the
        full-rule principal tangents: time of the snapshot pass and of the greedy, N_r, and the
        ROM operator's distance to every cell's own tangent (outside the timed steps)."""
        buf = {"snap": P._f64(P.nsnap * P.ld)}
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        cs = torch.cuda.current_stream()
        e[0].record(cs)
        P.residual_tangent(ug, mu_t, lam_t, snap_rule=rule, f=False, energy=False, snap=True, out=buf)
        e[1].record(cs)
        g = P.select_principal(buf["snap"], tol, keep_Z=False, rows=P.snapshot_rows(rule))
        e[2].record(cs)
        torch.cuda.synchronize()
        nr = int(g["n_r"].item())
        K = P.principal_ops(ug, mu_t, lam_t, g["S"], nr)["K"]
        Yv = P.unpack(P.apply_combo(K, nr, g["alpha"], Xp, m), m).cpu().numpy()
        ach = float(g["achieved"].item())
        return {"snap_ms": round(e[0].elapsed_time(e[1]), 4), "greedy_ms": round(e[1].elapsed_time(e[2]), 4),
                "n_r": nr, "capped": bool(ach > tol), "rom_vs_plain_rel": float(np.linalg.norm(Yv - Yp) /
                                                                                np.linalg.norm(Yp))}

    snap_variants = {f"{name}_tol_{tol:g}": snapshot_variant(rule, tol)
                     for tol in (1e-3, 1e-4) for name, rule in (("full", B.RULE_FULL), ("reduced", B.RULE_REDUCED),
                                                                ("material", B.RULE_MATERIAL),
                                                                ("sampled", B.RULE_SAMPLED))}
    P.reset_status()

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu, _ = cpu_baseline(cfg, keep, mu, lam, u_bg, X, budget_s=args.cpu_budget)

    configs = {}
    if not args.no_3d:
        del bufs, greedy_out, state
        torch.cuda.empty_cache()
        for idx in (2, 4):                  # BCC 10^3 (12^3 hexes), mixed BCC/octet 20^3 (16^3 hexes)
            rec = apply_stage(idx, cpu_budget=min(4.0, args.cpu_budget))
            configs[rec["workload"]] = rec
            log(f"apply stage {rec['workload']}: {rec['gdofs']}")

    out = {
        "metric": "GDOF/s of principal-combo apply vs plain per-cell apply at ≤1e-5 rel err",
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "cells": P.ncells, "elements_per_cell": f"{cfg.nel}^{cfg.dim}",
                   "right_hand_sides": m, "principal_cap": cfg.cap, "tol": cfg.tol, "n_r": n_r,
                   "active_local_dofs": active_dofs, "parallelism": "single GPU"},
        "roofline": rom_roof,
        "cpu_baseline": cpu,
        "adjoint_roofline": dict(adjoint_roof(adj_bytes, adj_flops, t_adj), ms=round(ms_stage["adjoint"], 4),
                                 stage="ROM apply adjoint (Xbar, alpha_bar, mu/lam through the principal "
                                       "tangents) + coefficient adjoint + residual adjoint"),
        "plain_apply_gdofs": round(dofs_rhs / t_plain / 1e9, 3),
        "rom_over_plain_speedup": round(t_plain / t_apply, 3),
        "reduced_precision": {"kernel": ("k_apply2d_rw" if cfg.dim == 2 else "k_apply3d_mfma")
                              + " (bf16 slice products on the matrix cores, FP64 level sums and apply; one node per workgroup formed "
                                "again in FP64 for the error estimate that decides further levels)",
                              "refine_tol": LOWP_REFINE, "starting_levels": 2,
                              "err_est": lp_est,
                              "gdofs": round(dofs_rhs / t_lp / 1e9, 3), "rel_err_vs_fp64_oracle": err_lp,
                              "over_fp64_plain_speedup": round(t_plain / t_lp, 3)},
        "rel_err_rom_apply_vs_fp64_oracle": err_rom,
        "rel_err_plain_apply_vs_fp64_oracle": err_plain,
        "rom_vs_plain_operator_rel_diff": rom_vs_plain,
        "stage_ms": {k: round(v, 4) for k, v in ms_stage.items()},
        "snapshot_variants": snap_variants,
        "device_status": {"code": code, "first_cell": cell},
        "configs": configs,
    }
    print(json.dumps(out))


def newton_cpu_baseline(cfg, case, args, budget_s=12.0):
    """The oracle's Newton iteration (snapshots + residual, greedy, sparse-LU tangent solve, one
    line-search evaluation) on the 8 x 8-cell corner of the lattice, repeated within the budget."""
    import numpy as np

    import lattice as L
    from oracle import newton as ON
    sub = tuple(min(8, c) for c in cfg.ncell)
    c2 = cfg.with_sub(sub)
    bvp = L.make_bvp(c2, case)
    mu, lam = L.make_material(c2)
    P = ON.Problem(c2.dim, c2.ncell_eff, c2.nel, L.make_keep(c2), mu, lam, bvp["fixed"], bvp["ubar"])
    u = P.ubar / case.n_inc
    lf = 1.0 / case.n_inc
    r, T, _, _ = P.evaluate(u, lf)
    n = 0
    t0 = time.perf_counter()
    while True:
        du, g = P.tangent_solve(u, T, -r, args.rb_tol, args.cap)
        r2, T2, _, _ = P.evaluate(u + du, lf)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 8:
            break
        u, r, T = u + du, r2, T2
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(el / n, 4), "unit": "s per Newton iteration", "cores": threads, "kind": "oracle",
            "sample": f"{n} Newton iteration(s) of the first increment on the {sub[0]} x {sub[1]}-cell corner of the "
                      f"workload ({P.ng * c2.dim} DOFs; the full lattice is {int(np.prod(cfg.ncell))} cells), "
                      f"SuperLU (one thread) tangent solve, element loops on the OpenMP threads"}


def feti_main(args):
    """One inexact FETI-DP solve (Sec. 3.3) of the ROM tangent system and the two-level MINRES solve of
    the same system, timed on the GPU; one JSON line with iterations, times, their agreement and the
    saddle-point residual."""
    import numpy as np
    import torch

    import lattice as L
    from paper_2603_10741_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = L.config(args.workload)
    case = L.LoadCase("compress_shear", args.strain, args.shear, 2)
    keep = L.make_keep(cfg)
    mu, lam = L.make_material(cfg)
    bvp = L.make_bvp(cfg, case)
    P = B.Plan(cfg.dim, cfg.ncell, cfg.nel, keep, cap=args.cap)
    _, nact, g2bg, _ = P.dofmap()
    g2bg = g2bg.cpu().numpy()
    fixed = torch.from_numpy(np.ascontiguousarray(bvp["fixed"][g2bg])).to(dev)
    ubar = torch.from_numpy(np.ascontiguousarray(bvp["ubar"][g2bg])).to(dev)
    mu_t, lam_t = torch.from_numpy(mu).to(dev), torch.from_numpy(lam).to(dev)
    if args.feti_newton_steps > 0:
        u = torch.zeros(P.nglobal, cfg.dim, dtype=torch.float64, device=dev)
        P.newton_solve(mu_t, lam_t, fixed, ubar, u, n_inc=2, max_newton=args.feti_newton_steps, cap=args.cap,
                       rb_tol=args.rb_tol, cg_tol=1e-8, cg_maxit=args.solve_maxit, cg_check=64, precond=1)
        state = f"after {args.feti_newton_steps} Newton step(s) of the first of 2 increments"
    else:
        u = (0.5 * ubar).contiguous()
        state = "affine, half the load"
    r = P.residual_tangent(u, mu_t, lam_t, f=False, energy=False, snap=True)
    g = P.select_principal(r["snap"], args.rb_tol, cap=args.cap)
    n_r = int(g["n_r"].item())
    K = P.principal_ops(u, mu_t, lam_t, g["S"], n_r)["K"]
    P.check_status(allow_cap=True)
    b = torch.from_numpy(np.random.default_rng(7).standard_normal((P.nglobal, cfg.dim))).to(dev)
    runs = []
    for _ in range(2):           # the second solve is the timed one (rocBLAS / rocSOLVER warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, info = P.feti_solve(K, n_r, g["alpha"], g["S"], fixed, b, R=g["R"], nu=g["nu"], beta=g["beta"],
                                   n_delta=args.feti_n_delta, inner_it=args.feti_inner, tol=args.solve_tol,
                                   inner_tol=args.feti_inner_tol,
                                   maxit=600, enrich=args.feti_enrich, prec=B.F32 if args.feti_f32 else B.F64,
                                   max_enrich=max(args.feti_max_enrich, args.feti_enrich))
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t0, x, st, info))
    wall, x, st, info = runs[-1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xm, stm, its, rr = P.rom_solve(K, n_r, g["alpha"], fixed, b, tol=args.solve_tol, maxit=args.solve_maxit, check=64)
    torch.cuda.synchronize()
    wall_m = time.perf_counter() - t0
    agree = (torch.linalg.norm(x - xm) / torch.linalg.norm(xm)).item()
    out = {
        "metric": "time of one tangent solve K~ x = b (inexact FETI-DP against two-level MINRES)",
        "value": round(wall, 4), "unit": "s", "higher_is_better": False, "n_gpus": 1, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "cells": P.ncells, "global_dofs": P.nglobal * cfg.dim,
                   "load": {"kind": case.kind, "strain": case.strain, "shear": case.shear}, "state": state,
                   "rb_tol": args.rb_tol, "n_r": n_r, "tol": args.solve_tol, "inner_it": args.feti_inner, "inner_tol": args.feti_inner_tol,
                   "enrich_start": args.feti_enrich, "local_blocks": "f32" if args.feti_f32 else "f64",
                   "n_delta": info["n_delta"], "rhs": "i.i.d. N(0,1)"},
        "feti": {"status": int(st), "iters": info["iters"], "restarts": info["restarts"], "enrich": info["enrich"],
                 "n_shift": info["n_shift"], "relres": info["relres"], "setup_ms": round(info["t_setup_ms"], 2),
                 "solve_ms": round(info["t_solve_ms"], 2),
                 "ms_per_iteration": round(info["t_solve_ms"] / max(info["iters"], 1), 3),
                 "primal_dofs": info["n_primal"], "multipliers": info["n_mult"], "remaining_rows": info["n_rdofs"],
                 "dual_rows": info["n_ddofs"]},
        "minres": {"status": int(stm), "iters": its, "relres_Minv": rr, "s": round(wall_m, 4)},
        "rel_diff_feti_vs_minres": agree,
    }
    print(json.dumps(out))


def newton_main(args):
    """One load-stepped Newton-Raphson solve (compression + shear of the top face, bottom face
    clamped) on the GPU; prints one JSON line with the time to solution and the per-iteration
    split into reduced-basis set-up, tangent solve and residual/snapshot evaluations."""
    import numpy as np
    import torch

    import lattice as L
    from paper_2603_10741_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = L.config(args.workload)
    if args.radius is not None:
        cfg = cfg.with_(radius=(args.radius, args.radius), name=cfg.name + f"_r{args.radius:g}")
    case = L.LoadCase("compress_shear", args.strain, args.shear, args.n_inc)
    log("newton workload", cfg.name, case)
    keep = L.make_keep(cfg)
    mu, lam = L.make_material(cfg)
    bvp = L.make_bvp(cfg, case)
    P = B.Plan(cfg.dim, cfg.ncell, cfg.nel, keep, cap=args.cap)
    _, nact, g2bg, _ = P.dofmap()
    g2bg = g2bg.cpu().numpy()
    fixed = torch.from_numpy(np.ascontiguousarray(bvp["fixed"][g2bg])).to(dev)
    ubar = torch.from_numpy(np.ascontiguousarray(bvp["ubar"][g2bg])).to(dev)
    mu_t, lam_t = torch.from_numpy(mu).to(dev), torch.from_numpy(lam).to(dev)
    u = torch.zeros(P.nglobal, cfg.dim, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, recs = P.newton_solve(mu_t, lam_t, fixed, ubar, u, n_inc=args.n_inc, max_newton=args.max_newton,
                              cap=args.cap, rb_tol=args.rb_tol, cg_tol=args.solve_tol, cg_maxit=args.solve_maxit,
                              cg_check=64, verbose=True, tangent=1 if args.tangent == "full" else 0,
                              snap_rule={"full": B.RULE_FULL, "reduced": B.RULE_REDUCED,
                                         "material": B.RULE_MATERIAL, "sampled": B.RULE_SAMPLED}[args.snap_rule],
                              matvec=1 if args.matvec == "rom" else 0,
                              precond={"diag": 0, "two-level": 1, "feti": 2}[args.precond],
                              feti_n_delta=args.feti_n_delta)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot = {k: float(sum(r[k] for r in recs)) for k in ("t_init_ms", "t_solve_ms", "t_eval_ms")}
    its = int(sum(r["cg_iters"] for r in recs))
    # the tangent solve's dominant kernel: the per-cell stencil apply with one right-hand side, timed
    # by the driver with HIP events around up to 64 products of every solve (on its stream)
    tp = [r["t_product_us"] for r in recs if r["t_product_us"] > 0]
    t_mv = float(np.mean(tp)) * 1e-6 if tp else float("nan")
    lane_nodes = int(nact.sum().item())
    rom_products = args.matvec == "rom" and args.tangent == "rom"
    if rom_products:
        # ROM apply forming the stencils on the matrix cores: 2 E N_r flops per packed lane-node
        # (combination) + 2 E per active lane-node (apply), against the FP64 matrix-core peak
        nr_avg = float(np.mean([r["n_r"] for r in recs])) if recs else 0.0
        mv_flops = 2.0 * P.E * nr_avg * P.npacked * 64 + 2.0 * P.E * lane_nodes
        mv_bytes = 16.0 * lane_nodes * cfg.dim + 8.0 * (P.nloc * P.E + P.ncells) * nr_avg
    else:
        # per-cell stencils (8 B x E per active lane-node) + X read + Y written
        mv_bytes = 8.0 * lane_nodes * P.E + 16.0 * lane_nodes * cfg.dim
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle Newton iterations on an 8 x 8-cell sample) ...")
        cpu = newton_cpu_baseline(cfg, case, args, budget_s=args.cpu_budget)
    out = {
        "metric": "time to solution of the load-stepped Newton-Raphson solve on the ROM tangent",
        "value": round(wall, 4),
        "unit": "s",
        "higher_is_better": False,
        "n_gpus": 1,
        "dtype": "f64",
        "data": "synthetic",
        "status": int(st),
        "config": {"workload": cfg.name, "cells": P.ncells, "global_dofs": P.nglobal * cfg.dim,
                   "load": {"kind": case.kind, "strain": case.strain, "shear": case.shear, "increments": case.n_inc},
                   "tangent": args.tangent, "snap_rule": args.snap_rule, "rb_tol": args.rb_tol, "cap": args.cap,
                   "newton_tol": 1e-6,
                   "armijo": [0.5, 1e-4],
                   "tangent_solve": ({"method": "inexact FETI-DP (FGMRES on the saddle-point system), MINRES "
                                                "two-level on a step it does not converge on",
                                      "n_delta": args.feti_n_delta, "products": args.matvec, "tol": args.solve_tol}
                                     if args.precond == "feti" else
                                     {"method": "MINRES", "preconditioner": args.precond, "products": args.matvec,
                                      "tol": args.solve_tol})},
        "roofline": ({"bound": "mfma", "achieved": round(mv_flops / t_mv / 1e12, 2), "peak": FP64_MFMA_PEAK_TF,
                      "unit": "TFLOP/s", "frac": round(mv_flops / t_mv / 1e12 / FP64_MFMA_PEAK_TF, 4),
                      "algorithmic_flops_per_launch": int(mv_flops)} if rom_products else
                     {"bound": "hbm", "achieved": round(mv_bytes / t_mv / 1e9, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(mv_bytes / t_mv / 1e9 / HBM_PEAK_GBS, 4)}) | {"traffic": None,
                     "kernel": ((("k_apply2d_rw<1,NR,0,0>" if cfg.dim == 2 else "k_apply3d_mfma<NR,0,0>")
                                 + " (ROM apply, one right-hand side, stencils formed on the matrix cores) in every "
                                 "MINRES iteration") if rom_products else
                                ("k_apply<2,1,8,2>" if cfg.dim == 2 else "k_apply<3,1,8,2>")
                                + " (per-cell stencil apply, one right-hand side) in every MINRES iteration"
                                + (" (standard method: the cells' own stencils)" if args.tangent == "full" else
                                   " (combined ROM stencils)")),
                     "algorithmic_bytes_per_launch": int(mv_bytes), "us_per_launch": round(t_mv * 1e6, 2)},
        "cpu_baseline": cpu,
        "newton_iterations": len(recs),
        "tangent_solve_iterations": its,
        "ms_per_tangent_solve_iteration": round(tot["t_solve_ms"] / max(its, 1), 5),
        "split_ms": {k[2:-3]: round(v, 2) for k, v in tot.items()},
        "iterations": [{"inc": r["increment"], "it": r["iteration"], "n_r": r["n_r"],
                        "rb_achieved": float("%.3g" % r["rb_achieved"]), "m": r["backtracks"],
                        "solve_its": r["cg_iters"], "solve_status": r["cg_status"], "solver": r["solver"],
                        "feti_its": r["feti_iters"], "feti_enrich": r["feti_enrich"],
                        "feti_setup_ms": round(r["t_feti_setup_ms"], 1),
                        "rel_res": float("%.3g" % (r["res_after"] / r["res0"])),
                        "ms": [round(r["t_init_ms"], 2), round(r["t_solve_ms"], 2), round(r["t_eval_ms"], 2)]}
                       for r in recs],
    }
    if not tp:
        out["roofline"] = None      # no MINRES product was timed (every step solved by FETI-DP)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
