"""Benchmark of the R-ChFSI filter path on one MI355X.

Workload: the paper-scale block -- periodic 20^3 cells of degree-6 elements
(1,728,000 DOFs, 8 Gauss points per direction), 128 PAW atoms x 18
projectors, 1024 states filtered in blocks of 256 with Chebyshev degree 30.

One step = one pass of the whole hot path: the residual-based Chebyshev
filter over all 1024 states (mixed precision: FP32 recurrence, FP64
residual correction) followed by the FP64 Rayleigh-Ritz and the residual
norms.  Reported value: seconds per SCF filter pass (mixed precision,
lower is better).  Also reported: the FP64 filter time per pass and the
ratio, the HX throughput, the eigenvalue error of the mixed filter against
the FP64 one after the FP64 Rayleigh-Ritz, the roofline of the dominant
kernel (the cell-local operator on the vector ALUs) and the oracle timed on
the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# FP32 vector peak: 256 CUs x 4 SIMDs x 64 lanes x 2 (FMA) x 2 (packed FP32) x 2.4 GHz
PEAK_VALU_F32_TFLOPS = 157.3
# the same without packed FP32 instructions (also the FP64 vector peak)
PEAK_VALU_F32_SCALAR_TFLOPS = 78.6
CELL_KERNEL_SRC = os.path.join(ROOT, "paper_2604_26037_amd", "csrc", "cell_valu.h")
# node part of the fused step per DOF-column: -ac x, -zz y, their sum, and
# the FP64 a lamY Y product-sum
STEP_NODE_FLOPS = 5
COUNTERS_FILE = os.path.join(ROOT, "profiles", "cell_step_f32_paper_counters.md")
METRIC = "ChFSI filter s/SCF pass & HX GFLOP/s, mixed vs FP64 at ≤1e-6 Ha eig err"


def local_flops_per_cell_col(np1, nq):
    """Sum-factorized cell operator K + V: 7 1-D contractions (kinetic) + 6 (V) + pointwise."""
    kin = 14 * np1 ** 4 + 2 * np1 ** 3
    pot = 4 * nq * np1 * (np1 * np1 + np1 * nq + nq * nq) + nq ** 3
    return kin + pot


def measured_traffic():
    """HBM bytes per launch of the cell kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    kernel source changed since the counters were taken."""
    import hashlib
    try:
        text = open(COUNTERS_FILE).read()
        src = hashlib.sha256(open(CELL_KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        line = line.strip().lstrip("-* ")
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip().strip("`")] = v.strip().strip("`")
    if fields.get("source_sha256") != src:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def gga_flops_per_cell_col(nq):
    """The GGA term on top of K + V: per quadrature line and axis, v u (nq
    products), two nq x nq collocation-derivative products and the final
    fma (4 nq^2 + 3 nq flops), over 3 nq^2 lines."""
    return 3 * nq * nq * (4 * nq * nq + 3 * nq)


def graded_gga_leg(s, N, B, m, dev):
    """The workload on a two-level mesh around the atoms with the GGA term:
    cell-kernel launches, apply_H and the mixed / FP64 filter passes."""
    import torch

    from paper_2604_26037_amd import FP32, FP64, Operator
    from workloads.configs import with_two_level_gga
    t0 = time.time()
    sg = with_two_level_gga(s, r_fine=1.0)
    op = Operator(sg)
    t_build = time.time() - t0
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(s.x_seed) % (2 ** 63) + 1)
    X = torch.randn((op.ndof, N), generator=gen, dtype=torch.float64, device=dev)
    tmin, tmax, beta = op.lanczos_bounds(k=20)
    bU = tmax + beta
    ws_f = op.workspace(max(op.cheb_filter_workspace(N, B, FP64), op.cheb_filter_workspace(N, B, FP32)))
    ws_r = op.workspace(op.rayleigh_ritz_workspace(N))
    lam, _ = op.rayleigh_ritz(X, ws=ws_r)
    lh = lam.cpu().numpy()
    out = {"workload": f"{s.name} on a two-level mesh (fine cells along the atoms, coarse cells twice as long) "
                       f"with a V_GGA field; operator built in {t_build:.1f} s",
           "cell_sizes": sorted(set(float(round(h, 9)) for b in sg.xgrid for h in np.diff(b)))}
    nloc = (local_flops_per_cell_col(s.degree + 1, s.nq) + gga_flops_per_cell_col(s.nq)) * op.ncells
    for name, prec, dt in (("fp64", FP64, torch.float64), ("fp32", FP32, torch.float32)):
        Xs = X[:, :B].to(dt).contiguous()
        Ys = torch.zeros_like(Xs)
        op.apply_local(Xs, Ys, 0, 1.0, prec)
        op.apply_H(Xs, out=Ys, prec=prec)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for _ in range(5):
            op.apply_local(Xs, Ys, 0, 1.0, prec)
        e[1].record()
        for _ in range(5):
            op.apply_H(Xs, out=Ys, prec=prec)
        e[2].record()
        torch.cuda.synchronize()
        t_loc = e[0].elapsed_time(e[1]) / 5 / 1e3
        out[name] = {"cell_launch_ms": t_loc / op.ncolour * 1e3, "apply_H_ms": e[1].elapsed_time(e[2]) / 5,
                     "local_tflops": nloc * B / t_loc / 1e12}
        del Xs, Ys
    for name, prec in (("mixed", FP32), ("fp64", FP64)):
        # warm-up: one whole pass (the first pass over freshly allocated
        # buffers runs about 10-20 % slower than the ones after it)
        Xc = X.clone()
        op.cheb_filter(Xc, lam, m, float(lh[0]), float(lh[-1]), bU, block=B, prec=prec, out=Xc, ws=ws_f)
        Xc.copy_(X)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        op.cheb_filter(Xc, lam, m, float(lh[0]), float(lh[-1]), bU, block=B, prec=prec, out=Xc, ws=ws_f)
        e1.record()
        torch.cuda.synchronize()
        out[f"filter_{name}_s_per_pass"] = e0.elapsed_time(e1) / 1e3
        del Xc
    out["speedup_mixed_vs_fp64"] = out["filter_fp64_s_per_pass"] / out["filter_mixed_s_per_pass"]
    out["flops_per_cell_col"] = int(local_flops_per_cell_col(s.degree + 1, s.nq) + gga_flops_per_cell_col(s.nq))
    log(f"two-level GGA: cell launch fp32 {out['fp32']['cell_launch_ms']:.3f} ms "
        f"({out['fp32']['local_tflops']:.1f} TFLOP/s), fp64 {out['fp64']['cell_launch_ms']:.3f} ms; "
        f"filter pass mixed {out['filter_mixed_s_per_pass']:.3f} s, FP64 {out['filter_fp64_s_per_pass']:.3f} s")
    op.close()
    return out


def nonlocal_flops_per_col(op_sys, supp_nodes_per_atom):
    npj = np.asarray(op_sys.nproj)
    return float(np.sum(4.0 * np.asarray(supp_nodes_per_atom) * npj + 2.0 * npj * npj))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    """Host cores, CPU model and the BLAS library NumPy calls (with its threads)."""
    import platform
    import threadpoolctl
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = [i for i in threadpoolctl.threadpool_info() if i.get("user_api") == "blas"]
    return {
        "os_cpu_count": os.cpu_count(),
        "cpu_model": model,
        "blas": ", ".join(f"{i.get('internal_api')} ({os.path.basename(i.get('filepath', ''))}, "
                          f"{i.get('num_threads')} threads)" for i in blas) or "none found",
        "blas_threads": max([int(i.get("num_threads", 1)) for i in blas] + [1]),
    }


def cpu_baseline(system, nstates, degree, ncols=64):
    """The oracle as it stands, on a bounded sample of the same workload:
    apply_H, apply_S and apply_Sinv on `ncols` columns, and Algorithm 2 with
    degree 2 on the same columns (initial residual, one Chebyshev step,
    finalize).  A filter pass is extrapolated as nstates/ncols such blocks,
    each the degree-2 filter plus (degree - 2) further steps of one H and one
    Sinv apply."""
    from oracle import chfsi
    from oracle.paw import PAWOperator
    info = host_info()
    t0 = time.time()
    ref = PAWOperator(system)
    t_build = time.time() - t0
    X = system.trial(ncols)
    tm = {}
    for name in ("H", "S", "Sinv"):
        t0 = time.perf_counter()
        getattr(ref, "apply_" + name)(X)
        tm[name] = time.perf_counter() - t0
    lam = np.linspace(-0.5, 0.5, ncols)
    t0 = time.perf_counter()
    chfsi.rchfsi_filter(ref, X, lam, 2, -1.0, 1.0, 300.0)
    tm["filter_m2"] = time.perf_counter() - t0
    step = tm["H"] + tm["Sinv"]
    per_pass = (nstates / ncols) * (tm["filter_m2"] + (degree - 2) * step)
    return {
        "value": per_pass, "unit": "s/pass (extrapolated)", "cores": int(info["blas_threads"]),
        "kind": "oracle",
        "sample": f"oracle on {ncols} of {nstates} columns of the same operator: apply_H {tm['H']:.2f} s, "
                  f"apply_S {tm['S']:.2f} s, apply_Sinv {tm['Sinv']:.2f} s, Algorithm 2 with degree 2 "
                  f"{tm['filter_m2']:.2f} s; pass = {nstates // ncols} blocks x (degree-2 filter + "
                  f"{degree - 2} x (H + Sinv)); oracle build {t_build:.1f} s not counted",
        "host": info,
    }


def time_step_kernel(op, X, B, prec, dt, reps):
    """Mean duration (s) of one colour launch of the filter's fused step
    kernel (pawfe_cheb_step_local) on a block of B columns, timed with events
    on the stream it is launched on (torch's current stream)."""
    import torch
    RY = X[:, :B].to(dt).contiguous()
    RX = torch.zeros_like(RY)
    Y = X[:, :B].contiguous()
    lamY = torch.linspace(-1.0, 2.0, B, dtype=torch.float64, device=X.device)
    # scalars of a degree-30 filter step (any values: the arithmetic does not depend on them)
    a, ac, zz = 0.011, 0.0425, 0.36
    op.cheb_step_local(RY, RX, Y, lamY, a, ac, zz, prec=prec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        op.cheb_step_local(RY, RX, Y, lamY, a, ac, zz, prec=prec)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps / op.ncolour
    del RY, RX, Y, lamY
    return t


def kernels_mode(op, s, gen, dev, args):
    """Short run for hardware counters: the cell-local operator and the
    filter's fused step kernel (FP32 and FP64) on one block, then a plain
    device copy of known size (counter calibration)."""
    import torch

    from paper_2604_26037_amd import BF16X3, FP32, FP64
    B = s.block
    X = torch.randn((op.ndof, B), generator=gen, dtype=torch.float64, device=dev)
    res = {}
    for name, prec, dt in (("fp32", FP32, torch.float32), ("fp64", FP64, torch.float64)):
        Xs = X.to(dt)
        Ys = torch.zeros_like(Xs)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        op.apply_local(Xs, Ys, 0, 1.0, prec)
        e0.record()
        for _ in range(args.hx_reps):
            op.apply_local(Xs, Ys, 0, 1.0, prec)
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / args.hx_reps / op.ncolour
        log(f"cell-local {name}: {res[name]:.3f} ms per colour launch")
        # the filter's fused step kernel on the same block
        res[name + "_step"] = time_step_kernel(op, X, B, prec, dt, args.hx_reps) * 1e3
        log(f"filter step (cell part) {name}: {res[name + '_step']:.3f} ms per colour launch")
        # the whole H and Sinv_hat applies (projector reductions included)
        for _ in range(2):
            op.apply_H(Xs, out=Ys, prec=prec)
            op.apply_Sinv(Xs, out=Ys, prec=prec)
        if prec == FP32:
            op.apply_H(Xs, out=Ys, prec=BF16X3)
        torch.cuda.synchronize()
        del Xs, Ys
    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"calibration copy: {nbytes} bytes read and written per launch, 3 launches")
    print(json.dumps({"mode": "kernels", "avg_launch_ms": res, "copy_bytes": nbytes}), flush=True)


def batch_mode(dev, args):
    """Uneven real problems (6^3-14^3 cells of degree 5, 8-64 atoms x 18
    projectors, 64-384 states, Chebyshev degree 25, FP32 recurrence) filtered
    as a graph-captured, autotuned multi-stream batch, against the same
    filters issued one after another on one stream.  (Not reachable while
    the full-size batch crash in pawfe_batch_create is open; main() exits
    before it.)"""
    import torch

    from paper_2604_26037_amd import FP32, Batch, Operator
    from workloads.configs import batch_systems
    t0 = time.time()
    systems = batch_systems(args.batch_count)
    jobs, ops = [], []
    gen = torch.Generator(device=dev)
    for i, s in enumerate(systems):
        op = Operator(s)
        gen.manual_seed(int(s.x_seed) % (2 ** 63))
        X = torch.randn((op.ndof, s.nstates), generator=gen, device=dev,
                        dtype=torch.complex128 if op.complex else torch.float64)
        lam, _ = op.rayleigh_ritz(X)
        tmin, tmax, beta = op.lanczos_bounds(k=20)
        lam_h = lam.cpu().numpy()
        jobs.append(dict(op=op, X=X, out=torch.empty_like(X), lam=lam, degree=25, b0=float(lam_h[0]),
                         bW=float(lam_h[-1]), bU=float(max(tmax + beta, lam_h[-1] + 1.0))))
        ops.append(op)
    ndof = [o.ndof for o in ops]
    log(f"{len(jobs)} problems built in {time.time() - t0:.1f} s: DOFs {min(ndof)}-{max(ndof)}, "
        f"states {min(s.nstates for s in systems)}-{max(s.nstates for s in systems)}, "
        f"{sum(o.complex for o in ops)} complex")
    t0 = time.time()
    b = Batch(jobs, prec=FP32)
    ns, blocks, sof = b.schedule()
    log(f"batch created (autotune + capture) in {time.time() - t0:.1f} s: {ns} streams, {b.ngraphs} graphs, "
        f"blocks {sorted(set(blocks.tolist()))}")
    reps = max(1, args.steps)
    b.run()
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(reps):
        b.run()
    e1.record()
    for _ in range(reps):
        for j, blk in zip(jobs, blocks):
            j["op"].cheb_filter(j["X"], j["lam"], j["degree"], j["b0"], j["bW"], j["bU"], block=int(blk),
                                prec=FP32, out=j["out"], ws=j.setdefault("ws", j["op"].workspace(
                                    j["op"].cheb_filter_workspace(j["X"].shape[1], int(blk), FP32))))
    e2.record()
    torch.cuda.synchronize()
    t_graph = e0.elapsed_time(e1) / reps / 1e3
    t_eager = e1.elapsed_time(e2) / reps / 1e3
    work = sum(o.ndof * s.nstates for o, s in zip(ops, systems))
    log(f"graph replay {t_graph:.3f} s, one stream eager {t_eager:.3f} s")
    print(json.dumps({"mode": "batch", "problems": len(jobs), "streams": ns, "graphs": b.ngraphs,
                      "blocks": blocks.tolist(),
                      "stream_of_job": sof.tolist(), "t_graph_s": t_graph, "t_eager_one_stream_s": t_eager,
                      "dof_columns_per_s_graph": work * 25 / t_graph}), flush=True)
    b.close()


def complex_mode(dev, args):
    """The paper workload as a complex (k-point) operator: Bloch vector at
    reduced coordinates (0.25, 0.10, 0.35), 1024 complex states filtered in
    blocks of 128 complex columns (256 real columns, as the real block),
    Chebyshev degree 30.  From one Rayleigh-Ritz of random vectors: one mixed
    and one FP64 filter pass from the same start, each followed by the FP64
    Rayleigh-Ritz; the wanted Ritz values of the two are compared."""
    import dataclasses

    import torch

    from paper_2604_26037_amd import FP32, FP64, Operator
    from workloads import make_system
    t0 = time.time()
    s = make_system(args.config)
    kappa = np.array([0.25, 0.10, 0.35])
    s = dataclasses.replace(s, kpoint=2.0 * np.pi * kappa / np.asarray(s.box, dtype=np.float64), is_complex=True)
    op = Operator(s)
    M, N, B, m = op.ndof, s.nstates, s.block // 2, s.cheb_degree
    log(f"complex operator built in {time.time() - t0:.1f} s: M={M} N={N} complex, block {B}, m={m}")
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(s.x_seed) % (2 ** 63))
    X = torch.randn((M, N), generator=gen, dtype=torch.complex128, device=dev)
    tmin, tmax, beta = op.lanczos_bounds(k=20)
    bU = tmax + beta
    ws_f = op.workspace(max(op.cheb_filter_workspace(N, B, FP64), op.cheb_filter_workspace(N, B, FP32)))
    ws_r = op.workspace(op.rayleigh_ritz_workspace(N))
    # warm-up: one Rayleigh-Ritz and one whole pass of each precision on a
    # copy (the first solver calls and the first pass over freshly allocated
    # buffers run slower than the ones after them)
    Xw = X.clone()
    lam_w, _ = op.rayleigh_ritz(Xw, ws=ws_r)
    lw = lam_w.cpu().numpy()
    for prec in (FP32, FP64):
        op.cheb_filter(Xw, lam_w, m, float(lw[0]), float(lw[-1]), bU, block=B, prec=prec, out=Xw, ws=ws_f)
    torch.cuda.synchronize()
    del Xw, lam_w
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    ev[0].record()
    lam, res = op.rayleigh_ritz(X, ws=ws_r)
    ev[1].record()
    lh = lam.cpu().numpy()
    Xb = X.clone()
    ev[2].record()
    op.cheb_filter(Xb, lam, m, float(lh[0]), float(lh[-1]), bU, block=B, prec=FP32, out=Xb, ws=ws_f)
    ev[3].record()
    lam32, _ = op.rayleigh_ritz(Xb, ws=ws_r)
    del Xb
    ev[4].record()
    op.cheb_filter(X, lam, m, float(lh[0]), float(lh[-1]), bU, block=B, prec=FP64, out=X, ws=ws_f)
    ev[5].record()
    lam64, _ = op.rayleigh_ritz(X, ws=ws_r)
    torch.cuda.synchronize()
    nw = int(np.ceil(N / 1.2))
    err = float((lam32[:nw] - lam64[:nw]).abs().max().item())
    t_rr, t32, t64 = (ev[2 * i].elapsed_time(ev[2 * i + 1]) / 1e3 for i in range(3))
    log(f"complex: mixed filter pass {t32:.3f} s, FP64 {t64:.3f} s, Rayleigh-Ritz {t_rr:.3f} s, "
        f"wanted-eigenvalue difference {err:.3e} Ha")
    print(json.dumps({"mode": "complex", "kpoint_reduced": kappa.tolist(), "M": M, "nstates": N, "block": B,
                      "degree": m, "filter_mixed_s": t32, "filter_fp64_s": t64, "speedup_mixed_vs_fp64": t64 / t32,
                      "rayleigh_ritz_s": t_rr, "eig_err_mixed_vs_fp64_ha": err}), flush=True)


def rr_mode(op, s, gen, dev, args):
    """Rayleigh-Ritz alone on the workload's N states (FP64 rotation and
    residual norms): one warm-up call, then `steps` timed calls, each on a
    fresh copy of the same random block (the copy is outside the timing)."""
    import torch

    M, N = op.ndof, s.nstates
    X = torch.randn((M, N), generator=gen, dtype=torch.float64, device=dev)
    ws_r = op.workspace(op.rayleigh_ritz_workspace(N))
    Xc = X.clone()
    op.rayleigh_ritz(Xc, ws=ws_r)
    ts = []
    for k in range(max(1, args.steps)):
        Xc.copy_(X)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lam, res = op.rayleigh_ritz(Xc, ws=ws_r)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
        log(f"Rayleigh-Ritz {k}: {ts[-1]:.4f} s")
    print(json.dumps({"mode": "rr", "M": M, "nstates": N, "rayleigh_ritz_s": float(np.mean(ts)),
                      "calls_s": ts, "lambda_min": float(lam[0].item())}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="paper")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true", help="do not time the FP64 filter")
    ap.add_argument("--hx-reps", type=int, default=5)
    ap.add_argument("--skip-graded", action="store_true",
                    help="do not time the two-level-mesh GGA variant of the workload")
    ap.add_argument("--mode", default="full", choices=["full", "kernels", "rr", "batch"],
                    help="kernels: only the cell-local operator and a calibration copy (for counters); "
                         "rr: Rayleigh-Ritz alone; batch: the graph-captured filter of 24 uneven problems")
    ap.add_argument("--batch-count", type=int, default=24)
    ap.add_argument("--one-stream", action="store_true",
                    help="filter blocks one after another on one stream (no two blocks in flight)")
    ap.add_argument("--complex", action="store_true",
                    help="time the filter of the workload as a complex (k-point) operator instead")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the filter shards "
              "by column blocks across GPUs but no multi-GPU path is built here.", file=sys.stderr)
        sys.exit(2)
    if args.mode == "batch":
        # The 24-problem batch (27,000-343,000 DOFs) ends the process with a
        # host segmentation fault early in pawfe_batch_create with the current
        # library (real and complex problems alike); the cause is not found
        # yet, so this mode stays off.  Small batches are covered by the tests.
        sys.exit("bench --mode batch is disabled: the full-size batch crashes in pawfe_batch_create "
                 "(host segmentation fault, cause not found)")

    import torch

    from paper_2604_26037_amd import BF16X3, FP32, FP64, Operator
    from workloads import make_system

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.complex:
        return complex_mode(dev, args)
    t0 = time.time()
    s = make_system(args.config)
    op = Operator(s)
    M, N, B, m = op.ndof, s.nstates, s.block, s.cheb_degree
    log(f"operator built in {time.time() - t0:.1f} s: M={M} N={N} B={B} m={m} colours={op.ncolour}")

    gen = torch.Generator(device=dev)
    gen.manual_seed(int(s.x_seed) % (2 ** 63))
    if args.mode == "kernels":
        return kernels_mode(op, s, gen, dev, args)
    if args.mode == "rr":
        return rr_mode(op, s, gen, dev, args)
    X = torch.randn((M, N), generator=gen, dtype=torch.float64, device=dev)

    tmin, tmax, beta = op.lanczos_bounds(k=20)
    bU = tmax + beta
    log(f"Lanczos: theta in [{tmin:.4f}, {tmax:.4f}], |beta_k| = {beta:.3e}, b_U = {bU:.4f}")

    # a workspace of one block state keeps the filter on one stream
    nws = B if args.one_stream else N
    ws_f = op.workspace(max(op.cheb_filter_workspace(nws, B, FP64), op.cheb_filter_workspace(nws, B, FP32)))
    ws_r = op.workspace(op.rayleigh_ritz_workspace(N))
    lam, res = op.rayleigh_ritz(X, ws=ws_r)
    torch.cuda.synchronize()
    log("initial Rayleigh-Ritz done")

    def filt(Xc, lamc, prec, out=None, R=None):
        lc = lamc.cpu().numpy()
        return op.cheb_filter(Xc, lamc, m, float(lc[0]), float(lc[-1]), bU, block=B, prec=prec,
                              out=Xc if out is None else out, ws=ws_f, R=R)

    # --- precision check: three ChFSI iterations (filter + FP64 Rayleigh-Ritz)
    # in FP64, FP32 and bf16x3 from the same Rayleigh-Ritz start; per
    # iteration the largest wanted-eigenvalue deviation from the FP64
    # trajectory and the largest wanted residual norm of each ---
    nw = int(np.ceil(N / 1.2))
    traj = {}
    for name, prec in (("fp64", FP64), ("fp32", FP32), ("bf16x3", BF16X3)):
        Xp, lp = X.clone(), lam.clone()
        rows = []
        for it in range(3):
            filt(Xp, lp, prec)
            lp, rp = op.rayleigh_ritz(Xp, ws=ws_r)
            rows.append((lp[:nw].clone(), float(rp[:nw].max().item())))
        traj[name] = rows
        del Xp
    precision = {}
    for name in ("fp32", "bf16x3"):
        precision[name] = [
            {"iteration": it + 1,
             "eig_err_vs_fp64_ha": float((traj[name][it][0] - traj["fp64"][it][0]).abs().max().item()),
             "max_wanted_resnorm": traj[name][it][1],
             "max_wanted_resnorm_fp64": traj["fp64"][it][1]} for it in range(3)]
        log(f"{name} vs FP64 over 3 iterations: eigenvalue error "
            + ", ".join(f"{r['eig_err_vs_fp64_ha']:.2e}" for r in precision[name])
            + " Ha; max wanted residual " + ", ".join(f"{r['max_wanted_resnorm']:.2e}" for r in precision[name]))
    eig_err = max(r["eig_err_vs_fp64_ha"] for r in precision["fp32"])
    del traj

    # --- warmup and timed steps: mixed filter pass + FP64 RR, as a ChFSI
    # iteration runs them: Rayleigh-Ritz keeps the residual of the Ritz pairs
    # it forms for the residual norms, and the next filter pass starts from it
    # (step 2 of Algorithm 2 is not formed twice) ---
    Rres = torch.empty_like(X)
    lam, res = op.rayleigh_ritz(X, ws=ws_r, R=Rres)
    for _ in range(args.warmup):
        filt(X, lam, FP32, R=Rres)
        lam, res = op.rayleigh_ritz(X, ws=ws_r, R=Rres)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_wall = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        filt(X, lam, FP32, R=Rres)
        ev[k][1].record()
        lam, res = op.rayleigh_ritz(X, ws=ws_r, R=Rres)
        ev[k][2].record()
        log(f"step {k}: done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    t_filter = float(np.mean([a.elapsed_time(b) for a, b, _ in ev])) / 1e3
    t_rr = float(np.mean([b.elapsed_time(c) for _, b, c in ev])) / 1e3

    # --- Rayleigh-Ritz with the mixed-precision subspace rotation, same input
    # (one untimed call first: the first FP32 GEMM loads its kernels) ---
    Xm = X.clone()
    op.rayleigh_ritz(Xm, ws=ws_r, sr_prec=FP32)
    Xm.copy_(X)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lam_m, res_m = op.rayleigh_ritz(Xm, ws=ws_r, sr_prec=FP32)
    e1.record()
    Xd64 = X.clone()
    lam_d, res_d = op.rayleigh_ritz(Xd64, ws=ws_r)
    torch.cuda.synchronize()
    t_rr_mixed = e0.elapsed_time(e1) / 1e3
    sr_res_change = float(((res_m[:nw] - res_d[:nw]).abs() / res_d[:nw]).max().item())
    del Xm, Xd64
    log(f"Rayleigh-Ritz with mixed-precision rotation {t_rr_mixed:.3f} s (FP64 rotation {t_rr:.3f} s); "
        f"wanted residual norms change by at most {sr_res_change:.2e} (relative)")

    # --- FP64 and bf16x3 filter passes (same work, from the same Ritz pairs
    # and handed-over residual, into a separate output), and the mixed and
    # FP64 passes that form the residual themselves (Algorithm 2 as a
    # stand-alone call) ---
    Xout = torch.empty_like(X)

    def timed_pass(prec, R, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(reps):
            e0.record()
            filt(X, lam, prec, out=Xout, R=R)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        return float(np.mean(times))

    t_filter64 = t_filter64_own = None
    if not args.skip_fp64:
        t_filter64 = timed_pass(FP64, Rres, args.steps)
        t_filter64_own = timed_pass(FP64, None, 1)
        log(f"FP64 filter pass {t_filter64:.3f} s, mixed {t_filter:.3f} s (residual from Rayleigh-Ritz); "
            f"FP64 {t_filter64_own:.3f} s forming it")
    t_filter_own = timed_pass(FP32, None, args.steps)
    log(f"mixed filter pass forming its own residual {t_filter_own:.3f} s")

    # --- bf16x3 filter pass timing (cell contractions as bf16x3 split products) ---
    t_filter_bf3 = timed_pass(BF16X3, Rres, 1)
    log(f"bf16x3 filter pass {t_filter_bf3:.3f} s")
    del Xout

    # --- dominant kernel: cell-local operator (K + V) on one 256-column block ---
    cd, col, sco, sc, sno, sn = op.dofmap()
    supp_nodes = np.diff(sno)
    nloc_flops = local_flops_per_cell_col(s.degree + 1, s.nq) * op.ncells
    nl_flops = nonlocal_flops_per_col(s, supp_nodes)
    hx = {}
    for name, prec, dt in (("fp64", FP64, torch.float64), ("fp32", FP32, torch.float32)):
        Xs = X[:, :B].to(dt).contiguous()
        Ys = torch.zeros_like(Xs)
        op.apply_local(Xs, Ys, 0, 1.0, prec)
        op.apply_H(Xs, out=Ys, prec=prec)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        for _ in range(args.hx_reps):
            op.apply_local(Xs, Ys, 0, 1.0, prec)
        e1.record()
        for _ in range(args.hx_reps):
            op.apply_H(Xs, out=Ys, prec=prec)
        e2.record()
        torch.cuda.synchronize()
        t_loc = e0.elapsed_time(e1) / 1e3 / args.hx_reps
        t_h = e1.elapsed_time(e2) / 1e3 / args.hx_reps
        esz = 8 if prec == FP64 else 4
        loc_bytes = (3.0 * M * B + op.nquad) * esz      # read X, read+write Y, V(q)W
        # algorithmic HBM bytes of apply_H: read X, write Y, read the support
        # rows of every atom for C^T X, the V(q)W table and the C^a values
        hx_bytes = ((2.0 * M + float(np.sum(supp_nodes))) * B + op.nquad
                    + float(np.sum(supp_nodes * np.asarray(s.nproj)))) * esz
        hx[name] = dict(t_local=t_loc, t_apply_H=t_h,
                        hx_gflops=(nloc_flops + nl_flops) * B / t_h / 1e9,
                        local_tflops=nloc_flops * B / t_loc / 1e12,
                        local_bytes=loc_bytes,
                        hx_bytes=hx_bytes,
                        hx_gbs=hx_bytes / t_h / 1e9,
                        hx_hbm_frac=hx_bytes / t_h / 1e9 / PEAK_HBM_GBS)
        log(f"HX {name}: apply_H {t_h * 1e3:.2f} ms ({hx[name]['hx_gflops']:.0f} GFLOP/s, "
            f"{hx[name]['hx_gbs']:.0f} GB/s = {100 * hx[name]['hx_hbm_frac']:.1f} % of HBM), "
            f"local {t_loc * 1e3:.2f} ms ({hx[name]['local_tflops']:.2f} TFLOP/s)")
        del Xs, Ys

    # --- the filter's fused step kernel (the dominant kernel of a filter pass) ---
    step_t = {}
    for name, prec, dt in (("fp64", FP64, torch.float64), ("fp32", FP32, torch.float32)):
        step_t[name] = time_step_kernel(op, X, B, prec, dt, args.hx_reps)
        log(f"filter step kernel {name}: {step_t[name] * 1e3:.3f} ms per colour launch "
            f"({nloc_flops * B / op.ncolour / step_t[name] / 1e12:.2f} TFLOP/s of cell flops)")

    # --- BF16 halo of a z-slab (one GPU's part of the reduced-precision
    # nearest-neighbour exchange): pack and unpack-add of the two shared node
    # planes of a 5-layer slab, one 256-column block ---
    Yh = X[:, :B].to(torch.float32).contiguous()
    hbuf = op.halo_pack_bf16(Yh, 5, 10)
    op.halo_unpack_bf16(hbuf, Yh, 5, 10)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    reps = 20
    e0.record()
    for _ in range(reps):
        op.halo_pack_bf16(Yh, 5, 10, buf=hbuf)
    e1.record()
    for _ in range(reps):
        op.halo_unpack_bf16(hbuf, Yh, 5, 10)
    e2.record()
    torch.cuda.synchronize()
    prow = (s.ncell[0] * s.degree) * (s.ncell[1] * s.degree)
    t_pack, t_unpack = e0.elapsed_time(e1) / reps / 1e3, e1.elapsed_time(e2) / reps / 1e3
    halo_info = {"planes": 2, "nodes_per_plane": prow, "columns": B,
                 "message_bytes_bf16": 2 * prow * B * 2, "message_bytes_fp64": 2 * prow * B * 8,
                 "pack_us": t_pack * 1e6, "unpack_add_us": t_unpack * 1e6,
                 "pack_gbs": 2 * prow * B * (4 + 2) / t_pack / 1e9,
                 "unpack_gbs": 2 * prow * B * (2 + 4 + 4) / t_unpack / 1e9}
    log(f"BF16 halo: pack {t_pack * 1e6:.1f} us, unpack-add {t_unpack * 1e6:.1f} us for 2 x {prow} nodes x {B} "
        f"columns ({halo_info['message_bytes_bf16'] / 1e6:.1f} MB in BF16, 4x less than FP64)")
    del Yh, hbuf

    # --- band-energy gradient (differentiation workload): 512 states ---
    ng = min(512, N)
    Xg = X[:, :ng].contiguous()
    op.band_energy_grad(Xg)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        Eg, dVg, dDg = op.band_energy_grad(Xg)
    e1.record()
    torch.cuda.synchronize()
    grad_info = {"states": ng, "s_per_call": e0.elapsed_time(e1) / 3 / 1e3,
                 "outputs": f"E, dE/dV at {op.nquad} quadrature points, dE/dDelta_H ({int(dDg.numel())} entries)"}
    log(f"band-energy gradient on {ng} states: {grad_info['s_per_call'] * 1e3:.1f} ms per call")
    del Xg, Eg, dVg, dDg

    graded = None if args.skip_graded else graded_gga_leg(s, N, B, m, dev)

    # roofline of the dominant kernel of the filter pass: its fused step
    # kernel on the vector ALUs (FP32), one colour (1/8 of the cells) x 256
    # columns per launch; algorithmic flops = 72,668 per cell-column
    # (sum-factorized K + V) plus 5 per DOF-column for the node part of the
    # step (on average 1/8 of the DOFs per launch); the launch duration is the
    # mean of the FP32 launches timed above with events on their stream
    per_launch_flops = (nloc_flops + STEP_NODE_FLOPS * M) * B / op.ncolour
    t_launch = step_t["fp32"]
    achieved = per_launch_flops / t_launch / 1e12
    roof = {
        "kernel": "k_cell_valu<float,7,8,Step> (filter step: cell-local K + V on M_D^-1 R_Y, node part at the "
                  "first visit; one colour per launch)",
        "bound": "alu",
        "achieved": achieved,
        "peak": PEAK_VALU_F32_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_VALU_F32_TFLOPS,
        "traffic": measured_traffic(),
        "per_launch_flops": per_launch_flops,
        "avg_launch_ms": t_launch * 1e3,
        "peak_without_packed_fp32": PEAK_VALU_F32_SCALAR_TFLOPS,
        "frac_without_packed_fp32": achieved / PEAK_VALU_F32_SCALAR_TFLOPS,
    }

    out = {
        "metric": METRIC,
        "value": t_filter,
        "unit": "s/pass",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (recurrence) + f64 (residual correction, Rayleigh-Ritz)",
        "data": "synthetic (seeded Gaussian wells, jittered lattice atoms, random-normal start)",
        "config": {
            "workload": f"{s.name}: periodic {s.ncell[0]}x{s.ncell[1]}x{s.ncell[2]} cells, degree "
                        f"{s.degree} ({M} DOFs), nq={s.nq}, {len(s.pos)} atoms x {int(s.nproj[0])} "
                        f"projectors, N={N}, block={B}, Chebyshev degree {m}",
            "step": "mixed filter pass over all states + FP64 Rayleigh-Ritz + residual norms; the filter "
                    "starts from the residual of the Ritz pairs that the previous Rayleigh-Ritz formed",
            "filter_streams": 1 if args.one_stream else 2,
        },
        "filter_fp64_s_per_pass": t_filter64,
        "filter_bf16x3_s_per_pass": t_filter_bf3,
        "speedup_mixed_vs_fp64": (t_filter64 / t_filter) if t_filter64 else None,
        "filter_mixed_s_per_pass_own_residual": t_filter_own,
        "filter_fp64_s_per_pass_own_residual": t_filter64_own,
        "rayleigh_ritz_s": t_rr,
        "rayleigh_ritz_mixed_rotation_s": t_rr_mixed,
        "mixed_rotation_resnorm_rel_change": sr_res_change,
        "eig_err_mixed_vs_fp64_ha": eig_err,
        "precision_3_iterations": precision,
        "band_energy_grad": grad_info,
        "halo_bf16": halo_info,
        "hx": hx,
        "step_kernel_ms_per_launch": {k: v * 1e3 for k, v in step_t.items()},
        "graded_gga": graded,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample)...")
        out["cpu_baseline"] = cpu_baseline(s, N, m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
