#!/usr/bin/env python3
"""Throughput of the MOT-JVIE march on one MI355X.

A step is one pass of the whole hot path for one time step: forward FFT of the newest
current, spectral multiply-accumulate over all ell history lags, inverse FFT, right-hand
side assembly (excitation, FIR, local terms) and the Z_0 solve.

Set-up marches an untimed prefill of at least ell + 1 steps (reported as
config.prefill_steps), so that every timed step sums the full history whatever the flags;
the prefill ends where the `warmup` steps that follow end on a time-block boundary.  Then
`warmup` untimed steps, then exactly `steps` timed steps.  The far part of the history sum
runs once per time block (8 steps by default), at the first step of each block, so the timed
window starts with one; a window that is a whole number of blocks (the default 48 steps hold
6) weighs it exactly.  Kernel generation and spectra are one-time setup and are reported
separately.

Prints one JSON line (metric voxel*steps/s, FP64).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # MI355X vector FP64 (MFMA FP64 has the same peak)
METRIC = "voxel·steps/s FP64 at 1.1M voxels; % HBM roofline; batched/adjoint vs plain"

WORKLOADS = {
    "C5": "104^3 cube of side 100h eps_r=12 in a 2-voxel eps_r=1 margin, c dt = h, x-pol +z Gaussian "
          "plane wave sigma=8 dt delay 6 sigma, 17-tap binomial FIR delta=0.01",
    "C2": "32^3 sphere r=15h eps_r=12, c dt = h, x-pol +z Gaussian sigma=4 dt, 17-tap binomial FIR delta=0.01",
    "C1": "8^3 cube eps_r=4, c dt = h, x-pol +z Gaussian sigma=4 dt, no FIR",
    "C3": "64^3 eps_r box-smoothed U[2,20], 16 plane waves sigma=6 dt, 17-tap binomial FIR delta=0.01",
    "C4": "48^3 eps_r=10 with a 16^3 design region U[1,12], x-pol +z Gaussian sigma=4 dt, 17-tap FIR delta=0.01",
    "C5s": "C5 with c dt = h/2 (ell = 362)",
    "C5p": "C5 on voxels 1 x 0.7 x 1.3 with c dt = 0.7 (ell = 266)",
}


def mac_source_digest() -> str:
    """Digest of the far-part MAC kernel's source (from its header comment to the next kernel)."""
    with open(os.path.join(ROOT, "paper_2407_03323_amd", "csrc", "mj_march.hip")) as fh:
        src = fh.read()
    a = src.index("// Far part.")
    b = src.index("// near part of step", a)
    return hashlib.sha1(src[a:b].encode()).hexdigest()[:12]


def mac_traffic(workload: str, overlap: bool = False):
    """HBM bytes per MAC launch from the committed rocprofv3 counter summary, if it was taken
    on the current MAC source and of the same launch (in line, or on the second stream);
    else None."""
    path = os.path.join(ROOT, "profiles", "mac_traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("mac_source_sha1_12") != mac_source_digest() or bool(d.get("overlap", False)) != overlap:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(prob, ell: int, target_seconds: float = 20.0):
    """The oracle's direct history sum (oracle/direct.c, unchanged) timed on the host on a
    bounded sample of the same grid: a few target voxels, every source voxel and 4 of the
    ell lags, scaled linearly to all voxels and all lags (the triple loop's cost is exactly
    linear in both).  The kernel table holds zeros: the loop's cost does not depend on the
    values.  Z_0 solve and excitation are not included (they are O(M) per step against
    O(M^2 ell) for the history sum)."""
    from oracle import mot
    U, V, W, M = prob.U, prob.V, prob.W, prob.M
    nlag = 4
    K = np.zeros((nlag + 1, 6, 2 * W - 1, 2 * V - 1, 2 * U - 1))
    Jh = np.zeros((nlag, 3, W, V, U))
    rng = np.random.default_rng(0)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    nt = max(threads, 8)
    t0 = time.perf_counter()
    mot.conv(K, Jh, rng.integers(0, M, nt))
    dt = time.perf_counter() - t0
    # grow the sample to about target_seconds
    nt2 = int(min(M, max(nt, nt * target_seconds / max(dt, 1e-3))))
    nt2 = max(threads, (nt2 // threads) * threads)
    t0 = time.perf_counter()
    mot.conv(K, Jh, rng.integers(0, M, nt2))
    dt2 = time.perf_counter() - t0
    per_step = dt2 * (M / nt2) * (ell / nlag)
    return {"value": M / per_step, "unit": "voxel·steps/s", "cores": threads, "kind": "oracle",
            "sample": "direct history sum of the oracle for %d target voxels x all %d sources x %d of %d lags "
                      "(%.1f s), scaled to %d targets and %d lags" % (nt2, M, nlag, ell, dt2, M, ell)}


def timed_march(solver, steps: int, warmup: int, probes_out=None):
    """Wall time of `steps` march steps after `warmup` untimed ones (device synchronised)."""
    import torch
    if warmup:
        solver.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.run(steps, None, probes_out)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def batched_ratio(steps: int = 16):
    """C3: 16 plane waves marched together against one, on the 64^3 heterogeneous grid.
    Throughput counted per right-hand side (voxel.RHS.steps/s) of the batched march over
    the single-RHS march of the same grid."""
    import torch
    import workloads as wl
    from paper_2407_03323_amd import motjvie
    prob = wl.config("C3")
    out = {"workload": "C3: 64^3 eps_r box-smoothed U[2,20], 16 plane waves sigma=6 dt, 17-tap FIR",
           "steps": steps}
    for nr in (16, 1):
        s = motjvie.Solver(prob.U, prob.V, prob.W, prob.eps, fir=prob.fir, n_rhs=nr)
        s.set_plane_waves(prob.waves[:nr])
        ell = s.ell
        dt = timed_march(s, steps, ell + 8)
        out["rhs%d_voxel_rhs_steps_per_s" % nr] = prob.M * steps * nr / dt
        out["rhs%d_ms_per_step" % nr] = 1e3 * dt / steps
        s.close()
        del s
        torch.cuda.synchronize()
    out["per_rhs_speedup"] = out["rhs16_voxel_rhs_steps_per_s"] / out["rhs1_voxel_rhs_steps_per_s"]
    return out


def adjoint_ratio(n_steps: int = 800, ckpt: int = 50):
    """C4: gradient of sum |E^s|^2 over 32 probes (radius 48 h) with respect to eps_r of all
    48^3 voxels by the checkpointed transposed march, against the plain forward march of the
    same steps with the probes."""
    import torch
    import workloads as wl
    from paper_2407_03323_amd import motjvie
    prob = wl.config("C4")
    s = motjvie.solver_for(prob)
    t0 = time.perf_counter()
    s.set_probes(prob.probes)
    torch.cuda.synchronize()
    t_table = time.perf_counter() - t0
    P = torch.zeros((n_steps, 1, len(prob.probes), 3), dtype=torch.float64, device="cuda")
    t_fwd = timed_march(s, n_steps, 0, P)
    s.reset()
    g = torch.zeros((prob.W, prob.V, prob.U), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.adjoint_gradient(n_steps, g, ckpt)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    st = s.stats()
    s.close()
    return {"workload": "C4: 48^3 eps_r=10 with a 16^3 design region U[1,12], 32 probes r=48h, 17-tap FIR",
            "steps": n_steps, "ckpt_every": ckpt, "segments": int(st["adjoint_segments"]),
            "forward_s": t_fwd, "gradient_s": t_adj, "gradient_over_forward": t_adj / t_fwd,
            "gradient_forward_pass_ms": st["adjoint_forward_ms"],
            "gradient_backward_pass_ms": st["adjoint_backward_ms"], "probe_table_s": t_table,
            "checkpoint_bytes": int(st["adjoint_checkpoint_bytes"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=48, help="timed steps; a multiple of the time block")
    ap.add_argument("--warmup", type=int, default=8,
                    help="untimed steps after the prefill of at least ell + 1 steps that set-up marches")
    ap.add_argument("--workload", default="C5", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched (C3) and adjoint (C4) ratios")
    ap.add_argument("--time-block", type=int, default=0, help="steps per time block (0 = library default)")
    ap.add_argument("--outer-block", type=int, default=0, help="steps per outer time block (three levels; 0 = two)")
    ap.add_argument("--z0-solver", type=int, default=0, help="0 by size, 1 CG, 2 Chebyshev")
    ap.add_argument("--z0-graphs", type=int, default=0, help="replay the Chebyshev batches from HIP graphs")
    ap.add_argument("--outer-overlap", type=int, default=0,
                    help="0 library default, 1 outer level in line, 2 on a second stream")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(how the march would shard is a design note, not code); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2407_03323_amd import motjvie
    if not os.path.exists(motjvie.LIB_PATH):
        from paper_2407_03323_amd import build
        build.build()
    import workloads as wl

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    prob = wl.config(args.workload)
    t_setup = time.perf_counter()
    solver = motjvie.solver_for(prob, time_block=args.time_block, outer_block=args.outer_block,
                                z0_solver=args.z0_solver, z0_graphs=args.z0_graphs,
                                outer_overlap=args.outer_overlap)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    info = solver.info()
    ell = info["ell"]
    warmup = max(0, args.warmup)
    B = info["time_block"]
    period = info["outer_block"] or B   # steps between far launches
    # prefill: at least ell + 1 steps, so that the ring holds ell sources and every far launch
    # sums all ell lags; blocks start at steps 2, 2 + period, ..., and the step after
    # prefill + warmup steps starts one when prefill + warmup = 1 mod period
    prefill = ell + 1
    while period > 1 and (prefill + warmup - 1) % period:
        prefill += 1
    print("setup %.2f s (kernels %.0f ms, spectra %.0f ms), ell=%d, pads %dx%dx%d, %.1f GB; prefill %d steps" % (
        t_setup, info["gen_ms"], info["spectra_ms"], ell, info["Nx"], info["Ny"], info["Nz"],
        info["device_bytes"] / 1e9, prefill), file=sys.stderr, flush=True)
    solver.run(prefill)
    if warmup:
        solver.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.run(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = solver.stats()
    if period > 1 and args.steps % period:
        print("note: %d timed steps are not a whole number of %d-step time blocks: the window starts with a "
              "far launch and holds %d of them, %.3f per step against 1/%d" % (
                  args.steps, period, st["far_launches"], st["far_launches"] / args.steps, period),
              file=sys.stderr, flush=True)
    M = prob.M
    value = M * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    print("phases ms/step: fft %.3f mac %.3f ifft %.3f epi %.3f z0 %.3f (cg %.1f it)" % (
        st["fft_fwd_ms"], st["mac_ms"], st["fft_inv_ms"], st["epilogue_ms"], st["z0_ms"], st["cg_iters"]),
        file=sys.stderr, flush=True)

    # roofline of the far-part MAC kernel: algorithmic bytes per launch
    Nx, Ny, Nz = info["Nx"], info["Ny"], info["Nz"]
    Hx = Nx // 2 + 1
    half = Hx * Ny * Nz                       # half-spectrum points
    octant = Hx * (Ny // 2 + 1) * (Nz // 2 + 1)
    R = info["n_rhs"]
    # bytes of the Jhat spectra of one step (all right-hand sides) and of one (octant) Khat lag,
    # which the right-hand sides share
    SJ, SK = 48.0 * half * R, 48.0 * octant
    B2 = info["outer_block"]
    TB = B2 if B2 else B                      # targets of one far launch
    ov = bool(info["outer_overlap"])
    if ov:
        # the launch on the second stream: lags B2 + 1 .. ell of the next outer block's B2
        # targets (sources before the current block), B2 partial sums written.  Its duration
        # is measured on that stream while the march shares the device
        bytes_launch = (ell - B2) * (SJ + SK) + B2 * SJ
        launch_ms = st["side_launch_ms"]
        kname = "k_mac_win<%d> (outer level of three, on the second stream, history MAC)" % TB
    elif B > 1:
        # per launch: every one of the ell lags once (Jhat and Khat) and TB partial sums written
        bytes_launch = ell * (SJ + SK) + TB * SJ
        launch_ms = st["far_launch_ms"]
        kname = ("k_mac_win<%d> (outer level of three, history MAC)" % TB if B2 else
                 "k_mac_win<%d> (time-blocked history MAC, far part)" % TB)
    else:
        bytes_launch = ell * (SJ + SK) + SJ
        launch_ms = st["mac_ms"]
        kname = "k_mac (history MAC, all lags every step)"
    achieved = bytes_launch / (launch_ms / 1e3) / 1e9
    # FP64 work of the same launch: a real symmetric 3x3 times a complex 3-vector is 36 FLOP per
    # (lag, half-spectrum point, target); target t of a block sums lags t + 1 .. ell
    flop_launch = 36.0 * half * R * (sum(ell - B2 - t for t in range(TB)) if ov else
                                     sum(ell - t for t in range(TB)) if B > 1 else ell)
    tflops = flop_launch / (launch_ms / 1e3) / 1e12
    fp64 = {"flop_per_launch": flop_launch, "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tflops / FP64_PEAK_TFLOPS}
    traffic = mac_traffic(args.workload, ov)
    # the whole FFT convolution of a step (forward FFT, MAC at every level, inverse FFT):
    # algorithmic bytes per step over the measured time of those three phases
    U, V, W = prob.U, prob.V, prob.W
    fft_bytes = R * (8.0 * 3 * M + 16.0 * 3 * (Hx * V * W + Hx * V * W + Hx * Ny * W + Hx * Ny * W + half))
    if B > 1:
        # near part of the step at position t of an inner block: read and write F[t], t lags
        near_bytes = sum(2 * SJ + t * (SJ + SK) for t in range(1, B)) / B
        if ov:
            # on the caller's stream at each outer block start: the B2 sums from the second
            # stream read, the B2 sources of the block before, lags 1 .. 2 B2 - 1, B2 sums written
            mac_step = (3 * B2 * SJ + (2 * B2 - 1) * SK) / B2 + near_bytes
        else:
            mac_step = bytes_launch / TB + near_bytes
        if B2:
            # middle part at the start of inner block q > 0: its B sums start from the outer ones,
            # q B sources of the outer block, lags up to q B + B - 1, B sums written
            mid = sum(B * SJ + q * B * SJ + (q * B + B - 1) * SK + B * SJ for q in range(1, B2 // B))
            mac_step += mid / B2
    else:
        mac_step = bytes_launch
    conv_bytes = 2 * fft_bytes + mac_step
    conv_ms = st["fft_fwd_ms"] + st["mac_ms"] + st["fft_inv_ms"]
    conv = {"bytes_per_step": conv_bytes, "ms_per_step": conv_ms,
            "achieved": conv_bytes / (conv_ms / 1e3) / 1e9, "unit": "GB/s",
            "frac": conv_bytes / (conv_ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel·steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.workload, WORKLOADS[args.workload]),
                   "grid": [prob.U, prob.V, prob.W], "voxels": M, "ell": ell, "pad": [Nx, Ny, Nz],
                   "fir_taps": len(prob.fir), "setup_s": round(t_setup, 3), "prefill_steps": prefill,
                   "far_launches_timed": int(st["far_launches"]),
                   "phase_ms": {k: round(st[k], 4) for k in ("fft_fwd_ms", "mac_ms", "fft_inv_ms", "epilogue_ms",
                                                              "z0_ms")},
                   "cg_iters": round(st["cg_iters"], 2), "time_block": B, "outer_block": B2,
                   "z0_solver": "CG" if info["z0_solver"] == 1 else "Chebyshev",
                   "mid_launch_ms": round(st["mid_launch_ms"], 4),
                   "fft_pencils": [info["fft_pencils_x"], info["fft_pencils_y"], info["fft_pencils_z"]],
                   "far_launch_ms": round(st["far_launch_ms"], 4), "near_launch_ms": round(st["near_launch_ms"], 4),
                   "outer_overlap": ov, "side_launch_ms": round(st["side_launch_ms"], 4),
                   "side_launches_timed": int(st["side_launches"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname, "bytes_per_launch": bytes_launch,
                     "avg_launch_ms": launch_ms, "fp64": fp64, "convolution": conv},
    }
    solver.close()
    del solver
    torch.cuda.synchronize()
    if not args.no_extras:
        line["batched"] = batched_ratio()
        print("batched: %.3g per-RHS speedup" % line["batched"]["per_rhs_speedup"], file=sys.stderr, flush=True)
        line["adjoint"] = adjoint_ratio()
        print("adjoint: gradient/forward %.2f" % line["adjoint"]["gradient_over_forward"], file=sys.stderr,
              flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, ell)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
