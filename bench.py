"""Benchmark of the velocity Schur-complement operator and the implicit time
step on one MI355X.

Workload (synthetic, shaped like the paper's 2D runs): 64x64 split-square
mesh of the unit square (8192 triangles) with +-20% vertex jitter, free
surface, p = 3 in space and p_gamma = 3 in time (space-time DG), three
lognormal layers, a 10 Hz Ricker point source, dt = 2.5e-3.

A "step" is one implicit time step of the whole hot path: right-hand side,
restarted GMRES on the velocity system to relative residual 1e-10, stress
back-substitution and end-of-slab update, all in the library's kernels on
inputs resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  `value` is the matvec-equivalent throughput of the
timed FP64 steps (velocity DOFs x operator applications / wall time);
`roofline` reports the operator apply (face + element kernels) against the
HBM peak from HIP-event timing of back-to-back applies; `cpu_baseline` is
the FP64 oracle's explicit Schur CSR mat-vec on a bounded 12x12 sample of
the same recipe.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(seconds=10.0):
    """The oracle, as it stands, timed on the host: explicit Schur CSR SpMV
    (SciPy, single-threaded) on the 12x12 version of the workload recipe."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle.assemble import Blocks
    from oracle.mesh import Topology
    from oracle.slab import Slab
    w = synth.workload("c2", scale=12)
    m = w["mesh"]
    with threadpool_limits(limits=1):
        B = Blocks(Topology(m.xyz, m.elem, m.period), w["p"], w["lam"], w["mu"], w["rho"])
        slab = Slab(B, w["p_gamma"], w["dt"], "stdg")
        S = slab.schur()
        v = np.random.default_rng(0).standard_normal(slab.nv)
        reps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            S @ v
            reps += 1
        dt = time.perf_counter() - t0
    return {"value": slab.nv * reps / dt / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": f"scipy CSR mat-vec of the explicit FP64 Schur complement on the 12x12 (288-triangle, "
                      f"{slab.nv} DOF, nnz {S.nnz}) version of the workload recipe, {reps} applies in {dt:.1f}s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--applies", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precond", default="block", choices=["none", "mass", "block"])
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB x 10 (scale for the rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1802_04516_amd as sdg
    import synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": nbytes, "copy_bytes_written_per_launch": nbytes,
                          "launches": 10}), flush=True)
        return
    w = synth.workload(args.workload)
    mesh = w["mesh"]
    scheme = sdg.SDG_SCHEME_CN if w["scheme"] == "cn" else sdg.SDG_SCHEME_STDG
    t0 = time.time()
    ctx = sdg.Context(0)
    sizes = ctx.setup(mesh.xyz, mesh.elem, mesh.period, w["p"], w["p_gamma"], scheme, w["dt"],
                      w["lam"], w["mu"], w["rho"],
                      sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND)
    log(f"setup {time.time() - t0:.1f}s: {sizes['n_elem']} elems, {sizes['n_face']} faces, "
        f"{sizes['n_vel_slab']} velocity DOFs, operator {sizes['op_bytes_f64'] / 1e6:.1f} MB")
    log(f"face-kernel autotune (us/apply, variants 0/1/2): f64 {sizes['tune_us_f64']} -> {sizes['op_variant']}, "
        f"f32 {sizes['tune_us_f32']} -> {sizes['op_variant_f32']}")
    src = w["sources"]
    if src is not None:
        ctx.set_sources(src["pos"], src["dir"])
    n = sizes["n_vel_slab"]
    tau = np.array(sizes["tau"])

    def amp_at(step):
        if src is None:
            return None
        t = step * w["dt"] + tau * w["dt"]
        return synth.ricker(t, src["f0"], src["t_delay"])[None, :]

    v = torch.zeros(sizes["n_vel_state"], dtype=torch.float64, device=dev)
    s = torch.zeros(sizes["n_stress_state"], dtype=torch.float64, device=dev)
    pc = {"none": sdg.SDG_PRECOND_NONE, "mass": sdg.SDG_PRECOND_MASS, "block": sdg.SDG_PRECOND_BLOCK}[args.precond]
    opts64 = sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F64, 1e-10, 5000, 30, 5, 10, 1e-4, pc)
    opts32 = sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F32, 1e-10, 5000, 30, 5, 10, 1e-4, pc)

    # the source switches on around t_delay; start the run so that the timed
    # steps see the wavelet
    step0 = int(0.05 / w["dt"]) if src is not None else 0
    for k in range(args.warmup):
        ctx.step(v, s, amp_at(step0 + k), opts=opts64)
    log(f"warmup {args.warmup} steps done")
    v_save, s_save = v.clone(), s.clone()

    # ---- timed FP64 steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    matvecs = iters = 0
    for k in range(args.steps):
        info = ctx.step(v, s, amp_at(step0 + args.warmup + k), opts=opts64)
        matvecs += info["matvecs"]
        iters += info["iterations"]
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    log(f"FP64: {args.steps} steps in {t64:.3f}s, {iters / args.steps:.1f} GMRES it/step, "
        f"{matvecs / args.steps:.1f} matvecs/step")
    v64 = v.clone()

    # ---- the chosen path: FP32 operator inside FP64 iterative refinement
    v.copy_(v_save)
    s.copy_(s_save)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it32 = mv32 = 0
    for k in range(args.steps):
        info = ctx.step(v, s, amp_at(step0 + args.warmup + k), opts=opts32)
        it32 += info["iterations"]
        mv32 += info["matvecs"]
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    err32 = float((v - v64).norm() / max(float(v64.norm()), 1e-300))
    log(f"FP32+IR: {args.steps} steps in {t32:.3f}s, {it32 / args.steps:.1f} inner it/step, "
        f"rel diff to FP64 {err32:.2e}")

    # ---- operator apply timing (HIP events on the launch stream)
    x = torch.randn(n, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    def time_applies(prec):
        for _ in range(20):
            ctx.apply(x, y, prec)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.applies):
            ctx.apply(x, y, prec)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1e3 / args.applies

    ta64 = time_applies(sdg.SDG_PREC_F64)
    ta32 = time_applies(sdg.SDG_PREC_F32)
    n_elem, n_face = sizes["n_elem"], sizes["n_face"]
    small = n_face * (16 + 16) + n_elem * 8
    balg64 = sizes["op_bytes_f64"] + 2 * n * 8 + small
    balg32 = sizes["op_bytes_f32"] + 2 * n * 8 + small
    ach = balg64 / ta64 / 1e9
    log(f"apply FP64 {ta64 * 1e6:.1f} us ({n / ta64 / 1e9:.2f} GDOF/s, {ach:.0f} GB/s algorithmic); "
        f"FP32 {ta32 * 1e6:.1f} us ({n / ta32 / 1e9:.2f} GDOF/s, {balg32 / ta32 / 1e9:.0f} GB/s)")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (cpu_baseline) ...")
        cpu = cpu_baseline()
        log(f"cpu_baseline {cpu['value']:.4f} GDOF/s")

    value = n * matvecs / t64 / 1e9
    out = {
        "metric": "velocity-matvec GDOF/s + s per implicit step to 1e-10 residual, FP64 vs chosen",
        "value": value,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t64 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D 64x64 jittered split square (8192 tris), p=3, p_gamma=3, layered "
                               "lognormal media, 10 Hz Ricker source, dt=2.5e-3, GMRES(30) to 1e-10",
                   "n_elem": n_elem, "velocity_dofs_per_slab": n, "parallelism": "single GPU"},
        "s_per_step": {"fp64": t64 / args.steps, "fp32_operator_fp64_refinement": t32 / args.steps},
        "iterations_per_step": {"fp64": iters / args.steps, "fp32_ir_inner": it32 / args.steps},
        "matvec_kernel": {"fp64_us": ta64 * 1e6, "fp64_gdofs": n / ta64 / 1e9,
                          "fp32_us": ta32 * 1e6, "fp32_gdofs": n / ta32 / 1e9},
        "fp32_ir_rel_diff_vs_fp64": err32,
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "velocity operator apply (face_kernel + elem_kernel), FP64",
                     "bytes_per_launch": balg64},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
