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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_traffic.json")


def kernel_source_hash():
    """Hash of the operator kernel sources the traffic counters describe."""
    import hashlib
    h = hashlib.sha256()
    for name in ("op_kernels.inc", "shapes.hpp"):
        with open(os.path.join(ROOT, "paper_1802_04516_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, variant):
    """HBM bytes per operator apply (face + element kernel) from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs recorded in profiles/, scaled by
    the same counters' readings for a plain copy; None when the kernels have
    changed since the counters were taken or no record exists."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    wl = rec.get(workload, {})
    v = wl.get("variants", {}).get(str(variant))
    e = wl.get("elem")
    if v is None or e is None:
        return None
    ff, wf = rec["copy_calibration"]["fetch_factor"], rec["copy_calibration"]["write_factor"]
    kib = (v["fetch_kib"] + e["fetch_kib"]) * ff + (v["write_kib"] + e["write_kib"]) * wf
    return kib * 1024.0


def apply_probe(args):
    """Operator applies only (for counter runs under rocprofv3)."""
    import torch

    import paper_1802_04516_amd as sdg
    import synth
    if args.variant >= 0:
        os.environ["SDG_OP_VARIANT"] = str(args.variant)
    w = synth.workload(args.workload)
    m = w["mesh"]
    sch = sdg.SDG_SCHEME_CN if w["scheme"] == "cn" else sdg.SDG_SCHEME_STDG
    prec = sdg.SDG_PREC_F64 if args.prec == "f64" else sdg.SDG_PREC_F32
    ctx = sdg.Context(0)
    sz = ctx.setup(m.xyz, m.elem, m.period, w["p"], w["p_gamma"], sch, w["dt"], w["lam"], w["mu"], w["rho"], prec)
    n = sz["n_vel_slab"]
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    ctx.apply(x, y, prec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.reps):
        ctx.apply(x, y, prec)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / args.reps
    print(json.dumps({"workload": args.workload, "variant": sz["op_variant"] if prec == sdg.SDG_PREC_F64
                      else sz["op_variant_f32"], "precision": args.prec, "apply_us": t * 1e6}), flush=True)
    ctx.close()


# GMRES restart length of every benchmarked solve: with the delayed
# reorthogonalisation each Arnoldi step sweeps the basis twice, and on C2 a
# sweep over restart lengths 10..32 gave 12.3 ms/step at 10-15 against
# 13.6 ms/step at 30 (149 against 144 iterations at 15).
GMRES_RESTART = 15
# Relative tolerance of each inner FP32 solve of the FP32 operator + FP64
# refinement path.  Two refinement sweeps reach 1e-10; a sweep on C2
# (restart 15, 20 steps) gave 12.7 / 14.3 / 13.3 / 10.5 / 11.2 / 12.1 /
# 12.7 / 13.8 ms/step for 3e-4 / 1e-4 / 3e-5 / 2e-5 / 1e-5 / 5e-6 / 3e-6 /
# 1e-6 against 11.6 ms/step for FP64.  The batched and 3D runs keep 1e-4
# (64 batched sources took 0.78 s/step at 1e-4 and 0.93 s/step at 2e-5).
IR_INNER_RTOL = 2e-5
# The same sweep on the 3D Crank-Nicolson workload (CG, 10 steps from the
# plane S-wave): 30.4 / 29.2 / 29.4 / 36.4 / 38.9 ms/step for 1e-4 / 3e-5 /
# 1e-5 / 3e-6 / 1e-6 (below about 3e-6 the FP32 inner CG stagnates), against
# 30.0 ms/step for FP64.
IR_INNER_RTOL_3D = 3e-5


def _solve_opts(sdg, precision, pc, flags=0, solver=None):
    o = sdg.SolveOpts(solver if solver is not None else sdg.SDG_SOLVER_AUTO, precision, 1e-10, 5000,
                      GMRES_RESTART, 5, 10, 1e-4, pc)
    o.flags = flags
    return o


def bench_batched(args, t_single_fp64):
    """64 Ricker point sources at seeded random positions (seed 4001) on the
    workload's mesh and material, one right-hand side each, solved in one
    batched step (shared launches, per-column GMRES)."""
    import numpy as np
    import torch

    import paper_1802_04516_amd as sdg
    import synth
    R = 64
    w = synth.workload("c2")
    mesh = w["mesh"]
    ctx = sdg.Context(0)
    sizes = ctx.setup(mesh.xyz, mesh.elem, mesh.period, w["p"], w["p_gamma"], sdg.SDG_SCHEME_STDG, w["dt"],
                      w["lam"], w["mu"], w["rho"],
                      sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND, max_rhs=R)
    pos = np.random.default_rng(4001).uniform(0.05, 0.95, size=(R, 2))
    ctx.set_sources(pos, np.tile([[0.0, 1.0]], (R, 1)))
    tau = np.array(sizes["tau"])
    dt = w["dt"]
    step0 = int(0.05 / dt)

    def amps(k):
        t = (step0 + k) * dt + tau * dt
        return np.tile(synth.ricker(t, 10.0, 0.1)[None, :], (R, 1)).ravel()

    n = sizes["n_vel_slab"]
    res = {"n_rhs": R, "velocity_dofs": n * R}
    for name, prec in (("fp64", sdg.SDG_PREC_F64), ("fp32_operator_fp64_refinement", sdg.SDG_PREC_F32)):
        v = torch.zeros(sizes["n_vel_state"] * R, dtype=torch.float64, device="cuda")
        s = torch.zeros(sizes["n_stress_state"] * R, dtype=torch.float64, device="cuda")
        o = _solve_opts(sdg, prec, sdg.SDG_PRECOND_BLOCK)
        ctx.step(v, s, amps(0), n_rhs=R, opts=o)
        torch.cuda.synchronize()
        steps = 2
        t0 = time.perf_counter()
        mv = it = 0
        for k in range(steps):
            info = ctx.step(v, s, amps(1 + k), n_rhs=R, opts=o)
            mv += info["matvecs"]
            it += info["iterations"]
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        res[name] = {"s_per_step": t, "s_per_step_per_rhs": t / R, "iterations_per_step": it / steps,
                     "gdofs": n * R * (mv / steps) / t / 1e9}
        log(f"batched {R} sources {name}: {t * 1e3:.1f} ms/step ({t / R * 1e3:.2f} ms per source), {it / steps:.0f} it")
    x = torch.randn(n * R, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for prec, key in ((sdg.SDG_PREC_F64, "apply_fp64_us"), (sdg.SDG_PREC_F32, "apply_fp32_us")):
        for _ in range(3):
            ctx.apply(x, y, prec, n_rhs=R)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            ctx.apply(x, y, prec, n_rhs=R)
        e1.record()
        e1.synchronize()
        res[key] = e0.elapsed_time(e1) * 1e3 / 10
    res["single_rhs_fp64_s_per_step"] = t_single_fp64
    res["speedup_vs_64_single_fp64_steps"] = R * t_single_fp64 / res["fp64"]["s_per_step"]
    log(f"batched apply FP64 {res['apply_fp64_us']:.0f} us, FP32 {res['apply_fp32_us']:.0f} us for {R} columns")
    ctx.close()
    return res


def bench_mesh_batch(args):
    """16 meshes with log-uniform sizes in [512, 16384] triangles (seed
    4002), jitter seeds 4100+k, layered lognormal media seeds 4200+k, one
    Ricker source each, one step of all meshes (HIP graphs and eager)."""
    import math

    import numpy as np
    import torch

    import paper_1802_04516_amd as sdg
    import synth
    rng = np.random.default_rng(4002)
    meshes, mats = [], []
    for k in range(16):
        Nk = math.exp(rng.uniform(math.log(512), math.log(16384)))
        nx = max(1, round(math.sqrt(Nk / 2)))
        ny = max(1, round(Nk / (2 * nx)))
        m = synth.split_square(nx, ny, jitter=0.2, seed=4100 + k)
        meshes.append(m)
        mats.append(synth.layered_material(m.centroids(), sigma=0.1, seed=4200 + k))
    lam, mu, rho = (np.concatenate([mt[i] for mt in mats]) for i in range(3))
    ctx = sdg.Context(0)
    dt = 2.5e-3
    sizes = ctx.setup_batch([(m.xyz, m.elem) for m in meshes], 3, 3, sdg.SDG_SCHEME_STDG, dt, lam, mu, rho,
                            sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND)
    ctx.set_mesh_sources(np.tile([[0.503, 0.497]], (16, 1)), np.tile([[0.0, 1.0]], (16, 1)),
                         np.arange(16, dtype=np.int32))
    tau = np.array(sizes["tau"])
    step0 = int(0.05 / dt)

    def amps(k):
        t = (step0 + k) * dt + tau * dt
        return np.tile(synth.ricker(t, 10.0, 0.1)[None, :], (16, 1)).ravel()

    res = {"n_mesh": 16, "elements": [m.n_elem for m in meshes], "velocity_dofs": sizes["n_vel_slab"]}
    for name, flags in (("fp64_hip_graph", sdg.SDG_SOLVE_GRAPH), ("fp64_eager", 0)):
        v = torch.zeros(sizes["n_vel_state"], dtype=torch.float64, device="cuda")
        s = torch.zeros(sizes["n_stress_state"], dtype=torch.float64, device="cuda")
        o = _solve_opts(sdg, sdg.SDG_PREC_F64, sdg.SDG_PRECOND_BLOCK, flags, sdg.SDG_SOLVER_GMRES)
        ctx.step(v, s, amps(0), opts=o)  # warm-up (records the graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.step(v, s, amps(1), opts=o)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res[name] = {"s_per_step": t, "iterations": info["iterations"], "matvecs": info["matvecs"],
                     "gdofs": sizes["n_vel_slab"] * info["matvecs"] / t / 1e9}
        log(f"mesh batch 16 ({sizes['n_elem']} elems) {name}: {t * 1e3:.1f} ms/step, {info['iterations']} it")
    ctx.close()
    return res


def nodal_points(mesh, p):
    """Physical coordinates of the velocity nodes, (n_elem, N_phi, dim), in
    the library's node order (equispaced nodes (i, j[, k]) / p, i fastest)."""
    import numpy as np
    V = mesh.unwrapped_vertices()
    d = V.shape[2]
    if d == 2:
        ref = [(i / p, j / p) for j in range(p + 1) for i in range(p + 1 - j)]
    else:
        ref = [(i / p, j / p, k / p) for k in range(p + 1) for j in range(p + 1 - k) for i in range(p + 1 - k - j)]
    ref = np.array(ref)
    E = V[:, 1:, :] - V[:, :1, :]                       # (n_elem, d, d): edge vectors
    return V[:, :1, :] + np.einsum("nl,eld->end", ref, E)


def bench_3d_operator(args):
    """3D operator on the 32^3 periodic Kuhn cube (196,608 tetrahedra, p=2,
    Crank-Nicolson, homogeneous): the stored blocks (about 2 GB FP64) exceed
    the last-level cache, so this apply runs from HBM.  Then the workload's 50
    implicit steps (preconditioned CG to 1e-10) from a plane S-wave velocity, FP64 and
    FP32 operator + FP64 refinement, with the energy drift (the scheme
    conserves energy exactly in this setting, Section 5)."""
    import numpy as np
    import torch

    import paper_1802_04516_amd as sdg
    import synth
    w = synth.workload("c3")
    mesh = w["mesh"]
    t0 = time.time()
    ctx = sdg.Context(0)
    sizes = ctx.setup(mesh.xyz, mesh.elem, mesh.period, 2, 0, sdg.SDG_SCHEME_CN, w["dt"], w["lam"], w["mu"],
                      w["rho"], sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND)
    log(f"3D setup {time.time() - t0:.1f}s: {sizes['n_elem']} tets, operator {sizes['op_bytes_f64'] / 1e9:.2f} GB; "
        f"autotune f64 {[round(x, 1) for x in sizes['tune_us_f64']]} -> {sizes['op_variant']}")
    n = sizes["n_vel_slab"]
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    res = {"elements": sizes["n_elem"], "velocity_dofs": n, "operator_bytes_f64": sizes["op_bytes_f64"],
           "face_kernel_variant": sizes["op_variant"]}
    for prec, key, ob in ((sdg.SDG_PREC_F64, "fp64", sizes["op_bytes_f64"]),
                          (sdg.SDG_PREC_F32, "fp32", sizes["op_bytes_f32"])):
        for _ in range(3):
            ctx.apply(x, y, prec)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        reps = 20
        for _ in range(reps):
            ctx.apply(x, y, prec)
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / reps
        b_alg = ob + 2 * n * 8 + sizes["n_face"] * 32 + sizes["n_elem"] * 8
        res[key] = {"apply_us": t * 1e6, "gdofs": n / t / 1e9, "algorithmic_gbs": b_alg / t / 1e9,
                    "hbm_frac": b_alg / t / 1e9 / HBM_PEAK_GBS}
        log(f"3D apply {key}: {t * 1e6:.0f} us, {n / t / 1e9:.2f} GDOF/s, {b_alg / t / 1e9:.0f} GB/s "
            f"({100 * b_alg / t / 1e9 / HBM_PEAK_GBS:.1f}% of HBM peak)")
    res["traffic_per_apply_bytes"] = measured_traffic("c3", sizes["op_variant"])

    # plane S-wave velocity: direction (1,1,1)/sqrt(3), polarisation (1,-1,0)/sqrt(2), alpha 0.1, c_s 1
    X = nodal_points(mesh, 2)                                # (n_elem, N_phi, 3)
    pol = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
    phase = 2.0 * np.pi * X.sum(axis=2)                      # k.x with k = 2 pi (1, 1, 1)
    v0 = 0.1 * pol[None, :, None] * np.sin(phase)[:, None, :]  # (n_elem, 3, N_phi)
    steps = w["steps"]  # 50
    for name, prec in (("fp64_steps", sdg.SDG_PREC_F64), ("fp32_operator_fp64_refinement_steps", sdg.SDG_PREC_F32)):
        v = torch.tensor(np.ascontiguousarray(v0).ravel(), dtype=torch.float64, device="cuda")
        s = torch.zeros(sizes["n_stress_state"], dtype=torch.float64, device="cuda")
        opts = _solve_opts(sdg, prec, sdg.SDG_PRECOND_BLOCK)
        if prec == sdg.SDG_PREC_F32:
            opts.inner_rtol = IR_INNER_RTOL_3D
        E0 = ctx.energy(v, s)
        drift = 0.0
        its = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = ctx.step(v, s, None, opts=opts)
            its += info["iterations"]
            drift = max(drift, abs(ctx.energy(v, s) - E0) / E0)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        res[name] = {"s_per_step": t, "iterations_per_step": its / steps, "max_rel_energy_drift": drift,
                     "note": "wall time includes one energy evaluation per step"}
        log(f"3D Crank-Nicolson {name}: {t * 1e3:.1f} ms/step, {its / steps:.1f} CG it/step, "
            f"energy drift {drift:.2e}")
    fast = min(("fp64_steps", "fp32_operator_fp64_refinement_steps"), key=lambda k: res[k]["s_per_step"])
    res["chosen"] = {"path": fast, "s_per_step": res[fast]["s_per_step"]}
    ctx.close()
    return res

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--applies", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precond", default="block", choices=["none", "mass", "block"])
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched (64 sources), mesh-batch (16 meshes) and 3D operator measurements")
    ap.add_argument("--apply-probe", action="store_true",
                    help="only run --reps operator applies of --workload (c2 or c3) with face-kernel --variant "
                         "(-1: autotuned) in --prec, for rocprofv3 counter runs")
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32"])
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
    if args.apply_probe:
        apply_probe(args)
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
    log(f"face-kernel autotune (us/apply, variants 0..7): f64 {[round(x, 1) for x in sizes['tune_us_f64']]} -> {sizes['op_variant']}, "
        f"f32 {[round(x, 1) for x in sizes['tune_us_f32']]} -> {sizes['op_variant_f32']}")
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
    opts64 = sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F64, 1e-10, 5000, GMRES_RESTART, 5, 10, 1e-4, pc)
    opts32 = sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F32, 1e-10, 5000, GMRES_RESTART, 5, 10, IR_INNER_RTOL,
                           pc)

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

    # ---- FP64 steps with the extrapolated initial guess
    v.copy_(v_save)
    s.copy_(s_save)
    optsx = sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F64, 1e-10, 5000, GMRES_RESTART, 5, 10, 1e-4, pc)
    optsx.flags = sdg.SDG_SOLVE_EXTRAPOLATE
    ctx.step(v, s, amp_at(step0 + args.warmup - 1), opts=optsx)  # seeds the previous slab
    v.copy_(v_save)
    s.copy_(s_save)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    itx = 0
    for k in range(args.steps):
        info = ctx.step(v, s, amp_at(step0 + args.warmup + k), opts=optsx)
        itx += info["iterations"]
    torch.cuda.synchronize()
    tx = time.perf_counter() - t0
    errx = float((v - v64).norm() / max(float(v64.norm()), 1e-300))
    log(f"FP64 extrapolated guess: {args.steps} steps in {tx:.3f}s, {itx / args.steps:.1f} it/step, "
        f"rel diff to FP64 {errx:.2e}")

    # ---- FP64 steps recorded in HIP graphs
    v.copy_(v_save)
    s.copy_(s_save)
    optsg = sdg.SolveOpts(sdg.SDG_SOLVER_GMRES, sdg.SDG_PREC_F64, 1e-10, 5000, GMRES_RESTART, 5, 10, 1e-4, pc)
    optsg.flags = sdg.SDG_SOLVE_GRAPH
    ctx.step(v, s, amp_at(step0 + args.warmup), opts=optsg)  # records the graphs
    v.copy_(v_save)
    s.copy_(s_save)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    itg = 0
    for k in range(args.steps):
        info = ctx.step(v, s, amp_at(step0 + args.warmup + k), opts=optsg)
        itg += info["iterations"]
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    errg = float((v - v64).norm() / max(float(v64.norm()), 1e-300))
    log(f"FP64 graph: {args.steps} steps in {tg:.3f}s, {itg / args.steps:.1f} it/step (full cycles), "
        f"rel diff to FP64 {errg:.2e}")

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
                               "lognormal media, 10 Hz Ricker source, dt=2.5e-3, GMRES(15) with the element "
                               "block preconditioner to 1e-10",
                   "n_elem": n_elem, "velocity_dofs_per_slab": n, "parallelism": "single GPU"},
        "s_per_step": {"fp64": t64 / args.steps, "fp32_operator_fp64_refinement": t32 / args.steps,
                       "fp64_hip_graph": tg / args.steps, "fp64_extrapolated_guess": tx / args.steps},
        "chosen": min(({"path": "fp64", "s_per_step": t64 / args.steps},
                       {"path": "fp32_operator_fp64_refinement", "s_per_step": t32 / args.steps}),
                      key=lambda d: d["s_per_step"]),
        "iterations_per_step": {"fp64": iters / args.steps, "fp32_ir_inner": it32 / args.steps,
                                "fp64_hip_graph": itg / args.steps, "fp64_extrapolated_guess": itx / args.steps},
        "fp64_extrapolated_rel_diff_vs_fp64": errx,
        "fp64_hip_graph_rel_diff_vs_fp64": errg,
        "matvec_kernel": {"fp64_us": ta64 * 1e6, "fp64_gdofs": n / ta64 / 1e9,
                          "fp32_us": ta32 * 1e6, "fp32_gdofs": n / ta32 / 1e9},
        "fp32_ir_rel_diff_vs_fp64": err32,
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS,
                     "traffic": measured_traffic("c2", sizes["op_variant"]),
                     "kernel": f"velocity operator apply (face kernel variant {sizes['op_variant']} + element "
                               f"kernel), FP64",
                     "bytes_per_launch": balg64},
        "cpu_baseline": cpu,
    }
    ctx.close()
    if not args.no_extras:
        out["batched_64_sources"] = bench_batched(args, t64 / args.steps)
        out["mesh_batch_16"] = bench_mesh_batch(args)
        out["operator_3d"] = bench_3d_operator(args)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
