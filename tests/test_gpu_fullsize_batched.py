"""Batched right-hand sides and mesh batches at their benchmarked shapes,
against the oracle on the patch of each sampled element (its rows of the
velocity Schur complement and of the coupled slab system are those of the
patch of the element and its face neighbours, tests/patch.py):

  64 columns on the 2D space-time workload (64x64 jittered split square,
  8192 triangles, p = 3, p_gamma = 3), with the batched kernel the tuner
  picks (the matrix-core kernel);
  16 meshes of 512-16384 triangles (log-uniform sizes) in one mesh batch.

Apply: each sampled element's rows of each column (mesh) to 1e-11 relative
(FP32 operator 1e-5), 1e-12 over the sample.  Step: the stress rows of each
sampled element's faces exact (1e-11 of their own right-hand side), and the
element's momentum residual within the column's (mesh's) own global bound
rtol ||b|| (||b|| = ||A v|| (1 + rtol) of that column or mesh).
"""
import numpy as np
import pytest

import synth
from patch import Patch, face_codes

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _sample(ne, rng, k):
    return sorted({0, ne - 1, ne // 2, *rng.choice(ne, k, replace=False).tolist()})


def _check_rows(label, got_rows, ref_rows, tol_elem, tol_all):
    num = den = worst = 0.0
    for got, ref in zip(got_rows, ref_rows):
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        worst = max(worst, e)
        num += np.linalg.norm(got - ref) ** 2
        den += np.linalg.norm(ref) ** 2
    print(f"{label}: worst element {worst:.2e}, sample {np.sqrt(num / den):.2e}")
    assert worst <= tol_elem and np.sqrt(num / den) <= tol_all


def test_c4a_64_columns_apply_and_step_sampled_rows():
    import torch
    import paper_1802_04516_amd as sdg
    R = 64
    w = synth.workload("c2")
    mesh = w["mesh"]
    ctx = sdg.Context(0)
    sz = ctx.setup(mesh.xyz, mesh.elem, mesh.period, w["p"], w["p_gamma"], sdg.SDG_SCHEME_STDG, w["dt"],
                   w["lam"], w["mu"], w["rho"], sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND,
                   max_rhs=R)
    print(f"batched variant picked: {sz['op_bvariant']} (timings {sz['tune_us_batched']})")
    n, ne = sz["n_vel_slab"], mesh.n_elem
    rng = np.random.default_rng(4401)
    sample = _sample(ne, rng, 3)
    patches = {i: Patch(mesh, i, w["p"], w["p_gamma"], w["dt"], w["scheme"], w["lam"], w["mu"], w["rho"])
               for i in sample}
    S = {i: P.slab.schur() for i, P in patches.items()}
    v = rng.standard_normal(n * R)
    for prec, tol_e, tol_a in ((sdg.SDG_PREC_F64, 1e-11, 1e-12), (sdg.SDG_PREC_F32, 1e-5, 2e-6)):
        y = torch.empty(n * R, dtype=torch.float64, device="cuda")
        ctx.apply(_t(v), y, prec, n_rhs=R)
        torch.cuda.synchronize()
        yh = y.cpu().numpy().reshape(R, n)
        got, ref = [], []
        for r in range(R):
            for i, P in patches.items():
                ref.append(P.schur_row(v[r * n:(r + 1) * n], S[i]))
                got.append(yh[r].reshape(ne, -1)[i])
        _check_rows(f"C4a apply, {R} columns, precision {prec}", got, ref, tol_e, tol_a)
    # one batched step of all columns from seeded random states
    rtol = 1e-10
    v_old = rng.standard_normal(sz["n_vel_state"] * R)
    s_old = rng.standard_normal(sz["n_stress_state"] * R)
    vg, sg = _t(v_old), _t(s_old)
    v_slab = torch.empty(n * R, dtype=torch.float64, device="cuda")
    s_slab = torch.empty(sz["n_stress_slab"] * R, dtype=torch.float64, device="cuda")
    o = sdg.SolveOpts(sdg.SDG_SOLVER_GMRES, sdg.SDG_PREC_F64, rtol, 20000, 15, 5, 10, 1e-4, sdg.SDG_PRECOND_BLOCK)
    info = ctx.step(vg, sg, None, n_rhs=R, opts=o, v_slab=v_slab, sigma_slab=s_slab)
    assert info["converged"]
    Av = torch.empty_like(v_slab)
    ctx.apply(v_slab, Av, sdg.SDG_PREC_F64, n_rhs=R)
    torch.cuda.synchronize()
    vs, ss, Avh = v_slab.cpu().numpy(), s_slab.cpu().numpy(), Av.cpu().numpy()
    codes = face_codes(mesh.elem)
    nvs, nss, nsl = sz["n_vel_state"], sz["n_stress_state"], sz["n_stress_slab"]
    worst_face = worst_glob = 0.0
    for r in range(0, R, 7):
        b_norm = np.linalg.norm(Avh[r * n:(r + 1) * n]) * (1 + rtol)
        for i, P in patches.items():
            rv, bv, faces = P.coupled_residual(vs[r * n:(r + 1) * n], ss[r * nsl:(r + 1) * nsl],
                                               v_old[r * nvs:(r + 1) * nvs], s_old[r * nss:(r + 1) * nss], codes)
            worst_glob = max(worst_glob, np.linalg.norm(rv) / b_norm)
            for rs, bs in faces:
                worst_face = max(worst_face, np.linalg.norm(rs) / np.linalg.norm(bs))
    print(f"C4a step: {info['iterations']} iterations; worst sampled momentum residual {worst_glob:.2e} of its "
          f"column's ||b||, worst stress rows {worst_face:.2e}")
    assert worst_face <= 1e-11 and worst_glob <= rtol
    ctx.close()


def test_c4b_16_meshes_apply_and_step_sampled_rows():
    import torch
    import paper_1802_04516_amd as sdg
    batch = synth.ragged_meshes(16, seed=4002)
    meshes = [m for m, _ in batch]
    lam, mu, rho = (np.concatenate([mt[k] for _, mt in batch]) for k in range(3))
    p, pg, dt = 3, 3, 2.5e-3
    ctx = sdg.Context(0)
    sz = ctx.setup_batch([(m.xyz, m.elem) for m in meshes], p, pg, sdg.SDG_SCHEME_STDG, dt, lam, mu, rho,
                         sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND)
    eoff = np.concatenate([[0], np.cumsum([m.n_elem for m in meshes])])
    n = sz["n_vel_slab"]
    blk = n // int(eoff[-1])
    rng = np.random.default_rng(4402)
    patches = []  # (mesh index, local element, Patch)
    for q, (m, mt) in enumerate(batch):
        for i in sorted({0, int(rng.integers(m.n_elem))}):
            patches.append((q, i, Patch(m, i, p, pg, dt, "stdg", *mt)))
    S = [P.slab.schur() for _, _, P in patches]
    v = rng.standard_normal(n)
    for prec, tol_e, tol_a in ((sdg.SDG_PREC_F64, 1e-11, 1e-12), (sdg.SDG_PREC_F32, 1e-5, 2e-6)):
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        ctx.apply(_t(v), y, prec)
        torch.cuda.synchronize()
        yh = y.cpu().numpy()
        got, ref = [], []
        for (q, i, P), Sq in zip(patches, S):
            vq = v[eoff[q] * blk:eoff[q + 1] * blk]
            ref.append(P.schur_row(vq, Sq))
            got.append(yh[(eoff[q] + i) * blk:(eoff[q] + i + 1) * blk])
        _check_rows(f"C4b apply, 16 meshes ({eoff[-1]} triangles), precision {prec}", got, ref, tol_e, tol_a)
    # one step of the batch (FP64, and FP32 operator + FP64 refinement)
    rtol = 1e-10
    nvs = sz["n_vel_state"] // int(eoff[-1])
    fcount = [len(face_codes(m.elem)) for m in meshes]
    foff = np.concatenate([[0], np.cumsum(fcount)])
    v_old = rng.standard_normal(sz["n_vel_state"])
    s_old = rng.standard_normal(sz["n_stress_state"])
    nsig_psi = sz["n_stress_state"] // int(foff[-1])
    for precision in (sdg.SDG_PREC_F64, sdg.SDG_PREC_F32):
        vg, sg = _t(v_old), _t(s_old)
        v_slab = torch.empty(n, dtype=torch.float64, device="cuda")
        s_slab = torch.empty(sz["n_stress_slab"], dtype=torch.float64, device="cuda")
        o = sdg.SolveOpts(sdg.SDG_SOLVER_GMRES, precision, rtol, 20000, 15, 5, 10, 2e-5, sdg.SDG_PRECOND_BLOCK)
        info = ctx.step(vg, sg, None, opts=o, v_slab=v_slab, sigma_slab=s_slab)
        assert info["converged"]
        Av = torch.empty_like(v_slab)
        ctx.apply(v_slab, Av, sdg.SDG_PREC_F64)
        torch.cuda.synchronize()
        vs, ss, Avh = v_slab.cpu().numpy(), s_slab.cpu().numpy(), Av.cpu().numpy()
        worst_face = worst_glob = 0.0
        for q, i, P in patches:
            m = meshes[q]
            e0, e1, f0, f1 = eoff[q], eoff[q + 1], foff[q], foff[q + 1]
            b_norm = np.linalg.norm(Avh[e0 * blk:e1 * blk]) * (1 + rtol)
            slab_f = (pg + 1) * nsig_psi  # stress slab values per face
            rv, bv, faces = P.coupled_residual(vs[e0 * blk:e1 * blk], ss[f0 * slab_f:f1 * slab_f],
                                               v_old[e0 * nvs:e1 * nvs], s_old[f0 * nsig_psi:f1 * nsig_psi],
                                               face_codes(m.elem))
            worst_glob = max(worst_glob, np.linalg.norm(rv) / b_norm)
            for rs, bs in faces:
                worst_face = max(worst_face, np.linalg.norm(rs) / np.linalg.norm(bs))
        print(f"C4b step precision {precision}: {info['iterations']} iterations; worst sampled momentum residual "
              f"{worst_glob:.2e} of its mesh's ||b||, worst stress rows {worst_face:.2e}")
        assert worst_face <= 1e-11 and worst_glob <= rtol
    ctx.close()
