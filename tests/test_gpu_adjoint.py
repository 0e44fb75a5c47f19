"""GPU discrete adjoint (receiver-misfit gradients with respect to the
per-element lambda, mu, rho) against the oracle's adjoint and against
central finite differences of the GPU forward map.

Tolerances: both sides solve the same slab systems, the oracle by sparse LU
and the GPU by Krylov iterations to a relative residual of 1e-13 in the
forward and adjoint sweeps.  One adjoint step (the adjoint of the old state
and the step's gradient increment) is held to 1e-11 relative L2, the
per-step bar; so are the forward seismograms.  The gradient is a sum of
per-step increments that partly cancel: each increment carries the per-step
error, so the sum's relative error is bounded by the per-step bar times the
amplification sum_n ||g_n|| / ||sum_n g_n||, which the oracle's increments
give; the bar is 1e-11 times that amplification.  Finite differences use a
relative step of 1e-6 with the 1e-6 relative bar of the method's target.
"""
import numpy as np
import pytest

import synth
from gpu_cases import rel
from oracle.adjoint import MisfitProblem
from oracle.assemble import Blocks
from oracle.mesh import Topology
from oracle.slab import Slab

pytestmark = pytest.mark.gpu

SRC = dict(pos=np.array([[0.41, 0.37]]), dir=np.array([[0.3, 1.0]]))
REC = np.array([[0.1, 0.9], [0.5, 0.95], [0.83, 0.71], [0.66, 0.2], [0.27, 0.52]])


def _amps(scheme, tau, dt, nsteps):
    tau = np.array([0.5]) if scheme == "cn" else np.asarray(tau)
    return np.array([synth.ricker((n + tau) * dt, 10.0, 0.02)[None, :] for n in range(nsteps)])


def _oracle(lam, mu, rho, mesh, p, pg, scheme, dt, nsteps, data=None):
    B = Blocks(Topology(mesh.xyz, mesh.elem, mesh.period), p, lam, mu, rho)
    S = Slab(B, pg, dt, scheme)
    amps = _amps(scheme, S.tb.tau, dt, nsteps)
    return MisfitProblem(S, REC, SRC, list(amps), data)


def _opts(rtol=1e-13, precond=None):
    import paper_1802_04516_amd as sdg
    return sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F64, rtol, 4000, 30, 5, 10, 1e-4,
                         sdg.SDG_PRECOND_MASS if precond is None else precond)


CASES = {
    # name: (n, p, p_gamma, scheme, dt, steps, checkpoint_every, preconditioner)
    "stdg_p2pg2": (5, 2, 2, "stdg", 0.01, 7, 3, "block"),
    "stdg_p1pg1_mass": (4, 1, 1, "stdg", 0.02, 5, 2, "mass"),
    "cn_p1": (5, 1, 0, "cn", 0.01, 6, 4, "mass"),
    # Crank-Nicolson with the explicit element block inverse (its transposed
    # application in the adjoint solves)
    "cn_p1_block": (5, 1, 0, "cn", 0.01, 6, 3, "block"),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def problem(request):
    import torch
    import paper_1802_04516_amd as sdg
    from paper_1802_04516_amd.adjoint import Seismograms
    n, p, pg, scheme, dt, nsteps, K, pc = CASES[request.param]
    mesh = synth.split_square(n, jitter=0.15, seed=3)
    lam, mu, rho = synth.lognormal_material(mesh.n_elem, sigma=0.2, seed=5)
    true = synth.lognormal_material(mesh.n_elem, sigma=0.2, seed=6)
    P_true = _oracle(*true, mesh, p, pg, scheme, dt, nsteps)
    S = P_true.S
    v0 = np.zeros((mesh.n_elem, S.d, S.nphi))
    s0 = np.zeros((S.nf, S.nsig, S.npsi))
    _, data, _, _ = P_true.forward(v0, s0, keep=False)
    P = _oracle(lam, mu, rho, mesh, p, pg, scheme, dt, nsteps, data)
    sim = Seismograms(mesh, p, pg, sdg.SDG_SCHEME_CN if scheme == "cn" else sdg.SDG_SCHEME_STDG, dt,
                      lam, mu, rho, SRC["pos"], SRC["dir"], _amps(scheme, S.tb.tau, dt, nsteps), REC,
                      checkpoint_every=K,
                      opts=_opts(precond=sdg.SDG_PRECOND_BLOCK if pc == "block" else sdg.SDG_PRECOND_MASS),
                      precisions=sdg.SDG_PREC_F64 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND)
    out = dict(name=request.param, mesh=mesh, lam=lam, mu=mu, rho=rho, P=P, v0=v0, s0=s0, data=data, sim=sim,
               data_t=torch.tensor(data, dtype=torch.float64, device="cuda"), nsteps=nsteps)
    yield out
    sim.close()


def _gpu_misfit_and_grad(pb, lam, mu, rho):
    import torch
    th = [torch.tensor(x, dtype=torch.float64, device="cuda", requires_grad=True) for x in (lam, mu, rho)]
    obs = pb["sim"](*th)
    J = ((obs - pb["data_t"]) ** 2).sum()
    J.backward()
    return float(J), obs.detach().cpu().numpy(), [t.grad.cpu().numpy() for t in th]


def test_forward_seismograms_match_oracle(problem):
    pb = problem
    _, obs_o, _, _ = pb["P"].forward(pb["v0"], pb["s0"], keep=False)
    obs, _ = pb["sim"].run(pb["lam"], pb["mu"], pb["rho"])
    err = rel(obs.cpu().numpy(), obs_o)
    print(f"{pb['name']}: seismogram rel err {err:.2e}")
    assert err <= 1e-11


def test_gradient_matches_oracle_adjoint(problem):
    pb = problem
    incs = []
    Jo, gl, gm, gr = pb["P"].gradient(pb["v0"], pb["s0"], increments=incs)
    J, _, (g_lam, g_mu, g_rho) = _gpu_misfit_and_grad(pb, pb["lam"], pb["mu"], pb["rho"])
    errs = (rel(g_lam, gl), rel(g_mu, gm), rel(g_rho, gr))
    amp = [sum(np.linalg.norm(inc[k]) for inc in incs) / np.linalg.norm(tot)
           for k, tot in enumerate((gl, gm, gr))]
    print(f"{pb['name']}: J {J:.6e} vs {Jo:.6e}; grad rel err lam {errs[0]:.2e} mu {errs[1]:.2e} "
          f"rho {errs[2]:.2e}; amplification of the per-step error {np.round(amp, 1)}")
    assert abs(J - Jo) <= 1e-11 * abs(Jo)
    for e, a in zip(errs, amp):
        assert e <= 1e-11 * max(1.0, a)


def test_gradient_matches_central_differences(problem):
    pb = problem
    sim = pb["sim"]
    theta = np.concatenate([pb["lam"], pb["mu"], pb["rho"]])
    _, _, g = _gpu_misfit_and_grad(pb, pb["lam"], pb["mu"], pb["rho"])
    g = np.concatenate(g)
    rng = np.random.default_rng(5003)
    ne = pb["mesh"].n_elem

    def J_of(th):
        obs, _ = sim.run(*np.split(th, 3))
        return float(((obs - pb["data_t"]) ** 2).sum())

    for _ in range(3):
        d = rng.standard_normal(3 * ne) * theta
        eps = 1e-6
        fd = (J_of(theta + eps * d) - J_of(theta - eps * d)) / (2 * eps)
        print(f"{pb['name']}: fd {fd:.10e} adjoint {g @ d:.10e}")
        assert abs(fd - g @ d) <= 1e-6 * abs(fd)
    sim.set_material(pb["lam"], pb["mu"], pb["rho"])


def test_checkpoint_interval_does_not_change_the_gradient(problem):
    """Recomputation is deterministic: every checkpoint interval gives the
    same gradient bit for bit."""
    import torch
    pb = problem
    sim = pb["sim"]
    K0 = sim.K
    try:
        res = []
        for K in (1, pb["nsteps"]):
            sim.K = K
            res.append(np.concatenate(_gpu_misfit_and_grad(pb, pb["lam"], pb["mu"], pb["rho"])[2]))
        sim.K = K0
        res.append(np.concatenate(_gpu_misfit_and_grad(pb, pb["lam"], pb["mu"], pb["rho"])[2]))
    finally:
        sim.K = K0
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[0], res[2])
    torch.cuda.synchronize()


def test_adjoint_step_argument_checks(problem):
    import torch
    import paper_1802_04516_amd as sdg
    ctx = problem["sim"].ctx
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    s = ctx.sizes
    with pytest.raises(ValueError):
        ctx.adjoint_step(z(s["n_vel_state"]), z(s["n_vel_slab"] + 1), z(s["n_vel_state"]),
                         z(s["n_stress_state"]), z(3 * s["n_elem"]))
    L = sdg.lib()
    assert L.sdg_adjoint_step(ctx.h, None, None, None, None, None, None, None, None) == sdg.SDG_EINVAL
    bad = _opts()
    bad.precision = sdg.SDG_PREC_F32
    with pytest.raises(sdg.SdgError) as ei:
        ctx.adjoint_step(z(s["n_vel_state"]), z(s["n_vel_slab"]), z(s["n_vel_state"]), z(s["n_stress_state"]),
                         z(3 * s["n_elem"]), opts=bad)
    assert ei.value.code == sdg.SDG_EUNSUPPORTED


STEP_CASES = {
    # name: (mesh, p, p_gamma, scheme, dt)
    "stdg_p2pg2": (lambda: synth.split_square(5, jitter=0.15, seed=3), 2, 2, "stdg", 0.01),
    "cn_p1": (lambda: synth.split_square(5, jitter=0.15, seed=3), 1, 0, "cn", 0.01),
    "stdg_3d_p1pg1": (lambda: synth.kuhn_cube(2, periodic=False), 1, 1, "stdg", 0.02),
}


@pytest.mark.parametrize("case", sorted(STEP_CASES))
def test_one_adjoint_step_matches_oracle(case):
    """One sdg_adjoint_step against the oracle's adjoint step from the same
    old state and adjoint of the new state (seeded random): the adjoint of
    the old state (velocity and canonical stress) and the step's gradient
    increment per element (lambda, mu, rho), each to 1e-11 relative L2.
    Each side runs its own forward step for the slab DOFs (GPU: Krylov to
    1e-13; oracle: sparse LU)."""
    import torch
    import paper_1802_04516_amd as sdg
    mk, p, pg, scheme, dt = STEP_CASES[case]
    mesh = mk()
    lam, mu, rho = synth.lognormal_material(mesh.n_elem, sigma=0.2, seed=15)
    B = Blocks(Topology(mesh.xyz, mesh.elem, mesh.period), p, lam, mu, rho)
    S = Slab(B, pg, dt, scheme)
    P = MisfitProblem(S, mesh.centroids()[:2])
    ctx = sdg.Context(0)
    sz = ctx.setup(mesh.xyz, mesh.elem, mesh.period, p, pg, sdg.SDG_SCHEME_CN if scheme == "cn" else sdg.SDG_SCHEME_STDG,
                   dt, lam, mu, rho, sdg.SDG_PREC_F64 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND)
    rng = np.random.default_rng(77)
    nf = B.topo.n_face
    Linv = [np.linalg.inv(B.L[j]) for j in range(nf)]
    v_old = rng.standard_normal((mesh.n_elem, B.dim, B.nphi))
    s_old = rng.standard_normal((nf, B.nsig, B.npsi))
    s_old_can = np.stack([B.to_canonical(j, s_old[j]) for j in range(nf)])
    vbar = rng.standard_normal((mesh.n_elem, B.dim, B.nphi))
    sbar_can = rng.standard_normal((nf, B.nsig, B.npsi))
    # the adjoint of canonical stress DOFs s_can = s_raw L is sbar_raw = sbar_can L^T
    sbar_raw = np.stack([sbar_can[j] @ B.L[j].T for j in range(nf)])
    # oracle: forward slab and one adjoint step
    X = S.solve(S.rhs(v_old, s_old))
    vb_o, sb_o, glj, gmj, gr_o = P.adjoint_step(v_old, s_old, X, vbar, sbar_raw)
    gl_o, gm_o = P.faces_to_elements(glj, gmj)
    sb_o_can = np.stack([sb_o[j] @ Linv[j].T for j in range(nf)])
    # GPU: forward step (slab output), then the adjoint step
    dev = dict(dtype=torch.float64, device="cuda")
    o = _opts(1e-13, sdg.SDG_PRECOND_BLOCK)
    vg, sg = torch.tensor(v_old.ravel(), **dev), torch.tensor(s_old_can.ravel(), **dev)
    v_slab = torch.empty(sz["n_vel_slab"], **dev)
    ctx.step(vg, sg, None, opts=o, v_slab=v_slab)
    vbg, sbg = torch.tensor(vbar.ravel(), **dev), torch.tensor(sbar_can.ravel(), **dev)
    grad = torch.zeros(3 * mesh.n_elem, **dev)
    ctx.adjoint_step(torch.tensor(v_old.ravel(), **dev), v_slab, vbg, sbg, grad, opts=o)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().reshape(3, -1)
    errs = {"vbar": rel(vbg.cpu().numpy(), vb_o), "sigma_bar": rel(sbg.cpu().numpy(), sb_o_can),
            "g_lambda": rel(g[0], gl_o), "g_mu": rel(g[1], gm_o), "g_rho": rel(g[2], gr_o)}
    print(f"{case}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= 1e-11, (k, v)
    ctx.close()
