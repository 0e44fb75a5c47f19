"""Pins of the whole scheme against Table 1 (Section 6.2): the periodic P+S
plane-wave test on [-1.5, 1.5]^2, (lambda, mu, rho) = (2, 1, 1),
p = p_gamma, dt = 0.112 h, t_end = 3 sqrt(2) (twelve P periods).

The paper's unstructured meshes are not available; the oracle runs on
split-square meshes of the same element counts.  On those the error
constant depends on how the split diagonals lie against the wave vector
k = 2 pi (1, 1): diagonals along k ('/') give errors several times the
paper's, diagonals across k ('\\') several times smaller, and the paper's
unstructured mesh lies between the two.  The observed order between two
mesh levels does not depend on the orientation and matches Table 1's.

A wrong sign, time matrix, stiffness or wave speed gives errors of order one
(no convergence); a missing factor in the coupling changes the phase speed
and the errors by far more than the mesh orientation does; a dropped term in
a block or a wrong quadrature degree lowers the observed order.
"""
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import synth
from oracle import waves
from oracle.assemble import Blocks
from oracle.mesh import Topology
from oracle.slab import Slab

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_convergence.txt")
NAMES = ("u", "v", "sigma_xx", "sigma_yy", "sigma_xy")


def table1():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows[(int(f[0]), int(f[1]))] = np.array([float(x) for x in f[2:7]])
    return rows


def run_table1_case(args):
    """L2 errors (u, v, sigma_xx, sigma_yy, sigma_xy) at t_end of the Table 1
    setup on an n x n split square with the given diagonal, degree p."""
    n, p, diagonal = args
    m = synth.split_square(n, periodic=True, lo=(-1.5, -1.5), hi=(1.5, 1.5), diagonal=diagonal)
    lam, mu, rho = synth.homogeneous_material(m.n_elem)
    B = Blocks(Topology(m.xyz, m.elem, m.period), p, lam, mu, rho)
    h = np.sqrt(2 * 9.0 / m.n_elem)  # the h of a mesh of equal-area triangles
    tend = 3 * np.sqrt(2)
    nsteps = int(np.ceil(tend / (0.112 * h)))
    S = Slab(B, p, tend / nsteps, "stdg")
    wave = waves.PlaneWave2D(waves=("p", "s"))
    v, s = waves.project(B, wave, 0.0)
    for _ in range(nsteps):
        _, _, v, s = S.step(v, s)
    ev, es = waves.l2_errors(B, v, s, wave, tend)
    return np.concatenate([ev, es])


@pytest.mark.slow
def test_table1_p1_error_magnitudes():
    """p = 1 on 1800 triangles against the 1760-triangle row: each error
    within a factor 4.5 of the paper's."""
    ref = table1()[(1, 1760)]
    got = run_table1_case((30, 1, "/"))
    ratio = got / ref
    assert np.all(ratio < 4.5) and np.all(ratio > 1 / 4.5), (got, ref)


@pytest.mark.slow
def test_table1_p2_convergence_order_and_orientation_bracket():
    """p = p_gamma = 2 on 450 and 1800 triangles, both diagonal orientations.

    - Observed order log2(e_450 / e_1800) of every variable in [3.6, 4.2]
      for both orientations (Table 1's p = 2 orders between its 1760- and
      3960-triangle meshes are 3.5-4.0).
    - For every variable, the 1800-triangle errors of the two orientations
      bracket the paper's 1760-triangle value, and each lies within a factor
      12 of it (measured: '/' 1.2-7.4x, '\\' 0.09-0.39x).
    """
    cases = [(15, 2, "/"), (30, 2, "/"), (15, 2, "\\"), (30, 2, "\\")]
    with ProcessPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        e = dict(zip(cases, ex.map(run_table1_case, cases)))
    ref = table1()[(2, 1760)]
    for diag in ("/", "\\"):
        order = np.log2(e[(15, 2, diag)] / e[(30, 2, diag)])
        print(diag, "order", dict(zip(NAMES, np.round(order, 2))), "ratio to paper",
              dict(zip(NAMES, np.round(e[(30, 2, diag)] / ref, 3))))
        assert np.all(order >= 3.6) and np.all(order <= 4.2), (diag, order)
    along, across = e[(30, 2, "/")], e[(30, 2, "\\")]
    assert np.all(across < ref) and np.all(ref < along), (across, ref, along)
    assert np.all(along / ref < 12.0) and np.all(ref / across < 12.0), (across, ref, along)
