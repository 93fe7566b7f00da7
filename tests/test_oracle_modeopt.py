"""Pins of O-MODE (the mode-optimization micro-iteration, Sec. II.B) and
of the library's host-side integral rotation:

* the rotated state under the rotated integrals has the old energy (the
  state rotation and the integral rotation are written independently, one
  from the many-body generator on determinants, one from the 2 x 2 orbital
  matrix; a wrong sign or index in either breaks the equality);
* rotations compose, angle 0 is the identity, the norm is kept;
* the angle search finds the minimum of a dense brute-force scan;
* heff_rotate_integrals (host code of the library, callable without a GPU)
  equals U^T h U and the four-index transform of V."""
import ctypes
import math
import os

import numpy as np
import pytest

from paper_2501_18263_amd import synth
from oracle import explicit, fci, grad, modeopt


@pytest.fixture(scope="module")
def case():
    p = synth.make_problem(8, 16, 1)
    return p, synth.random_psi(p)


def _energy_fock(p, psi, h, V):
    P, basis = explicit.projector(p)
    H, _ = fci.hamiltonian(h, V, p.n_up, p.n_dn, basis=basis)
    phi = P @ psi
    return float(phi @ (H @ phi))


@pytest.mark.parametrize("theta", [0.3, -1.1, math.pi / 2])
def test_rotated_state_under_rotated_integrals_keeps_the_energy(case, theta):
    p, psi = case
    ps = modeopt.rotate_state(p, psi, theta)
    h2, V2 = modeopt.rotated_integrals(p, theta)
    e0 = _energy_fock(p, psi, p.h, p.V)
    e1 = _energy_fock(p, ps, h2, V2)
    assert abs(e1 - e0) <= 1e-12 * abs(e0)
    # and the unrotated integrals do see a different energy (the check has teeth)
    assert abs(_energy_fock(p, ps, p.h, p.V) - e0) > 1e-6


def test_rotation_group_properties(case):
    p, psi = case
    a, b = 0.4, -0.9
    assert np.linalg.norm(modeopt.rotate_state(p, psi, 0.0) - psi) <= 1e-14
    two = modeopt.rotate_state(p, modeopt.rotate_state(p, psi, a), b)
    one = modeopt.rotate_state(p, psi, a + b)
    assert np.linalg.norm(two - one) <= 1e-12
    assert abs(np.linalg.norm(one) - 1.0) <= 1e-13


def test_angle_search_finds_the_brute_force_minimum(case):
    p, psi = case
    t, st, s0 = modeopt.optimize(p, psi)
    grid = np.linspace(-math.pi / 2, math.pi / 2, 361)
    brute = min(modeopt.entropies(p, modeopt.rotate_state(p, psi, g))[0] for g in grid)
    assert st <= brute + 1e-9 and st <= s0


def test_library_integral_rotation_matches_oracle():
    from paper_2501_18263_amd import heff
    rng = np.random.default_rng(3)
    n = 7
    h, V = synth.integrals(n, 11)
    for x, y, th in ((2, 3, 0.37), (0, 5, -1.2), (6, 1, 2.5)):
        U = np.eye(n)
        U[x, x] = U[y, y] = math.cos(th)
        U[x, y] = math.sin(th)
        U[y, x] = -math.sin(th)
        h_ref, V_ref = grad.rotate(h, V, U)
        h2, V2 = heff.rotate_integrals(h, V, x, y, th)
        assert np.abs(h2 - h_ref).max() <= 1e-13
        assert np.abs(V2 - V_ref).max() <= 1e-13
    with pytest.raises(heff.HeffError):
        heff.rotate_integrals(h, V, 2, 2, 0.1)
