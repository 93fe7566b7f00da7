"""Pins of O-SWEEP (one left-to-right sweep step, Sec. II.A / Sec. IV.A)
against facts that do not depend on it:

* keeping every non-zero singular value loses nothing: the start vector
  represents the old state exactly, so its norm and its energy under the new
  pair's explicit H_eff equal the old ones;
* with truncation, the norm lost is the discarded weight (the sum of the
  squared discarded singular values, Eckart-Young);
* the new pair's block states are orthonormal (its H_eff spectrum interlaces
  the full-CI one from above);
* the block-sparse oracle O-BLOCK on the new pair equals its explicit
  P'^T H P' (the new problem is a valid two-site problem)."""
import numpy as np
import pytest

from paper_2501_18263_amd import synth
from oracle import block, explicit, fci, svd, sweep


def _energy(p, psi):
    H = explicit.heff_dense(p)
    return float(psi @ H @ psi) / float(psi @ psi)


@pytest.mark.parametrize("N,D,seed", [(8, 16, 1), (7, 12, 2)])
def test_lossless_step_keeps_the_state(N, D, seed):
    p = synth.make_problem(N, D, seed)
    psi = synth.random_psi(p)
    mats = svd.sector_matrices(p, psi)
    rank = sum(min(M.shape) for M, _, _ in mats.values())
    p2, psi2, sing, disc = sweep.sweep_right(p, psi, rank)
    assert p2.k0 == p.k0 + 1 and disc <= 1e-24
    assert abs(np.linalg.norm(psi2) - 1.0) <= 1e-12
    assert abs(_energy(p2, psi2) - _energy(p, psi)) <= 1e-11 * abs(_energy(p, psi))


@pytest.mark.parametrize("N,D,seed,keep", [(8, 16, 1, 10), (8, 32, 4, 20), (9, 24, 3, 16)])
def test_truncated_step_loses_the_discarded_weight(N, D, seed, keep):
    p = synth.make_problem(N, D, seed)
    psi = synth.random_psi(p)
    p2, psi2, sing, disc = sweep.sweep_right(p, psi, keep)
    assert disc > 1e-6
    assert abs(float(psi2 @ psi2) - (1.0 - disc)) <= 1e-12
    assert abs(float(sing @ sing) - (1.0 - disc)) <= 1e-12


def test_new_pair_is_a_valid_two_site_problem():
    p = synth.make_problem(8, 16, 1)
    psi = synth.random_psi(p)
    p2, psi2, _, _ = sweep.sweep_right(p, psi, 12)
    H2 = explicit.heff_dense(p2)
    w = np.linalg.eigvalsh(H2)
    Hf, _ = fci.hamiltonian(p2.h, p2.V, p2.n_up, p2.n_dn)
    wf = np.linalg.eigvalsh(Hf.toarray())
    assert np.all(w >= wf[: len(w)] - 1e-10)          # Cauchy interlacing
    x = synth.random_psi(p2, seed=17)
    y = block.apply(p2, block.heff_terms(p2), x)
    assert np.linalg.norm(y - H2 @ x) <= 1e-12 * np.linalg.norm(H2 @ x)
