"""Pins of the oracle's energy derivatives (orbital rotations, Sec. II.B)."""
import numpy as np
import pytest

from paper_2501_18263_amd import synth
from oracle import explicit, fci, grad


@pytest.fixture(scope="module")
def small():
    # N=6 with every sector kept: the two-site space is the whole Fock sector
    p = synth.make_problem(6, 400, 5)
    psi = np.random.default_rng(7).standard_normal(synth.psi_size(p))
    return p, psi


def test_kappa_gradient_matches_central_differences(small):
    p, psi = small
    phi = grad.state(p, psi)
    pairs = [(0, 1), (1, 4), (2, 5), (0, 5)]
    g = grad.kappa_gradient(p, psi, pairs)
    eps = 1e-5
    for (x, y), gxy in zip(pairs, g):
        K = grad.generator(p.n_orb, x, y)
        ep = grad.energy_rotated(p, psi, eps * K, phi=phi)
        em = grad.energy_rotated(p, psi, -eps * K, phi=phi)
        fd = (ep - em) / (2 * eps)
        assert abs(fd - gxy) <= 1e-7 * max(1.0, abs(gxy)), (x, y, fd, gxy)


def test_kappa_gradient_vanishes_at_the_ground_state(small):
    # generalized Brillouin: the exact ground state is stationary under all
    # orbital rotations
    p, _ = small
    P, basis = explicit.projector(p)
    assert P.shape[0] == P.shape[1]  # complete two-site space
    H, _ = fci.hamiltonian(p.h, p.V, p.n_up, p.n_dn, basis=basis)
    w, U = np.linalg.eigh(H.toarray())
    psi0 = P.T @ U[:, 0]
    pairs = [(x, y) for x in range(p.n_orb) for y in range(x + 1, p.n_orb)]
    g = grad.kappa_gradient(p, psi0, pairs)
    assert np.abs(g).max() <= 1e-9 * abs(w[0])


def test_one_body_gradient_is_the_generalized_fock_commutator(small):
    # with V = 0, g_xy = 2 (F_xy - F_yx) with F = h gamma
    p, psi = small
    n = p.n_orb
    p0 = synth.make_problem(6, 400, 5, h=p.h, V=np.zeros((n,) * 4))
    gam = grad.one_rdm(p0, psi)
    phi = grad.state(p0, psi)
    assert abs(np.trace(gam) - phi[0] @ phi[0] * (p.n_up + p.n_dn)) <= 1e-10 * np.trace(gam)
    F = p0.h @ gam
    pairs = [(x, y) for x in range(n) for y in range(x + 1, n)]
    g = grad.kappa_gradient(p0, psi, pairs)
    ref = np.array([2 * (F[x, y] - F[y, x]) for x, y in pairs])
    assert np.abs(g - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
