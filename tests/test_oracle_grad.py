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


@pytest.fixture(scope="module")
def small4():
    # N=4 with every sector kept (the whole Fock sector), random state
    p = synth.make_problem(4, 400, 3)
    psi = np.random.default_rng(5).standard_normal(synth.psi_size(p))
    return p, psi


def test_v_orbits_partition_the_index_space():
    n = 4
    orbs = grad.v_orbits(n)
    members = [q for o in orbs for q in o]
    assert len(members) == n ** 4 and len(set(members)) == n ** 4
    m = n * (n + 1) // 2
    assert len(orbs) == m * (m + 1) // 2   # distinct (ij|kl) of real integrals
    assert all(len(o) in (1, 2, 4, 8) for o in orbs)


def test_integral_gradient_euler_relation(small4):
    # E is linear (homogeneous of degree one) in the integrals
    p, psi = small4
    gh, gV = grad.integral_gradient(p, psi)
    e = grad.energy(p, psi)
    assert abs(np.sum(gh * p.h) + np.sum(gV * p.V) - e) <= 1e-10 * max(1.0, abs(e))


def test_integral_gradient_density_matrix_identities(small4):
    # trace gamma = N_e |Phi|^2; contracting the two-particle part over one
    # index pair gives (N_e - 1)/2 gamma (the state has N_e electrons);
    # gamma is symmetric positive semidefinite with eigenvalues <= 2 |Phi|^2
    p, psi = small4
    gh, gV = grad.integral_gradient(p, psi)
    phi, _ = grad.state(p, psi)
    nrm = float(phi @ phi)
    ne = p.n_up + p.n_dn
    assert abs(np.trace(gh) - ne * nrm) <= 1e-10 * ne * nrm
    assert np.allclose(gh, gh.T, atol=1e-12 * nrm)
    w = np.linalg.eigvalsh(gh)
    assert w.min() >= -1e-10 * nrm and w.max() <= 2 * nrm * (1 + 1e-10)
    contr = np.einsum("ijkk->ij", gV)
    assert np.abs(contr - 0.5 * (ne - 1) * gh).max() <= 1e-10 * nrm
    # the one-body part agrees with gamma read off at V = 0
    assert np.abs(gh - grad.one_rdm(p, psi)).max() <= 1e-10 * nrm
