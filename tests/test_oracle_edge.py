"""Oracle pins on the degenerate cases of the two-site product (Sec. II.A,
the Hamiltonian of Eq. Hamiltonian projected on the two-site space and
restricted to one U(1)xU(1) sector).

Each case has a closed form independent of the block algebra:
  * no electrons: every term of H holds an annihilator, so H_eff = 0;
  * every spin-orbital filled: one determinant, whose energy is the
    closed-shell expression 2 sum_i h_ii + sum_ij [2 (ii|jj) - (ij|ji)];
  * one electron: H acts on the one-electron sector as h alone, so with
    0/1 determinant isometries H_eff is the submatrix of h on the orbitals
    the basis keeps, and with orthonormal random isometries (a compression
    of h) its spectrum interlaces that of h (Cauchy).
"""
import numpy as np
import pytest

from paper_2501_18263_amd import synth
from oracle import block


def _explicit(p, terms):
    n = synth.psi_size(p)
    return np.stack([block.apply(p, terms, np.eye(n)[j]) for j in range(n)], axis=1)


def test_vacuum_is_annihilated():
    p = synth.make_problem(6, 16, 7, n_up=0, n_dn=0)
    assert synth.psi_size(p) == 1
    y = block.apply(p, block.heff_terms(p), np.array([0.7]))
    assert np.abs(y).max() == 0.0


@pytest.mark.parametrize("N,seed", [(6, 7), (7, 8)])
def test_full_filling_is_closed_shell_energy(N, seed):
    p = synth.make_problem(N, 16, seed, n_up=N, n_dn=N)
    assert synth.psi_size(p) == 1
    h, V = p.h, p.V
    e = 2.0 * np.trace(h) + 2.0 * np.einsum("iijj->", V) - np.einsum("ijji->", V)
    y = block.apply(p, block.heff_terms(p), np.array([1.0]))
    assert abs(y[0] - e) <= 1e-12 * abs(e)


@pytest.mark.parametrize("N,n_up,n_dn", [(7, 1, 0), (8, 0, 1)])
def test_one_electron_det_basis_is_h_submatrix(N, n_up, n_dn):
    from oracle import detbasis
    p = synth.make_problem(N, 64, 9, n_up=n_up, n_dn=n_dn, iso_kind="det")
    H = _explicit(p, block.heff_terms(p))
    dets = detbasis.psi_determinants(p)
    assert np.all(dets[:, 1] == 0)
    orb = [int(d).bit_length() - 1 for d in dets[:, 0]]
    assert all(int(d) & (int(d) - 1) == 0 for d in dets[:, 0])     # one bit each
    orb = np.array(orb) // 2
    assert len(set(orb.tolist())) == len(orb)
    assert np.abs(H - p.h[np.ix_(orb, orb)]).max() <= 1e-13


@pytest.mark.parametrize("N,n_up,n_dn", [(7, 1, 0), (8, 0, 1)])
def test_one_electron_spectrum_interlaces_h(N, n_up, n_dn):
    p = synth.make_problem(N, 64, 9, n_up=n_up, n_dn=n_dn)
    m = synth.psi_size(p)
    assert 1 < m < N                       # the kept space is a compression
    H = _explicit(p, block.heff_terms(p))
    assert np.abs(H - H.T).max() <= 1e-13
    mu = np.linalg.eigvalsh(0.5 * (H + H.T))
    lam = np.linalg.eigvalsh(p.h)
    for k in range(m):
        assert lam[k] - 1e-12 <= mu[k] <= lam[k + N - m] + 1e-12
