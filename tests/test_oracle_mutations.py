"""Planted mistakes in the oracle, on the CPU: each plausible slip in the
block algebra of the two-site product (Sec. II.A, Eq. Hamiltonian, and
Sec. II.C) must make one of
the pins fail.  The pins used are the explicit projection P^T H P (O-DEF,
built from the determinant Hamiltonian, no code shared with the block
oracle) and the closed-shell energy of a completely filled problem.  A
mistake that every pin missed would leave the oracle unpinned there."""
import numpy as np
import pytest

from paper_2501_18263_amd import synth
from oracle import block, explicit


@pytest.fixture(scope="module")
def case():
    p = synth.make_problem(6, 16, 3)
    H = explicit.heff_dense(p)
    psi = synth.random_psi(p)
    return p, H @ psi, psi


def _err(p, y0, psi, terms):
    y = block.apply(p, terms, psi)
    return np.linalg.norm(y - y0) / np.linalg.norm(y0)


def _closed_shell_err(n=6, seed=7):
    p = synth.make_problem(n, 16, seed, n_up=n, n_dn=n)
    h, V = p.h, p.V
    e = 2.0 * np.trace(h) + 2.0 * np.einsum("iijj->", V) - np.einsum("ijji->", V)
    y = block.apply(p, block.heff_terms(p), np.array([1.0]))
    return abs(y[0] - e) / abs(e)


def test_unmutated_oracle_meets_the_pins(case):
    p, y0, psi = case
    assert _err(p, y0, psi, block.heff_terms(p)) <= 1e-12
    assert _closed_shell_err() <= 1e-12


def test_transposed_integral_index_is_caught(case, monkeypatch):
    # (pr|qs) read as (pq|rs): a transposed operand of the two-body term
    def g_bad(self, p_, q, r, s):
        if (p_ & 1) != (r & 1) or (q & 1) != (s & 1):
            return 0.0
        return self.V[p_ >> 1, q >> 1, r >> 1, s >> 1]
    monkeypatch.setattr(block.Integrals, "g", g_bad)
    p, y0, psi = case
    assert _err(p, y0, psi, block.heff_terms(p)) > 1e-3
    assert _closed_shell_err() > 1e-3


def test_lost_middle_site_parity_is_caught(case, monkeypatch):
    # the fermionic sign of an odd number of middle-site modes dropped
    monkeypatch.setattr(block, "_mu_par", lambda mu: 0)
    p, y0, psi = case
    assert _err(p, y0, psi, block.heff_terms(p)) > 1e-3


def test_dropped_or_sign_flipped_term_is_caught(case):
    p, y0, psi = case
    terms = block.heff_terms(p)
    # the term that contributes most to the product
    contrib = [np.linalg.norm(block.apply(p, [t], psi)) for t in terms]
    k = int(np.argmax(contrib))
    assert _err(p, y0, psi, terms[:k] + terms[k + 1:]) > 1e-3
    c, ell, mu, rho = terms[k]
    assert _err(p, y0, psi, terms[:k] + [(-c, ell, mu, rho)] + terms[k + 1:]) > 1e-3
    # and a term of median size: small slips are caught too
    m = int(np.argsort(contrib)[len(contrib) // 2])
    assert contrib[m] > 0
    assert _err(p, y0, psi, terms[:m] + terms[m + 1:]) > 1e-9


def test_one_body_spin_mixing_is_caught(case, monkeypatch):
    # spin selection rule of t_pq dropped (hopping between up and down modes)
    monkeypatch.setattr(block.Integrals, "t", lambda self, p_, q: self.h[p_ >> 1, q >> 1])
    p, y0, psi = case
    try:
        e = _err(p, y0, psi, block.heff_terms(p))
    except (KeyError, ValueError, AssertionError):
        return                              # rejected outright: caught
    assert e > 1e-3
