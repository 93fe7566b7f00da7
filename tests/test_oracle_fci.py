"""Pins of the full-CI oracle (O-FCI) against values fixed independently of it."""
import json
import os

import numpy as np
import pytest

from oracle import fci

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_one_body_closed_form():
    # V = 0: the ground state fills the lowest orbital energies of h per spin.
    rng = np.random.default_rng(11)
    n = 6
    a = rng.standard_normal((n, n))
    h = (a + a.T) / 2
    V = np.zeros((n,) * 4)
    for n_up, n_dn in [(3, 3), (3, 2), (1, 4)]:
        e = fci.lowest(h, V, n_up, n_dn)[0]
        w = np.linalg.eigvalsh(h)
        assert abs(e - (w[:n_up].sum() + w[:n_dn].sum())) < 1e-12


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.7, 0.0), (1.3, 9.0)])
def test_hubbard_dimer(t, U):
    # two sites, one up and one down electron: E0 = U/2 - sqrt(U^2/4 + 4 t^2)
    h = np.array([[0.0, -t], [-t, 0.0]])
    V = np.zeros((2,) * 4)
    V[0, 0, 0, 0] = V[1, 1, 1, 1] = U
    e = fci.lowest(h, V, 1, 1)[0]
    assert abs(e - (U / 2 - np.sqrt(U * U / 4 + 4 * t * t))) < 1e-12


def spinless_torus(L=4, t=1.0, Vnn=1.0):
    """Spinless model of Eq. Spinless mapped on spin-up orbitals: one orbital
    per lattice site, h_ij = -t per nearest-neighbour bond and
    V n_i n_j = (1/2) sum over both orderings of (ii|jj) a+_i a+_j a_j a_i."""
    n = L * L
    h = np.zeros((n, n))
    V = np.zeros((n,) * 4)
    bonds = set()
    for x in range(L):
        for y in range(L):
            i = x * L + y
            for j in (((x + 1) % L) * L + y, x * L + (y + 1) % L):
                bonds.add((min(i, j), max(i, j)))
    for i, j in bonds:
        h[i, j] = h[j, i] = -t
        V[i, i, j, j] = V[j, j, i, i] = Vnn
    return h, V, len(bonds)


def test_spinless_torus_printed_energies():
    gold = json.load(open(os.path.join(GOLD, "spinless_4x4_torus.json")))
    h, V, nb = spinless_torus()
    assert nb == 32
    e = fci.lowest(h, V, gold["model"]["n_fermions"], 0, k=2)
    half_ulp = 0.5 * 10.0 ** (-gold["printed_decimals"])
    assert abs(e[0] - gold["printed"]["E_GS"]) <= half_ulp
    assert abs(e[1] - gold["printed"]["E_1"]) <= half_ulp


def test_apply_det_single_excitation_sign():
    # a+_{1 up} a_{0 up} on |0up 0dn> (modes 0,1): moves mode 0 to mode 2,
    # passing mode 1 (occupied) -> sign -1 by the Jordan-Wigner rule.
    n = 2
    h = np.zeros((n, n))
    h[1, 0] = h[0, 1] = 1.0
    V = np.zeros((n,) * 4)
    d = fci.det_from_occ([0], [0])
    dets, vals = fci.apply_det(h, V, d)
    got = {}
    for dd, v in zip(dets, vals):
        got[fci.det_to_int(dd)] = got.get(fci.det_to_int(dd), 0.0) + v
    assert got == {0b0110: -1.0, 0b1001: 1.0}
