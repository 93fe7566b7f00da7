"""Test infrastructure: reference (oracle) code.  Only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg may import it.

O-MODE: the mode optimization micro-iteration at the bond (k, k+1)
(Sec. II.B, Fig. ``microiter``).  After the two-site eigenvector is found,
the rotation u of the two orbitals k and k+1 (the identity except for the
2 x 2 block at rows and columns k, k+1) that minimizes the half-Renyi block
entropy S_1/2 = 2 ln Tr sqrt(rho) of the left part {0..k} is searched, one
SVD per trial; the state is then rotated and the integrals t, v are
transformed with it.

Conventions (a reading of the passage, which leaves them open):
* spin-independent real rotation, U = exp(theta (E_xy - E_yx)) on the
  orbital pair (x, y) = (k, k+1): U_xx = U_yy = cos theta, U_xy = sin theta,
  U_yx = -sin theta;
* the new orbitals are c'+_i = sum_a U_ai c+_a, so the integrals become
  h' = U^T h U, V'_ijkl = sum U_ai U_bj U_ck U_dl V_abcd (``grad.rotate``);
* the same physical state in the new orbitals has the Fock coefficients
  phi' = exp(-K) phi with K = sum_{ab} kappa_ab sum_s c+_as c_bs the
  many-body generator (exp(K) c+_p exp(-K) = sum_q c+_q [exp(kappa)]_qp),
  so <phi'|H(h', V')|phi'> = <phi|H(h, V)|phi>;
* the rotated two-site vector is psi' = P^T phi' with phi = P psi (the maps
  of O-DEF; the rotation acts on the middle sites only, so psi' lies in the
  same two-site space);
* the search: S_1/2 on 16 equally spaced angles of [-pi/2, pi/2) (S has
  period pi), then golden-section refinement on the bracket around the best
  grid angle to |bracket| < 1e-10.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import explicit, fci, grad, svd


def rotation(n, x, y, theta):
    """n x n orbital rotation of the pair (x, y)."""
    U = np.eye(n)
    c, s = math.cos(theta), math.sin(theta)
    U[x, x] = U[y, y] = c
    U[x, y] = s
    U[y, x] = -s
    return U


def _det_int(b):
    return int(b[0]) | (int(b[1]) << 64)


def _hop(det, a, b):
    """c+_a c_b |det> as (sign, new det) or None (modes are bit positions,
    Jordan-Wigner order = bit order)."""
    if not (det >> b) & 1:
        return None
    d1 = det & ~(1 << b)
    sign = -1 if bin(det & ((1 << b) - 1)).count("1") & 1 else 1
    if (d1 >> a) & 1:
        return None
    if bin(d1 & ((1 << a) - 1)).count("1") & 1:
        sign = -sign
    return sign, d1 | (1 << a)


def generator(n, basis, x, y):
    """K = sum_s (c+_xs c_ys - c+_ys c_xs) on the determinant basis (sparse)."""
    keys = [_det_int(b) for b in basis]
    index = {k: i for i, k in enumerate(keys)}
    rows, cols, vals = [], [], []
    for j, det in enumerate(keys):
        for sgm in (0, 1):
            mx, my = 2 * x + sgm, 2 * y + sgm
            for a, b, w in ((mx, my, 1.0), (my, mx, -1.0)):
                r = _hop(det, a, b)
                if r is None:
                    continue
                rows.append(index[r[1]])
                cols.append(j)
                vals.append(w * r[0])
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(keys), len(keys)))


def rotate_state(p, psi, theta, x=None):
    """psi' = P^T exp(-theta K) P psi for the pair (x, x+1), x = k0 by
    default."""
    x = p.k0 if x is None else x
    P, basis = explicit.projector(p)
    K = generator(p.n_orb, basis, x, x + 1)
    phi = spla.expm_multiply(-theta * K, P @ psi)
    return P.T @ phi


def entropies(p, psi):
    """(S_1/2, S_1) of the left part {0..k} from the singular values of psi
    over the enlarged-left sectors (O-SVD), for the normalized state."""
    s = []
    for M, _, _ in svd.sector_matrices(p, psi).values():
        s.extend(np.linalg.svd(M, compute_uv=False))
    s = np.array(s)
    s = s / np.linalg.norm(s)
    lam = s * s
    lam = lam[lam > 0]
    return 2.0 * math.log(float(np.sum(s))), float(-np.sum(lam * np.log(lam)))


def rotated_integrals(p, theta, x=None):
    x = p.k0 if x is None else x
    return grad.rotate(p.h, p.V, rotation(p.n_orb, x, x + 1, theta))


def optimize(p, psi, n_grid=16, tol=1e-10):
    """theta minimizing S_1/2 of the rotated state: grid, then golden
    section.  Returns (theta, S_1/2(theta), S_1/2(0))."""
    f = lambda t: entropies(p, rotate_state(p, psi, t))[0]
    grid = [-math.pi / 2 + math.pi * i / n_grid for i in range(n_grid)]
    vals = [f(t) for t in grid]
    i = int(np.argmin(vals))
    h = math.pi / n_grid
    a, b = grid[i] - h, grid[i] + h
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    while b - a > tol:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
    t = 0.5 * (a + b)
    st = f(t)
    if vals[i] < st:
        t, st = grid[i], vals[i]
    return t, st, f(0.0)
