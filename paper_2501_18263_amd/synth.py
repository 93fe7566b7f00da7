"""Seeded synthetic inputs for the two-site effective-Hamiltonian problem.

This module produces the *inputs* of the two-site DMRG step and nothing of
its arithmetic: the one- and two-electron integrals of the second-quantized
Hamiltonian (Sec. II.A, Eq. ``Hamiltonian``), the U(1)xU(1) sector tables of
every bond, the left-/right-canonical MPS isometries that define the
truncated block bases (Eq. ``DefinitionMPS``; Sec. II.C), the layout of the
two-site wavefunction Psi_{alpha,sigma_k,sigma_k+1,beta} and a random start
vector.  Both the CPU oracle and the GPU library consume what is generated
here; neither shares any other code.

Conventions (used identically by every consumer):

* Sites are 0-based, ``0..N-1``.  The two-site pair is ``(k0, k0+1)`` with
  ``k0 = N//2 - 1`` (the 1-based pair ``(N//2, N//2+1)``).  The left block
  L holds sites ``0..k0-1``, the right block R holds ``k0+2..N-1``.
* Site state index ``s = 0..3`` is ``(empty, down, up, up+down)`` with
  ``|up down> = c^dag_up c^dag_down |0>``.  Its label is ``(n_up, n_dn)``.
* A sector label is ``q = (n_up, n_dn)`` of the block it refers to (left
  sectors count the particles of L, right sectors those of R).  Sector
  lists are sorted lexicographically.
* Left isometry of site ``l`` maps ``(bond l) x (site l) -> bond l+1``; for
  every out-sector ``q`` its matrix has ``sum_s D_l(q - q(s))`` rows stacked
  in the order ``s = 0..3`` and ``D_{l+1}(q)`` orthonormal columns; it is
  stored row-major, out-sectors concatenated in sorted order.
* Right isometry of site ``j`` maps ``(site j) x (R block j+1..N-1)`` to the
  R block ``j..N-1`` with the same stacking rule (rows ordered by ``s`` of
  site ``j``, then by the old right-block state).
* The two-site vector is the concatenation, in the order
  ``(index of q_alpha, s_k, s_k1)``, of row-major blocks of shape
  ``D_L(q_alpha) x D_R(q_beta)`` with
  ``q_alpha + q(s_k) + q(s_k1) + q_beta = (n_up, n_dn)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SITE_Q = ((0, 0), (0, 1), (1, 0), (1, 1))


def _qadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def _qsub(a, b):
    return (a[0] - b[0], a[1] - b[1])


# --------------------------------------------------------------------------
# integrals
# --------------------------------------------------------------------------
def integrals(n_orb: int, seed: int):
    """One- and two-electron integrals of the synthetic Hamiltonian.

    ``h_ij = N(0,1) exp(-|i-j|/2)`` mirrored from the upper triangle, with
    ``h_ii -= 2 i / N`` (1-based ``i``); ``V_ijkl = (ij|kl) = sum_{P<16}
    B^P_ij B^P_kl`` with ``B^P`` symmetric ``N(0,0.3^2) exp(-|i-j|/3)``.
    Draw order: the N x N matrix for h, then B^0..B^15.
    """
    n = n_orb
    rng = np.random.default_rng(seed)
    idx = np.arange(n)
    dist = np.abs(idx[:, None] - idx[None, :])
    a = rng.standard_normal((n, n))
    h = np.triu(a) + np.triu(a, 1).T
    h = h * np.exp(-dist / 2.0)
    h[idx, idx] -= 2.0 * (idx + 1) / n
    bs = []
    for _ in range(16):
        b = rng.standard_normal((n, n)) * 0.3
        b = np.triu(b) + np.triu(b, 1).T
        bs.append(b * np.exp(-dist / 3.0))
    bmat = np.stack(bs).reshape(16, n * n)
    v = (bmat.T @ bmat).reshape(n, n, n, n)
    return np.ascontiguousarray(h), np.ascontiguousarray(v)


# --------------------------------------------------------------------------
# sector tables
# --------------------------------------------------------------------------
def _waterfill(cands, d_max):
    """cands: list of (q, cap, weight).  Returns {q: dim} with sum == d_max
    (or all caps when they fit), dims <= cap, zero dims dropped."""
    caps = {q: c for q, c, _ in cands}
    tot = sum(caps.values())
    if tot <= d_max:
        return {q: c for q, c in caps.items() if c > 0}
    ws = {q: w for q, _, w in cands}
    lo, hi = 0.0, 1.0
    while sum(min(caps[q], hi * ws[q]) for q in caps) < d_max:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sum(min(caps[q], mid * ws[q]) for q in caps) < d_max:
            lo = mid
        else:
            hi = mid
    real = {q: min(float(caps[q]), hi * ws[q]) for q in caps}
    base = {q: min(caps[q], int(math.floor(real[q]))) for q in caps}
    rem = d_max - sum(base.values())
    order = sorted((q for q in caps if base[q] < caps[q]),
                   key=lambda q: (-(real[q] - math.floor(real[q])), q))
    for q in order[: max(rem, 0)]:
        base[q] += 1
    return {q: d for q, d in sorted(base.items()) if d > 0}


def bond_tables(n_orb, n_up, n_dn, d_max, beta=0.5):
    """Sector -> dimension tables of every bond the problem needs.

    Returns ``(left, right)``: ``left[l]`` for the left block of ``l`` sites
    (``l = 0..k0``), ``right[m]`` for the right block of ``m`` sites
    (``m = 0..N-k0-2``).  Each table is a dict sorted by sector.  The rule:
    the kept dimension of sector q is capped by what the previous bond can
    reach and by the dimension of the complementary Fock sector; when the
    caps exceed ``d_max`` the dimensions are water-filled with weight
    ``(f_block f_other)^beta`` (binomial Fock-sector sizes).
    """
    n = n_orb
    k0 = n // 2 - 1
    C = math.comb

    def grow(n_sites_max):
        tabs = [{(0, 0): 1}]
        for l in range(1, n_sites_max + 1):
            prev = tabs[-1]
            cands = []
            for a in range(0, min(l, n_up) + 1):
                for b in range(0, min(l, n_dn) + 1):
                    if n_up - a > n - l or n_dn - b > n - l:
                        continue
                    reach = sum(prev.get(_qsub((a, b), SITE_Q[s]), 0) for s in range(4))
                    f_other = C(n - l, n_up - a) * C(n - l, n_dn - b)
                    cap = min(reach, f_other)
                    if cap <= 0:
                        continue
                    w = float(C(l, a) * C(l, b)) * float(f_other)
                    cands.append(((a, b), cap, w ** beta))
            tabs.append(_waterfill(cands, d_max))
        return tabs

    left = grow(k0)
    right = grow(n - k0 - 2)
    return left, right


# --------------------------------------------------------------------------
# isometries
# --------------------------------------------------------------------------
def _stack_rows(old_tab, q_out):
    """Row offsets of the s-stacked in-space of out-sector q_out."""
    offs, r = [], 0
    for s in range(4):
        offs.append(r)
        r += old_tab.get(_qsub(q_out, SITE_Q[s]), 0)
    return offs, r


def _make_iso(old_tab, new_tab, rng, kind):
    blocks = {}
    for q_out, d_out in new_tab.items():
        _, n_rows = _stack_rows(old_tab, q_out)
        if kind == "random":
            g = rng.standard_normal((n_rows, d_out))
            qm, rm = np.linalg.qr(g)
            sgn = np.sign(np.diag(rm))
            sgn[sgn == 0] = 1.0
            qm = qm * sgn[None, :]
        elif kind == "det":
            rows = np.sort(rng.choice(n_rows, size=d_out, replace=False))
            qm = np.zeros((n_rows, d_out))
            qm[rows, np.arange(d_out)] = 1.0
        else:
            raise ValueError(kind)
        blocks[q_out] = np.ascontiguousarray(qm)
    return blocks


def iso_flat(old_tab, new_tab, blocks):
    """Concatenate the per-out-sector stacked matrices (canonical layout)."""
    parts = [blocks[q].reshape(-1) for q in new_tab]
    return np.concatenate(parts) if parts else np.zeros(0)


def iso_block(old_tab, new_tab, blocks, s, q_out):
    """Row block of site state s inside out-sector q_out (a view)."""
    offs, _ = _stack_rows(old_tab, q_out)
    q_in = _qsub(q_out, SITE_Q[s])
    d_in = old_tab.get(q_in, 0)
    return blocks[q_out][offs[s]: offs[s] + d_in, :]


# --------------------------------------------------------------------------
# problem
# --------------------------------------------------------------------------
@dataclass
class Problem:
    n_orb: int
    n_up: int
    n_dn: int
    k0: int
    h: np.ndarray
    V: np.ndarray
    left: list          # left[l]: sector table of the left block with l sites
    right: list         # right[m]: sector table of the right block with m sites
    iso_left: list      # iso_left[l]: {q_out: stacked matrix}, site l, l=0..k0-1
    iso_right: list     # iso_right[m-1]: site N-m, block m-1 -> m, m=1..N-k0-2
    seeds: dict = field(default_factory=dict)

    @property
    def tab_L(self):
        return self.left[self.k0]

    @property
    def tab_R(self):
        return self.right[self.n_orb - self.k0 - 2]

    def right_site(self, m):
        """Site index whose isometry builds the right block of m sites."""
        return self.n_orb - m


def make_problem(n_orb, d_max, seed, beta=0.5, n_up=None, n_dn=None,
                 iso_kind="random", h=None, V=None):
    """Seeded synthetic two-site problem.

    Seeds: integrals ``seed``, isometries ``seed+100+site1`` (1-based site
    number), start vector ``seed+200`` (see :func:`random_psi`).  Default
    filling is ``N`` electrons with ``S_z = 0`` (``S_z = +1/2`` for odd N).
    """
    n = n_orb
    if n < 4:
        raise ValueError("need at least 4 orbitals")
    if n_up is None:
        n_up = (n + 1) // 2
    if n_dn is None:
        n_dn = n // 2
    k0 = n // 2 - 1
    if h is None or V is None:
        h, V = integrals(n, seed)
    left, right = bond_tables(n, n_up, n_dn, d_max, beta)
    seed_mps = seed + 100
    iso_left = []
    for l in range(k0):
        rng = np.random.default_rng(seed_mps + l + 1)
        iso_left.append(_make_iso(left[l], left[l + 1], rng, iso_kind))
    iso_right = []
    for m in range(1, n - k0 - 1):
        site = n - m
        rng = np.random.default_rng(seed_mps + site + 1)
        iso_right.append(_make_iso(right[m - 1], right[m], rng, iso_kind))
    return Problem(n, n_up, n_dn, k0, np.asarray(h, float), np.asarray(V, float),
                   left, right, iso_left, iso_right,
                   dict(seed=seed, beta=beta, d_max=d_max, iso_kind=iso_kind))


def psi_blocks(p: Problem):
    """Two-site blocks in canonical order: list of
    ``(q_alpha, s_k, s_k1, q_beta, rows, cols, offset)``."""
    out, off = [], 0
    tl, tr = p.tab_L, p.tab_R
    tot = (p.n_up, p.n_dn)
    for qa, da in tl.items():
        for sk in range(4):
            for sk1 in range(4):
                qb = _qsub(_qsub(_qsub(tot, qa), SITE_Q[sk]), SITE_Q[sk1])
                db = tr.get(qb, 0)
                if db == 0:
                    continue
                out.append((qa, sk, sk1, qb, da, db, off))
                off += da * db
    return out


def psi_size(p: Problem):
    b = psi_blocks(p)
    return 0 if not b else b[-1][6] + b[-1][4] * b[-1][5]


def random_psi(p: Problem, seed=None):
    """Normalised standard-normal start vector (seed default ``seed+200``)."""
    if seed is None:
        seed = p.seeds.get("seed", 0) + 200
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(psi_size(p))
    return x / np.linalg.norm(x)


def batch_specs(n_problems=64, seed=4):
    """(N, D, seed) of the batched workload: one generator draws
    N ~ U{12..28} and D ~ U{128, 256, 512, 1024} per problem; problem i uses
    integral seed 1000 + i (odd N gives S_z = +1/2)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_problems):
        n = int(rng.integers(12, 29))
        d = int(rng.choice([128, 256, 512, 1024]))
        out.append((n, d, 1000 + i))
    return out
