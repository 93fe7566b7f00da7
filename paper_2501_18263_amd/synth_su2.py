"""Seeded synthetic inputs of the SU(2) spin-adapted two-site product.

Inputs only, none of the product's arithmetic: the multiplet sectors of the
left and right blocks, their irreducible tensor operators given by random
reduced matrix elements, a list of Hamiltonian terms (Sec. II.C: each term
is a product of a left-block, a site-k, a site-(k+1) and a right-block
operator, coupled to a scalar), the target particle number and total spin,
the layout of the reduced two-site vector and a random start vector.  The
CPU oracle and the GPU library both consume what is generated here.

Conventions (shared by every consumer):

* Spins are stored doubled (``ts = 2 S``), so half-integers are integers.
* A block sector is ``(n, ts, dim)``: particle number, doubled spin and the
  number of multiplets.  ``ts`` has the parity of ``n``.
* Site multiplets of one spatial orbital: code 0 empty (n=0, S=0), code 1
  the doublet (n=1, S=1/2), code 2 the doubly occupied singlet (n=2, S=0).
* Site operators by code (rank, particle-number change): 0 identity (0, 0),
  1 creation tensor (1/2, +1), 2 annihilation tensor (1/2, -1), 3 number
  (0, 0), 4 spin vector (1, 0), 5 pair creation (0, +2), 6 pair
  annihilation (0, -2).  Their matrices are defined in the oracle.
* A block operator is ``(ts_k, dn, blocks)``: doubled rank, particle-number
  change and ``blocks[(o, i)]`` the ``dim_o x dim_i`` reduced matrix between
  sectors ``i -> o``; every block allowed by ``n_o = n_i + dn`` and the
  triangle rule ``|S_i - k| <= S_o <= S_i + k`` is present.  A block
  operator is odd (fermionic) when ``dn`` is odd.
* A term is ``(l_op, site_k, site_k1, r_op, ts_c, coef)``: operator indices
  (-1 = identity of the block), site-operator codes, the doubled spin of the
  coupled left part ``[O_L x O_k]`` (equal to that of the right part
  ``[O_k1 x O_R]``, which the two couple to a scalar) and a coefficient.
* The reduced two-site vector: blocks ``(il, mk, tsg, mk1, ir, tsd)`` -- left
  sector, site-k multiplet, doubled spin of left x site k, site-(k+1)
  multiplet, right sector, doubled spin of site k+1 x right -- with total
  particle number ``n_tot`` and ``ts_tot`` in the product of ``tsg`` and
  ``tsd``; sorted lexicographically by that key, each a row-major
  ``dim_l x dim_r`` matrix, concatenated.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SITE_MULT = ((0, 0), (1, 1), (2, 0))  # (n, ts) of site multiplets 0, 1, 2
SITE_OPS = ((0, 0), (1, 1), (1, -1), (0, 0), (2, 0), (0, 2), (0, -2))  # (ts_k, dn)


def triangle(ta, tb, tc):
    """Doubled spins a, b, c satisfy the triangle rule."""
    return abs(ta - tb) <= tc <= ta + tb and (ta + tb + tc) % 2 == 0


def couple(ta, tb):
    """Doubled spins in the product of spins a and b."""
    return list(range(abs(ta - tb), ta + tb + 1, 2))


@dataclass
class Block:
    sectors: list  # (n, ts, dim)
    ops: list = field(default_factory=list)  # (ts_k, dn, {(o, i): ndarray})

    def dim_m(self):
        """States with the magnetic quantum number resolved."""
        return sum(d * (ts + 1) for _, ts, d in self.sectors)


@dataclass
class Su2Problem:
    L: Block
    R: Block
    terms: list  # (l_op, site_k, site_k1, r_op, ts_c, coef)
    n_tot: int
    ts_tot: int


def sectors(rng, n_range, ts_max, dmax, dmin=1):
    out = []
    for n in n_range:
        for ts in range(n % 2, min(n, ts_max) + 1, 2):
            out.append((n, ts, int(rng.integers(dmin, dmax + 1))))
    return out


def random_op(rng, blk: Block, ts_k, dn):
    blocks = {}
    for o, (no, tso, do) in enumerate(blk.sectors):
        for i, (ni, tsi, di) in enumerate(blk.sectors):
            if no == ni + dn and triangle(tsi, ts_k, tso):
                blocks[(o, i)] = rng.standard_normal((do, di)) / np.sqrt(di)
    return (ts_k, dn, blocks)


OP_KINDS = ((0, 0), (2, 0), (1, 1), (1, -1), (0, 2), (0, -2), (2, 2), (2, -2))


def make_problem(seed, l_sectors, r_sectors, n_lops, n_rops, n_terms, n_tot, ts_tot=0):
    """Random operators (kinds cycling through OP_KINDS) and terms whose
    particle-number changes cancel and whose ranks couple to a scalar."""
    rng = np.random.default_rng(seed)
    L, R = Block(list(l_sectors)), Block(list(r_sectors))
    for blk, n_ops in ((L, n_lops), (R, n_rops)):
        for j in range(n_ops):
            ts_k, dn = OP_KINDS[j % len(OP_KINDS)]
            blk.ops.append(random_op(rng, blk, ts_k, dn))
    lk = [(-1, 0, 0)] + [(j, op[0], op[1]) for j, op in enumerate(L.ops)]
    rk = [(-1, 0, 0)] + [(j, op[0], op[1]) for j, op in enumerate(R.ops)]
    terms = []
    tries = 0
    while len(terms) < n_terms and tries < 200 * n_terms:
        tries += 1
        l, tl, dl = lk[int(rng.integers(len(lk)))]
        sk = int(rng.integers(len(SITE_OPS)))
        sk1 = int(rng.integers(len(SITE_OPS)))
        r, tr, dr = rk[int(rng.integers(len(rk)))]
        if dl + SITE_OPS[sk][1] + SITE_OPS[sk1][1] + dr != 0:
            continue
        tcs = [t for t in couple(tl, SITE_OPS[sk][0]) if triangle(SITE_OPS[sk1][0], tr, t)]
        if not tcs:
            continue
        tc = tcs[int(rng.integers(len(tcs)))]
        terms.append((l, sk, sk1, r, tc, float(rng.standard_normal())))
    return Su2Problem(L, R, terms, n_tot, ts_tot)


def psi_blocks(p: Su2Problem):
    """[(key, offset, rows, cols)] of the reduced two-site vector."""
    out = []
    off = 0
    for il, (nl, tsl, dl) in enumerate(p.L.sectors):
        for mk, (nk, tsk) in enumerate(SITE_MULT):
            for tsg in couple(tsl, tsk):
                for mk1, (nk1, tsk1) in enumerate(SITE_MULT):
                    for ir, (nr, tsr, dr) in enumerate(p.R.sectors):
                        if nl + nk + nk1 + nr != p.n_tot:
                            continue
                        for tsd in couple(tsk1, tsr):
                            if not triangle(tsg, tsd, p.ts_tot):
                                continue
                            out.append(((il, mk, tsg, mk1, ir, tsd), off, dl, dr))
                            off += dl * dr
    return out


def psi_size(p: Su2Problem):
    b = psi_blocks(p)
    return b[-1][1] + b[-1][2] * b[-1][3] if b else 0


def random_psi(p: Su2Problem, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(psi_size(p))
    return x / np.linalg.norm(x)


def op_arrays(blk: Block):
    """Flat form of a block's operators for the C ABI: per block of every
    operator (op, out sector, in sector, element offset) and the data."""
    bop, bout, bin_, boff, data = [], [], [], [], []
    off = 0
    for j, (_, _, blocks) in enumerate(blk.ops):
        for (o, i), a in sorted(blocks.items()):
            bop.append(j)
            bout.append(o)
            bin_.append(i)
            boff.append(off)
            data.append(np.ascontiguousarray(a, dtype=np.float64).reshape(-1))
            off += a.size
    flat = np.concatenate(data) if data else np.zeros(0)
    return (np.array(bop, np.int32), np.array(bout, np.int32), np.array(bin_, np.int32),
            np.array(boff, np.int64), flat)


def small_problem(seed=1, dmax=3):
    """A problem whose magnetic-resolved space the oracle handles densely."""
    rng = np.random.default_rng(seed + 500)
    Ls = sectors(rng, range(0, 4), 3, dmax)
    Rs = sectors(rng, range(0, 4), 3, dmax)
    return make_problem(seed, Ls, Rs, 8, 8, 60, 4, 0)


def bench_problem(seed=3, d_scale=1.0, n_terms=1500):
    """The benchmark problem: blocks of 4..20 electrons with spins up to
    11/2 and multiplet dimensions shaped like a truncated bond (largest at 12
    electrons and low spin, at most 256): 75 sectors, 2692 multiplets per
    block (10645 states with the magnetic quantum number resolved, the
    compression the paper quotes for its largest SU(2) runs), 48 random
    operators per block, 26 electrons in a singlet."""
    rng = np.random.default_rng(seed + 500)

    def secs():
        out = []
        for n in range(4, 21):
            for ts in range(n % 2, min(n, 11) + 1, 2):
                w = np.exp(-0.5 * ((n - 12) / 2.2) ** 2 - 0.25 * ts)
                d = int(round(d_scale * 230 * w * (0.8 + 0.4 * rng.random())))
                if d >= 1:
                    out.append((n, ts, min(d, 256)))
        return out

    Ls = secs()
    Rs = secs()
    return make_problem(seed, Ls, Rs, 48, 48, n_terms, 26, 0)
