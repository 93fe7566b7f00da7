"""Test infrastructure: reference (oracle) code.  Only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg may import it.

Determinant labels of the two-site basis when every isometry is a 0/1
selection matrix (``iso_kind="det"``): each kept block state is then one
occupation configuration, and each two-site basis vector
|alpha>|s_k>|s_k+1>|beta> is one determinant with coefficient +1 (the
creation strings of L, the middle sites and R are already in mode order).
This lets the full-CI determinant action (``fci.c``) check single output
entries of H_eff . psi at any size.
"""
from __future__ import annotations

import numpy as np

from paper_2501_18263_amd import synth

SITE_Q = synth.SITE_Q


def _site_bits(i, s):
    v = 0
    if s in (2, 3):
        v |= 1 << (2 * i)
    if s in (1, 3):
        v |= 1 << (2 * i + 1)
    return v


def _grow(tabs, isos, site_of_step, left):
    cfg = {(0, 0): [0]}
    for step in range(len(isos)):
        old, new = tabs[step], tabs[step + 1]
        site = site_of_step(step)
        nc = {}
        for q_out, d_out in new.items():
            m = isos[step][q_out]
            offs, r = [], 0
            for s in range(4):
                offs.append(r)
                r += old.get((q_out[0] - SITE_Q[s][0], q_out[1] - SITE_Q[s][1]), 0)
            lst = []
            for j in range(d_out):
                col = m[:, j]
                nz = np.nonzero(col)[0]
                if len(nz) != 1 or col[nz[0]] != 1.0:
                    raise ValueError("isometry is not a 0/1 selection")
                row = int(nz[0])
                s = max(k for k in range(4) if offs[k] <= row and
                        old.get((q_out[0] - SITE_Q[k][0], q_out[1] - SITE_Q[k][1]), 0) > row - offs[k])
                q_in = (q_out[0] - SITE_Q[s][0], q_out[1] - SITE_Q[s][1])
                lst.append(cfg[q_in][row - offs[s]] | _site_bits(site, s))
            nc[q_out] = lst
        cfg = nc
    return cfg


def left_configs(p):
    return _grow(p.left, p.iso_left, lambda l: l, True)


def right_configs(p):
    return _grow(p.right, p.iso_right, lambda step: p.n_orb - (step + 1), False)


def psi_determinants(p):
    """(dim psi, 2) uint64 (lo, hi) determinant of every two-site basis vector."""
    Lc, Rc = left_configs(p), right_configs(p)
    out = np.empty((synth.psi_size(p), 2), dtype=np.uint64)
    mask = (1 << 64) - 1
    for (qa, sk, sk1, qb, da, db, off) in synth.psi_blocks(p):
        mid = _site_bits(p.k0, sk) | _site_bits(p.k0 + 1, sk1)
        la = np.array([[(v | mid) & mask, (v | mid) >> 64] for v in Lc[qa]], dtype=np.uint64)
        rb = np.array([[v & mask, v >> 64] for v in Rc[qb]], dtype=np.uint64)
        lo = la[:, None, 0] | rb[None, :, 0]
        hi = la[:, None, 1] | rb[None, :, 1]
        out[off: off + da * db, 0] = lo.reshape(-1)
        out[off: off + da * db, 1] = hi.reshape(-1)
    return out
