"""Helpers for the GPU tests: flatten oracle operators in the library's
block order and run the library on a generated problem."""
import numpy as np

from paper_2501_18263_amd import synth


def flat_oracle_op(op, tab):
    """Concatenate an oracle operator's blocks ordered by in-sector (table order)."""
    parts = []
    for q in tab:
        if q in op.blocks:
            parts.append(op.blocks[q][1].reshape(-1))
    return np.concatenate(parts) if parts else np.zeros(0)


def layout_matches(p, blocks):
    ref = synth.psi_blocks(p)
    if len(ref) != len(blocks):
        return False
    for (qa, sk, sk1, qb, da, db, off), (u, d, s1, s2, r, c, o) in zip(ref, blocks):
        if (qa, sk, sk1, da, db, off) != ((u, d), s1, s2, r, c, o):
            return False
    return True
