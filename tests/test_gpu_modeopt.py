"""GPU parity of the mode-rotation micro-iteration (Sec. II.B, Fig.
microiter) against the oracle O-MODE: the rotated two-site vector element
by element, the block entropies, the optimized angle's entropy, and the
energy invariance of the rotated vector under blocks rebuilt from the
rotated integrals (heff_rotate_integrals) at a size beyond the oracle's."""
import math

import numpy as np
import pytest

from paper_2501_18263_amd import synth
from oracle import modeopt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def heff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_18263_amd import heff as H
    return H


@pytest.fixture(scope="module")
def ctx(heff):
    return heff.Context(0)


def _dev(x):
    return torch.tensor(x, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("N,D,seed", [(8, 16, 1), (10, 32, 7), (7, 24, 2)])
def test_rotation_and_entropies_match_oracle(heff, ctx, N, D, seed):
    p = synth.make_problem(N, D, seed)
    print("case N=%d D=%d seed=%d" % (N, D, seed), flush=True)
    B = heff.Blocks(ctx, p)
    psi = synth.random_psi(p)
    x = _dev(psi)
    for theta in (0.3, -1.1, math.pi / 2):
        got = B.rotate_pair(x, theta).cpu().numpy()
        ref = modeopt.rotate_state(p, psi, theta)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        sh, sv = B.pair_entropy(_dev(ref))
        rh, rv = modeopt.entropies(p, ref)
        assert abs(sh - rh) <= 1e-10 and abs(sv - rv) <= 1e-10


def test_angle_search_matches_oracle(heff, ctx):
    p = synth.make_problem(8, 16, 1)
    B = heff.Blocks(ctx, p)
    psi = synth.random_psi(p)
    th, out, sb, sa, ne = B.optimize_pair(_dev(psi))
    t_ref, s_ref, s0 = modeopt.optimize(p, psi)
    print("theta %.10f (oracle %.10f), S %.12f (oracle %.12f), S(0) %.12f, %d trials" % (th, t_ref, sa, s_ref, sb, ne))
    assert abs(sb - s0) <= 1e-10
    assert abs(sa - s_ref) <= 1e-8 and sa <= sb
    ref = modeopt.rotate_state(p, psi, th)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_rotated_vector_keeps_energy_under_rotated_integrals(heff, ctx):
    # N=16, D=256: the optimized rotation of the middle pair, then blocks
    # rebuilt from the rotated integrals with the same isometries
    p = synth.make_problem(16, 256, 5)
    print("case N=16 D=256 seed=5", flush=True)
    B = heff.Blocks(ctx, p)
    x = _dev(synth.random_psi(p))
    e0 = B.energy(x)
    th, xr, sb, sa, ne = B.optimize_pair(x)
    h2, V2 = heff.rotate_integrals(p.h, p.V, p.k0, p.k0 + 1, th)
    p2 = synth.make_problem(16, 256, 5, h=h2, V=V2)
    B2 = heff.Blocks(ctx, p2)
    e1 = B2.energy(xr)
    print("theta %.6f S %.6f -> %.6f, E %.15f %.15f" % (th, sb, sa, e0, e1))
    assert abs(e1 - e0) <= 1e-10 * abs(e0)
    assert abs(B.energy(xr) - e0) > 1e-8  # the old integrals see a different energy
