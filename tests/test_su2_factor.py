"""The library's factor table of the SU(2) product (rescaled 9j symbols by
Racah's 6j formula, host code, no GPU) against the oracle's contraction of
six Clebsch-Gordan coefficients (Fig. SU2FactorCell), over every admissible
combination of the spins the two-site tasks use."""
import itertools

from paper_2501_18263_amd import heff, synth_su2 as S
from oracle import su2


def test_library_factor_matches_six_cg_contraction():
    n = 0
    worst = 0.0
    for ta, tb, tka, tkb in itertools.product(range(0, 9), (0, 1), range(0, 4), range(0, 3)):
        for tc, tkc in itertools.product(S.couple(ta, tb), S.couple(tka, tkb)):
            for ta2, tb2 in itertools.product(S.couple(ta, tka), S.couple(tb, tkb)):
                if tb2 > 1:
                    continue
                for tc2 in S.couple(ta2, tb2):
                    if not su2._tri(tc, tkc, tc2):
                        continue
                    j = (ta, tb, tc, tka, tkb, tkc, ta2, tb2, tc2)
                    f0 = su2.factor_fig(*j)
                    f1 = heff.su2_factor(j)
                    worst = max(worst, abs(f1 - f0))
                    assert abs(f1 - f0) <= 1e-13, (j, f0, f1)
                    n += 1
    # the total level (rank-S parts coupled to a scalar)
    for tg, td, tk in itertools.product(range(0, 7), range(0, 7), range(0, 4)):
        for tt in S.couple(tg, td):
            for tg2, td2 in itertools.product(S.couple(tg, tk), S.couple(td, tk)):
                if not su2._tri(tg2, td2, tt):
                    continue
                j = (tg, td, tt, tk, tk, 0, tg2, td2, tt)
                assert abs(heff.su2_factor(j) - su2.factor_fig(*j)) <= 1e-13
                n += 1
    assert n > 1000


def test_library_factor_zero_outside_triangles():
    assert heff.su2_factor((1, 1, 4, 0, 0, 0, 1, 1, 4)) == 0.0
    # a spin above the table's range is refused
    import pytest
    with pytest.raises(heff.HeffError):
        heff.su2_factor((200, 1, 1, 0, 0, 0, 1, 1, 1))
