"""GPU parity of the SU(2) spin-adapted product (heff_su2_*, Sec. II.C,
Eq. Hamilton_act_su2) against the oracle O-SU2.

Small problems are compared element by element with the definition
E^T H E (the state-resolved product restricted to the multiplet basis);
a medium problem whose blocks span two 64-row work items with ragged
edges, and the benchmark problem on sampled output blocks, with the task
form (which the oracle pins equal to the definition).  Bars: FP64 1e-12 of
the largest output element; FP32 and the bf16 split, relative norm error
1e-5 and 4e-5, the bars of the U(1) products."""
import numpy as np
import pytest

from paper_2501_18263_amd import synth_su2 as S
from oracle import su2

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


def _run(heff, H, x, prec):
    dt = torch.float64 if prec == heff.FP64 else torch.float32
    xd = torch.tensor(x, dtype=dt, device="cuda")
    y = torch.empty_like(xd)
    H.apply(xd, y, prec)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def _medium():
    rng = np.random.default_rng(9)
    Ls = S.sectors(rng, range(2, 7), 5, 70, 20)
    Rs = S.sectors(rng, range(2, 7), 5, 70, 20)
    return S.make_problem(9, Ls, Rs, 16, 16, 120, 9, 1)


@pytest.mark.parametrize("seed,n_tot,ts_tot", [(1, 4, 0), (4, 4, 2), (5, 3, 1), (6, 5, 3)])
def test_su2_product_matches_definition(heff, ctx, seed, n_tot, ts_tot):
    p = S.small_problem(seed)
    p.n_tot, p.ts_tot = n_tot, ts_tot
    print("case small seed=%d n=%d 2S=%d" % (seed, n_tot, ts_tot), flush=True)
    H = heff.Su2(ctx, p)
    assert [(k, o, r, c) for k, o, r, c in S.psi_blocks(p)] == [(k, o, r, c) for k, o, r, c in H.blocks]
    assert H.n_elem == S.psi_size(p)
    x = S.random_psi(p, seed=seed)
    y0 = su2.apply_definition(p, x)
    y = _run(heff, H, x, heff.FP64)
    assert np.abs(y - y0).max() <= 1e-12 * np.abs(y0).max()
    st = H.stats()
    assert st["n_tasks"] > 0 and st["flops"] > 0 and st["n_resolved"] >= H.n_elem


def test_su2_product_medium_all_precisions(heff, ctx):
    p = _medium()
    print("case medium", flush=True)
    H = heff.Su2(ctx, p, precs=(heff.FP64, heff.FP32, heff.BF16X3))
    x = S.random_psi(p, seed=3)
    y0 = su2.apply_tasks(p, x)
    y = _run(heff, H, x, heff.FP64)
    assert np.abs(y - y0).max() <= 1e-12 * np.abs(y0).max()
    for prec, bar in ((heff.FP32, 1e-5), (heff.BF16X3, 4e-5)):
        yr = _run(heff, H, x, prec)
        err = np.linalg.norm(yr - y0) / np.linalg.norm(y0)
        print("precision %d: relative error %.2e" % (prec, err))
        assert err <= bar


def test_su2_product_wide_middle_dimension(heff, ctx):
    # right sectors up to 200 wide beside narrow ones: outputs wider than
    # 128 (run as column slices) and tasks with a middle dimension above 128
    # (run as ranges of it); element-wise vs the task form
    rng = np.random.default_rng(10)
    Ls = S.sectors(rng, range(2, 5), 3, 24, 4)
    Rs = [(2, 0, 200), (2, 2, 40), (3, 1, 150), (3, 3, 20), (4, 0, 90), (4, 2, 130)]
    p = S.make_problem(11, Ls, Rs, 12, 12, 60, 7, 1)
    print("case wide middle dimension", flush=True)
    H = heff.Su2(ctx, p, precs=(heff.FP64, heff.FP32))
    x = S.random_psi(p, seed=4)
    y0 = su2.apply_tasks(p, x)
    y = _run(heff, H, x, heff.FP64)
    assert np.abs(y - y0).max() <= 1e-12 * np.abs(y0).max()
    yr = _run(heff, H, x, heff.FP32)
    assert np.linalg.norm(yr - y0) / np.linalg.norm(y0) <= 1e-5


def test_su2_product_benchmark_size_sampled(heff, ctx):
    # the benchmark problem (75 sectors, 2692 multiplets per block, 1500
    # terms): output blocks sampled (the two largest, whose task chains run
    # split over several work-groups, and six random); a second product is
    # bitwise the first (the split chains' parts are added in a fixed order)
    p = S.bench_problem(3)
    print("case benchmark size", flush=True)
    H = heff.Su2(ctx, p)
    x = S.random_psi(p, seed=5)
    y = _run(heff, H, x, heff.FP64)
    assert np.array_equal(_run(heff, H, x, heff.FP64), y)
    blocks = S.psi_blocks(p)
    rng = np.random.default_rng(0)
    pick = sorted(blocks, key=lambda b: -b[2] * b[3])[:2] + [blocks[i] for i in rng.choice(len(blocks), 6, replace=False)]
    y0 = su2.apply_tasks(p, x, only={b[0] for b in pick})
    scale = max(np.abs(y0[o:o + r * c]).max() for _, o, r, c in pick)
    for key, o, r, c in pick:
        assert np.abs(y[o:o + r * c] - y0[o:o + r * c]).max() <= 1e-12 * scale, key
    st = H.stats()
    print("tasks %d, flops %.3e, reduced %d, resolved %.3e" % (st["n_tasks"], st["flops"], H.n_elem, st["n_resolved"]))


def test_su2_refusals(heff, ctx):
    p = S.small_problem(1)
    bad = S.Su2Problem(p.L, p.R, p.terms + [(-1, 1, 0, -1, 1, 1.0)], p.n_tot, p.ts_tot)  # creates a particle
    with pytest.raises(heff.HeffError) as ei:
        heff.Su2(ctx, bad)
    assert ei.value.code == heff.HEFF_EINVAL and "particle" in str(ei.value)
    bad = S.Su2Problem(p.L, p.R, p.terms + [(-1, 4, 0, -1, 0, 1.0)], p.n_tot, p.ts_tot)  # rank 1 x 0 -> 0
    with pytest.raises(heff.HeffError) as ei:
        heff.Su2(ctx, bad)
    assert ei.value.code == heff.HEFF_EINVAL and "triangle" in str(ei.value)
    L2 = S.Block([(1, 0, 2)] + p.L.sectors[1:], [])  # one electron, spin 0
    with pytest.raises(heff.HeffError) as ei:
        heff.Su2(ctx, S.Su2Problem(L2, p.R, [], p.n_tot, p.ts_tot))
    assert ei.value.code == heff.HEFF_EINVAL
    with pytest.raises(heff.HeffError) as ei:
        heff.Su2(ctx, S.Su2Problem(p.L, p.R, p.terms, 40, 0))
    assert ei.value.code == heff.HEFF_ESECTOR
    H = heff.Su2(ctx, p)  # FP64 only
    x = torch.zeros(H.n_elem, dtype=torch.float32, device="cuda")
    with pytest.raises(heff.HeffError) as ei:
        H.apply(x, torch.empty_like(x), heff.FP32)
    assert ei.value.code == heff.HEFF_ENOTSUP
