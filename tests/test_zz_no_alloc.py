"""heff_energy_noalloc through the C ABI against heff_energy (GPU).

The allocation-free entry point keeps its scratch in a static device array;
it must give the energy of heff_energy (same kernels, same order: bitwise
equal, held here to 1e-12 relative) on consecutive calls whose inputs
shrink, allocate nothing through the context's memory provider, and refuse
a psi larger than its scratch with HEFF_EINVAL."""
import numpy as np
import pytest

from paper_2501_18263_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def heff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_18263_amd import heff as H
    return H


def test_energy_noalloc_matches_energy(heff):
    counts = {"alloc": 0, "free": 0}

    def alloc(n):
        counts["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(max(n, 1), 0, torch.cuda.current_stream(0).cuda_stream)

    def free(p):
        counts["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    ctx = heff.Context(0, allocator=(alloc, free))
    # two calls in a row, the second with a smaller input
    for N, D, seed in ((16, 256, 5), (8, 32, 1)):
        p = synth.make_problem(N, D, seed)
        print("case N=%d D=%d seed=%d" % (N, D, seed), flush=True)
        B = heff.Blocks(ctx, p, precs=(heff.FP64, heff.FP32))
        psi = torch.tensor(synth.random_psi(p), device="cuda")
        for prec, x in ((heff.FP64, psi), (heff.FP32, psi.float())):
            e_ref = B.energy(x, prec)
            torch.cuda.synchronize()
            before = dict(counts)
            e_na = B.energy_noalloc(x, prec)
            torch.cuda.synchronize()
            assert counts == before  # nothing allocated or freed through the provider
            print("prec %d: energy %.15f, no-alloc %.15f" % (prec, e_ref, e_na))
            assert abs(e_na - e_ref) <= 1e-12 * abs(e_ref)
        B.close()
    ctx.close()


def test_energy_noalloc_rejects_oversized_psi(heff):
    # N=40, D=4096 with beta=1: 7.55M elements, 60 MB in FP64 (beyond the
    # 48 MiB scratch: HEFF_EINVAL naming the limit), 30 MB in FP32 (accepted)
    ctx = heff.Context(0)
    p = synth.make_problem(40, 4096, 3, beta=1.0)
    print("case N=40 D=4096 seed=3 beta=1", flush=True)
    B = heff.Blocks(ctx, p, precs=(heff.FP64, heff.FP32))
    assert B.n_elem * 8 > (48 << 20) >= B.n_elem * 4
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.standard_normal(B.n_elem), device="cuda")
    with pytest.raises(heff.HeffError) as ei:
        B.energy_noalloc(x, heff.FP64)
    assert ei.value.code == heff.HEFF_EINVAL and "static scratch" in str(ei.value)
    x32 = x.float()
    e_ref = B.energy(x32, heff.FP32)
    e_na = B.energy_noalloc(x32, heff.FP32)
    assert abs(e_na - e_ref) <= 1e-12 * abs(e_ref)
    B.close()
    ctx.close()
