"""GPU test of the allocation-free entry point mderi_eri4_noalloc: two calls
in a row through the C ABI (the second with a smaller batch, so it runs on
scratch that still holds the first call's data) against mderi_eri4 on the
same inputs, element by element at the FP64 bar |d| <= 1e-14 + 1e-12 |ref|,
and against the oracle; oversized batches are refused before anything is
enqueued."""
import numpy as np
import pytest

import oracle
from paper_2405_01834_amd import inputs

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-12, 1e-14


@pytest.fixture(scope="module")
def ctx(need_gpu):
    from paper_2405_01834_amd import Context
    return Context(0)


def _close(got, ref, what):
    err = np.abs(got - ref)
    bad = err > ATOL + RTOL * np.abs(ref)
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} outside; max abs err {err.max():.3e}"


CASES = [  # (la, lb, lc, ld), K, nbra, nket, seed -- the second is smaller
    ((2, 1, 2, 2), 2, 6, 7, 11),
    ((1, 1, 1, 0), 1, 3, 2, 12),
]


def test_noalloc_two_calls_match_eri4(ctx):
    import torch
    for (la, lb, lc, ld), K, nbra, nket, seed in CASES:
        sh_b, bra = inputs.near_pairs(seed, la, lb, K, nbra, box=6.0)
        sh_k, ket = inputs.near_pairs(seed + 100, lc, ld, K, nket, box=6.0)
        sh = sh_b.concat(sh_k)
        ket = ket + sh_b.n
        b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
        print(f"noalloc case ({la}{lb}|{lc}{ld}) K={K} {nbra}x{nket}", flush=True)
        ref = ctx.eri4(b, bra, ket)
        torch.cuda.synchronize()
        n = ref.numel()
        out = torch.full((n + 5,), float("nan"), dtype=torch.float64, device="cuda:0")
        got = ctx.eri4_noalloc(b, bra, ket, out)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(g).all()
        _close(g, r, f"noalloc vs eri4 ({la}{lb}|{lc}{ld})")
        assert torch.isnan(out[n:]).all(), "wrote past the batch"
        ob = oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1)
        _close(g, oracle.eri4(ob, bra, ket), f"noalloc vs oracle ({la}{lb}|{lc}{ld})")


def test_noalloc_refuses_oversized_batches(ctx):
    import torch
    from paper_2405_01834_amd.mderi import MderiError
    # 280 x 280 [gg|gg] pairs need about 77 MB of transform matrices: more
    # than the 64 MiB scratch, refused on the host before any launch
    sh, pairs = inputs.class_pairs(5, 4, 4, 1, 560)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    out = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    with pytest.raises(MderiError) as e:
        ctx.eri4_noalloc(b, pairs[:280], pairs[280:], out)
    assert e.value.status == -5  # MDERI_ESIZE (the output check fires first here, also ESIZE)
    big = torch.zeros(280 * 81 * 81 * 280, dtype=torch.float64, device="cuda:0")
    with pytest.raises(MderiError) as e:
        ctx.eri4_noalloc(b, pairs[:280], pairs[280:], big)
    assert e.value.status == -5 and "scratch" in str(e.value)
    del big
    torch.cuda.synchronize()
