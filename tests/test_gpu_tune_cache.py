"""Persistent autotune cache (mderi_tune_save / mderi_tune_load): the tile
choices one context's autotuner made, written to a file and read into a
fresh context, give that context the same work split without timing the
candidates again (the same integrals, up to the order in which row parts
add into LDS); the file round-trips unchanged; files that do not parse or
come from another architecture are refused and leave the context as it was;
a stored choice that is not among a class's candidates is ignored."""
import numpy as np
import pytest

from paper_2405_01834_amd import inputs

pytestmark = pytest.mark.gpu


def _batch(ctx, l, K, seed, n=24):
    sh, cand = inputs.class_pairs(seed, l, l, K, 2 * n, box=6.0)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    return b, cand[:n], cand[n:]


def test_tune_cache_round_trip(need_gpu, tmp_path):
    import torch
    from paper_2405_01834_amd import Context
    from paper_2405_01834_amd.mderi import FLAG_AUTOTUNE, MderiError
    c1 = Context(0)
    runs = {}
    for l, K in ((3, 1), (2, 2)):
        b, bra, ket = _batch(c1, l, K, 50 + l)
        c1.eri4(b, bra, ket, flags=FLAG_AUTOTUNE)
        runs[(l, K)] = (bra, ket, c1.eri4(b, bra, ket).clone())
    torch.cuda.synchronize()
    p = tmp_path / "tune.txt"
    c1.tune_save(p)
    text = p.read_text()
    head, count = text.splitlines()[:2]
    assert head.startswith("mderi-tune 1 gfx950") and int(count) >= 1

    c2 = Context(0)
    c2.tune_load(p)
    for (l, K), (bra, ket, ref) in runs.items():
        b2, _, _ = _batch(c2, l, K, 50 + l)
        got = c2.eri4(b2, bra, ket)
        torch.cuda.synchronize()
        # equal up to the order of the row parts' LDS adds (nps > 1 splits)
        assert float((got - ref).abs().max()) <= 1e-13 * float(ref.abs().max()), (l, K)
    p2 = tmp_path / "tune2.txt"
    c2.tune_save(p2)
    assert p2.read_text() == text

    bad = {"missing": None, "header": "not a cache\n0\n",
           "arch": text.replace(head, "mderi-tune 1 gfx000")}
    bad["entry"] = "\n".join([head, str(int(count) + 1)] + text.splitlines()[2:] + ["1 2 x 4 5 6 7 8 9"]) + "\n"
    for name, body in bad.items():
        q = tmp_path / f"bad_{name}.txt"
        if body is not None:
            q.write_text(body)
        with pytest.raises(MderiError) as e:
            c2.tune_load(q)
        assert e.value.status == -1, name
    p3 = tmp_path / "tune3.txt"
    c2.tune_save(p3)
    assert p3.read_text() == text

    # an entry naming tiles no class offers is ignored when the class runs
    fake = "\n".join([head, "1", "3 3 3 3 1 1 999 999 1"]) + "\n"
    q = tmp_path / "fake.txt"
    q.write_text(fake)
    c2.tune_load(q)
    bra, ket, ref = runs[(3, 1)]
    b2, _, _ = _batch(c2, 3, 1, 53)
    got = c2.eri4(b2, bra, ket)
    torch.cuda.synchronize()
    assert float((got - ref).abs().max()) <= 1e-13 * float(ref.abs().max())
