"""GPU parity of the 4-centre class batches (Eqs. (ket-from-hermite),
(bra-from-hermite) on the matrix cores) against the FP64 CPU oracle, element
by element: |gpu - ref| <= 1e-14 + 1e-12 |ref|."""
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


def _both(ctx, sh, bra, ket, normalize=1):
    import torch
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, normalize=normalize)
    V = ctx.eri4(b, bra, ket)
    torch.cuda.synchronize()
    got = V.cpu().numpy()
    ob = oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, normalize)
    ref = oracle.eri4(ob, bra, ket)
    return got, ref


def _assert_close(got, ref, what):
    err = np.abs(got - ref)
    bad = err > ATOL + RTOL * np.abs(ref)
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} outside tolerance; max abs err {err.max():.3e}, "
                           f"max |ref| {np.abs(ref).max():.3e}")


def test_pp_quartets_full(ctx):
    """[pp|pp], K=1, 16 bra x 32 ket pairs (512 quartets), all elements."""
    sh, bra, ket = inputs.pp_quartets(seed=0)
    got, ref = _both(ctx, sh, bra, ket)
    _assert_close(got, ref, "[pp|pp]")


CLASSES = [
    ((0, 0, 0, 0), 1), ((1, 0, 0, 0), 2), ((0, 0, 1, 0), 1), ((1, 1, 1, 1), 2), ((2, 0, 1, 1), 1),
    ((2, 1, 2, 0), 2), ((2, 2, 2, 2), 1), ((2, 2, 2, 2), 3), ((3, 1, 2, 2), 1), ((3, 3, 3, 3), 1),
    ((3, 3, 3, 3), 2), ((4, 0, 4, 1), 1), ((4, 2, 3, 2), 1), ((4, 3, 1, 1), 2), ((4, 4, 4, 4), 1),
    ((4, 4, 4, 4), 3), ((0, 0, 4, 4), 1), ((4, 4, 0, 0), 2),
]


@pytest.mark.parametrize("cls,K", CLASSES)
def test_class_batch_parity(ctx, cls, K):
    la, lb, lc, ld = cls
    nbra, nket = (3, 5) if max(cls) < 4 or K == 1 else (2, 2)
    sh_b, bra = inputs.near_pairs(100 + 7 * sum(cls) + K, la, lb, K, nbra, box=6.0)
    sh_k, ket = inputs.near_pairs(200 + 7 * sum(cls) + K, lc, ld, K, nket, box=6.0)
    sh = sh_b.concat(sh_k)
    ket = ket + sh_b.n
    got, ref = _both(ctx, sh, bra, ket)
    _assert_close(got, ref, f"{cls} K={K}")


@pytest.mark.parametrize("cls,Kb,Kk,nbra,nket", [((2, 2, 2, 2), 1, 2, 3, 5), ((2, 1, 2, 2), 2, 1, 3, 5),
                                                  ((3, 3, 3, 3), 1, 1, 64, 131), ((4, 4, 4, 4), 1, 1, 64, 67),
                                                  ((1, 1, 1, 0), 1, 1, 64, 133), ((2, 2, 2, 2), 1, 1, 7, 13),
                                                  ((3, 2, 1, 0), 1, 1, 5, 1)])
def test_single_primitive_paths(ctx, cls, Kb, Kk, nbra, nket):
    """Single-primitive pairs on both sides go through quartet runs once the
    batch is large enough to keep 2048 workgroups (runs of 4 from 8192
    quartets, of 2 from 4096; ket counts that runs do not divide): the first
    four bra pairs against every ket pair are checked, which covers every
    position in a run.  Small single-primitive batches, a single-primitive
    bra with a contracted ket (V stored from registers without runs) and a
    contracted bra (plain path) are checked whole."""
    import torch
    la, lb, lc, ld = cls
    sh_b, bra = inputs.near_pairs(300 + 7 * sum(cls) + Kb, la, lb, Kb, nbra, box=6.0)
    sh_k, ket = inputs.near_pairs(400 + 7 * sum(cls) + Kk, lc, ld, Kk, nket, box=6.0)
    sh = sh_b.concat(sh_k)
    ket = ket + sh_b.n
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    V = ctx.eri4(b, bra, ket)
    torch.cuda.synchronize()
    nb = min(nbra, 4)
    got = V[:nb].cpu().numpy()
    ref = oracle.eri4(oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1), bra[:nb], ket)
    _assert_close(got, ref, f"{cls} K={Kb},{Kk} {nbra}x{nket}")
    if nbra * nket >= 4096:
        # every work split at run size (one or more row parts, one or two cubes)
        nv = ctx.eri4_tile_variants(b, bra, ket)
        for v in range(1, nv + 1):
            print(f"tile variant {v} of {nv} for {cls} {nbra}x{nket}", flush=True)
            V = ctx.eri4(b, bra, ket, tile_variant=v)
            torch.cuda.synchronize()
            _assert_close(V[:nb].cpu().numpy(), ref, f"{cls} {nbra}x{nket} variant {v}")


@pytest.mark.parametrize("seed", range(24))
def test_random_class_batches(ctx, seed):
    """Seeded random class batches: l of each centre 0..3, 1..3 primitives
    per shell drawn per pair, 1..9 bra and ket pairs, near and far pairs in
    an 8-bohr cube, normalised or bare primitives; every element against the
    oracle.  Covers the plain, single-primitive and V-from-registers paths on
    shapes the fixed cases do not pick."""
    rng = np.random.default_rng(5000 + seed)
    la, lb, lc, ld = (int(x) for x in rng.integers(0, 4, 4))
    nbra, nket = (int(x) for x in rng.integers(1, 10, 2))
    Kb = int(rng.integers(1, 4)) if seed % 3 else 1
    Kk = int(rng.integers(1, 4)) if seed % 4 else 1
    ls = [la, lb] * nbra + [lc, ld] * nket
    Ks = [Kb] * (2 * nbra) + [Kk] * (2 * nket)
    if seed % 5 == 0:  # contraction degrees that differ from pair to pair
        Ks = [int(x) for x in rng.integers(1, 4, len(ls))]
    sh = inputs.random_shells(rng, ls, Ks, 8.0, 0.1, 50.0)
    pairs = np.arange(2 * (nbra + nket), dtype=np.int32).reshape(-1, 2)
    got, ref = _both(ctx, sh, pairs[:nbra], pairs[nbra:], normalize=int(seed % 7 != 0))
    _assert_close(got, ref, f"seed {seed}: ({la}{lb}|{lc}{ld}) {nbra}x{nket}")


def test_mixed_contraction_degrees(ctx):
    """Pairs of one class may have different primitive counts."""
    rng = np.random.default_rng(5)
    sh = inputs.random_shells(rng, [2, 1, 2, 1, 3, 0, 3, 0], [1, 3, 2, 1, 2, 2, 1, 3], 5.0, 0.1, 20.0)
    got, ref = _both(ctx, sh, [[0, 1], [2, 3]], [[4, 5], [6, 7]])
    _assert_close(got, ref, "mixed K")


def test_unnormalised_basis(ctx):
    rng = np.random.default_rng(6)
    sh = inputs.random_shells(rng, [1, 2, 2, 1], [2, 1, 1, 2], 4.0, 0.2, 5.0)
    got, ref = _both(ctx, sh, [[0, 1]], [[2, 3]], normalize=0)
    _assert_close(got, ref, "raw")


def test_validation_errors(ctx):
    from paper_2405_01834_amd import MderiError
    sh, bra, ket = inputs.pp_quartets(seed=0, nbra=2, nket=2)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    with pytest.raises(MderiError):  # out-of-range shell index
        ctx.eri4(b, [[0, 99]], ket)
    sh2 = sh.concat(inputs.random_shells(np.random.default_rng(1), [2, 2], 1, 3.0, 0.5, 2.0))
    b2 = ctx.basis(sh2.l, sh2.nprim, sh2.exps, sh2.coefs, sh2.centers)
    with pytest.raises(MderiError):  # mixed classes in one batch
        ctx.eri4(b2, [[0, 1], [sh.n, sh.n + 1]], ket)
    with pytest.raises(MderiError):  # output too small
        import torch
        ctx.eri4(b, bra, ket, out=torch.empty(3, dtype=torch.float64, device="cuda"))
    with pytest.raises(MderiError):  # non-positive exponent
        ctx.basis([0], [1], [-1.0], [1.0], [[0, 0, 0]])
    with pytest.raises(MderiError):  # l beyond the built maximum
        ctx.basis([9], [1], [1.0], [1.0], [[0, 0, 0]])
    with pytest.raises(MderiError) as e:  # the FP32 split is declared but not built
        ctx.eri4(b, bra, ket, precision=2)
    assert e.value.status == -3


def test_schwarz_factors_mixed_classes(ctx):
    """Q_ij = sqrt(max_ab |(ab|ab)|) for a list mixing classes, in input order."""
    import torch
    rng = np.random.default_rng(17)
    ls = [0, 1, 2, 3, 4, 2, 1, 4, 3, 0, 2, 2]
    sh = inputs.random_shells(rng, ls, [1, 2, 1, 3, 1, 2, 1, 2, 1, 3, 1, 1], 6.0, 0.1, 30.0)
    pairs = np.array([[0, 1], [2, 3], [4, 4], [5, 6], [7, 8], [9, 10], [11, 2], [3, 3], [1, 0], [8, 7]], np.int32)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    Q = ctx.schwarz(b, pairs)
    torch.cuda.synchronize()
    ref = oracle.schwarz(oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1), pairs)
    np.testing.assert_allclose(Q.cpu().numpy(), ref, rtol=1e-12, atol=1e-14)


HIGH_L = [((5, 5, 5, 5), 1, 3, 2), ((6, 6, 6, 6), 1, 2, 2), ((6, 5, 4, 4), 1, 2, 2), ((5, 5, 5, 5), 2, 1, 2),
          ((6, 6, 3, 2), 1, 2, 3),
          # shells beyond l = 6 (total degree within the [r] builder's 26)
          ((7, 0, 7, 0), 1, 3, 2), ((8, 1, 2, 0), 2, 2, 2), ((8, 8, 4, 2), 1, 1, 2), ((7, 7, 6, 0), 1, 1, 2)]


@pytest.mark.parametrize("cls", [(5, 5, 5, 5), (6, 6, 6, 6)])
def test_high_l_single_primitive_at_size(ctx, cls):
    """Column-slab classes with single-primitive pairs at a size where the
    smaller classes take quartet runs (64 x 67 pairs; these keep one quartet
    per workgroup, their [r] cube being too large for two copies): sampled
    quartets (both ends of the bra list, neighbouring ket pairs, the tail)
    against the matrix-form reference."""
    import torch
    from tests.ref import md_matrix
    la, lb, lc, ld = cls
    nbra, nket = 64, 67
    rng = np.random.default_rng(1300 + la)
    ls = [la, lb] * nbra + [lc, ld] * nket
    sh = inputs.random_shells(rng, ls, 1, 4.0, 0.1, 30.0)
    pairs = np.arange(2 * (nbra + nket), dtype=np.int32).reshape(-1, 2)
    bra, ket = pairs[:nbra], pairs[nbra:]
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    V = ctx.eri4(b, bra, ket)
    torch.cuda.synchronize()
    for i in (0, 37, 63):
        for k in (0, 1, 2, 33, 65, 66):
            got = V[i, :, :, k].cpu().numpy()
            ref = md_matrix.shellset(sh, *bra[i], *ket[k])
            _assert_close(got, ref.reshape(got.shape), f"{cls} runs, quartet ({i},{k})")


@pytest.mark.parametrize("cls,K,nbra,nket", HIGH_L)
def test_high_l_parity(ctx, cls, K, nbra, nket):
    """[hh|hh] and [ii|ii]-type classes, whose quartets the kernel splits into
    ket-column slabs over several workgroups, against the matrix-form
    assembly of the oracle's pinned building blocks (tests/ref/md_matrix)."""
    import torch
    from tests.ref import md_matrix
    la, lb, lc, ld = cls
    rng = np.random.default_rng(1000 + 7 * la + lc + K)
    n = nbra + nket
    ls = [la, lb] * nbra + [lc, ld] * nket
    sh = inputs.random_shells(rng, ls, K, 4.0, 0.1, 30.0)
    pairs = np.arange(2 * n, dtype=np.int32).reshape(-1, 2)
    bra, ket = pairs[:nbra], pairs[nbra:]
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    V = ctx.eri4(b, bra, ket)
    torch.cuda.synchronize()
    got = V.cpu().numpy()
    for i, (p0, p1) in enumerate(bra):
        for k, (q0, q1) in enumerate(ket):
            ref = md_matrix.shellset(sh, p0, p1, q0, q1)
            _assert_close(got[i, :, :, k], ref, f"{cls} K={K} quartet ({i},{k})")


def test_beyond_fused_tiles_is_refused(ctx):
    """(77|75): V of one quartet (225 x 165) and its 455 ket Hermite rows do
    not fit the fused kernel's tiles; the call is refused, nothing runs."""
    from paper_2405_01834_amd.mderi import MderiError
    rng = np.random.default_rng(5)
    sh = inputs.random_shells(rng, [7, 7, 7, 5], 1, 4.0, 0.1, 30.0)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    with pytest.raises(MderiError, match="beyond the fused kernel"):
        ctx.eri4(b, [[0, 1]], [[2, 3]])


def test_schwarz_high_l(ctx):
    """Schwarz factors of [hh| and [ii| pairs, whose diagonal quartets run in
    column slabs, against the matrix-form reference."""
    import torch
    from tests.ref import md_matrix
    rng = np.random.default_rng(77)
    sh = inputs.random_shells(rng, [5, 5, 6, 6, 6, 5], 1, 4.0, 0.1, 30.0)
    pairs = np.array([[0, 1], [2, 3], [4, 5]], dtype=np.int32)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    Q = ctx.schwarz(b, pairs).cpu().numpy()
    torch.cuda.synchronize()
    for n, (i, j) in enumerate(pairs):
        V = md_matrix.shellset(sh, i, j, i, j)
        ref = np.sqrt(np.max(np.abs(np.diag(V))))
        assert abs(Q[n] - ref) <= 1e-12 * ref, (n, Q[n], ref)


def _class_of_total(L):
    """A class (la lb|lc ld) with la+lb+lc+ld = L, each l <= 6, bra-heavy."""
    ls = []
    for _ in range(4):
        ls.append(min(6, L - sum(ls)))
    return tuple(ls)


@pytest.mark.parametrize("L", list(range(0, 19)))
def test_every_total_l(ctx, L):
    """One class for every total L the compiled-per-L [r] builder handles
    (0..18: its y-stage lane groups and x-chain passes differ per L), with
    ragged bra/ket counts and mixed contraction, against the matrix-form
    assembly of the oracle's pinned building blocks."""
    import torch
    from tests.ref import md_matrix
    la, lb, lc, ld = _class_of_total(L)
    rng = np.random.default_rng(5000 + L)
    nbra, nket = 2, 3
    n = nbra + nket
    ls = [la, lb] * nbra + [lc, ld] * nket
    K = [1 + (i % 2) for i in range(2 * n)]
    sh = inputs.random_shells(rng, ls, K, 4.0, 0.1, 30.0)
    pairs = np.arange(2 * n, dtype=np.int32).reshape(-1, 2)
    bra, ket = pairs[:nbra], pairs[nbra:]
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    V = ctx.eri4(b, bra, ket)
    torch.cuda.synchronize()
    got = V.cpu().numpy()
    for i, (p0, p1) in enumerate(bra):
        for k, (q0, q1) in enumerate(ket):
            ref = md_matrix.shellset(sh, p0, p1, q0, q1)
            _assert_close(got[i, :, :, k], ref, f"L={L} {(la, lb, lc, ld)} quartet ({i},{k})")


@pytest.mark.parametrize("cls,K", [((2, 2, 2, 2), 1), ((3, 2, 2, 1), 2), ((4, 4, 4, 4), 1), ((3, 3, 3, 3), 3)])
def test_every_tile_variant(ctx, cls, K):
    """Every work split the autotuner may choose (mderi_eri4_tile_variants),
    forced one at a time, against the oracle; and the autotuned call."""
    import torch
    from paper_2405_01834_amd.mderi import FLAG_AUTOTUNE
    la, lb, lc, ld = cls
    nbra, nket = (3, 4) if max(cls) < 4 else (2, 2)
    sh_b, bra = inputs.near_pairs(700 + 7 * sum(cls) + K, la, lb, K, nbra, box=6.0)
    sh_k, ket = inputs.near_pairs(800 + 7 * sum(cls) + K, lc, ld, K, nket, box=6.0)
    sh = sh_b.concat(sh_k)
    ket = ket + sh_b.n
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    nv = ctx.eri4_tile_variants(b, bra, ket)
    assert nv >= 1
    ref = oracle.eri4(oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1), bra, ket)
    for v in range(1, nv + 1):
        print(f"tile variant {v} of {nv} for {cls} K={K}", flush=True)
        V = ctx.eri4(b, bra, ket, tile_variant=v)
        torch.cuda.synchronize()
        _assert_close(V.cpu().numpy(), ref, f"{cls} K={K} variant {v}")
    V = ctx.eri4(b, bra, ket, flags=FLAG_AUTOTUNE)
    torch.cuda.synchronize()
    _assert_close(V.cpu().numpy(), ref, f"{cls} K={K} autotuned")
    from paper_2405_01834_amd import MderiError
    with pytest.raises(MderiError):
        ctx.eri4(b, bra, ket, tile_variant=nv + 1)
