"""GPU parity of 3-centre class batches (ab|P) (1-centre Hermite expansion of
Eqs. (E1rr)-(E1-aa); only the top-degree Hermite functions of the auxiliary
shell enter) against the FP64 CPU oracle: |gpu - ref| <= 1e-14 + 1e-12 |ref|."""
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


def _run(ctx, sh, aux, pairs, auxidx):
    import torch
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    a = ctx.basis(aux.l, aux.nprim, aux.exps, aux.coefs, aux.centers)
    V = ctx.eri3(b, a, pairs, auxidx)
    torch.cuda.synchronize()
    got = V.cpu().numpy()
    ref = oracle.eri3(oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1),
                      oracle.Basis(aux.l, aux.nprim, aux.exps, aux.coefs, aux.centers, 1), pairs, auxidx)
    err = np.abs(got - ref)
    bad = err > ATOL + RTOL * np.abs(ref)
    assert not bad.any(), f"{bad.sum()} of {bad.size} outside tolerance; max err {err.max():.3e}"


CASES = [((0, 0), 0, 1, 1), ((1, 0), 2, 2, 1), ((1, 1), 1, 3, 1), ((2, 1), 3, 1, 1), ((3, 3), 6, 1, 1),
         ((2, 2), 4, 5, 1), ((3, 2), 5, 2, 1), ((0, 0), 6, 3, 1), ((3, 3), 0, 2, 1), ((1, 3), 4, 4, 1),
         # auxiliary shells beyond l = 6
         ((1, 1), 8, 2, 1), ((3, 2), 7, 1, 1), ((0, 0), 8, 3, 1), ((3, 3), 8, 1, 1)]


@pytest.mark.parametrize("cls,lP,K,KP", CASES)
def test_eri3_class_parity(ctx, cls, lP, K, KP):
    la, lb = cls
    sh, pairs = inputs.near_pairs(300 + 11 * la + lb + 5 * K, la, lb, K, 3, box=6.0)
    aux = inputs.random_shells(np.random.default_rng(400 + lP), [lP] * 4, KP, 6.0, 0.05, 50.0)
    _run(ctx, sh, aux, pairs, np.arange(4, dtype=np.int32))


def test_eri3_mixed_primary_contraction(ctx):
    rng = np.random.default_rng(9)
    sh = inputs.random_shells(rng, [2, 1, 2, 1, 2, 1], [1, 5, 3, 2, 4, 1], 5.0, 0.05, 500.0)
    aux = inputs.random_shells(rng, [3, 3, 3], 1, 5.0, 0.05, 500.0)
    _run(ctx, sh, aux, [[0, 1], [2, 3], [4, 5]], [2, 0, 1])


def _mixed(seed, npair, naux):
    """Pairs of every class with l <= 3 and K 1..3 per shell; aux l 0..6, K=1."""
    rng = np.random.default_rng(seed)
    ls = [int(x) for x in rng.integers(0, 4, 2 * npair)]
    Ks = [int(x) for x in rng.integers(1, 4, 2 * npair)]
    sh = inputs.random_shells(rng, ls, Ks, 6.0, 0.05, 500.0)
    lP = [k % 7 for k in range(naux)]
    aux = inputs.random_shells(rng, lP, 1, 6.0, 0.05, 500.0)
    return sh, aux, np.arange(2 * npair, dtype=np.int32).reshape(-1, 2), np.arange(naux, dtype=np.int32)


def _batch_ref(sh, aux, pairs, auxidx):
    """Oracle (ab|P) per (pair, aux shell), assembled into the batch matrix."""
    ob = oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1)
    oa = oracle.Basis(aux.l, aux.nprim, aux.exps, aux.coefs, aux.centers, 1)
    nab = [(2 * sh.l[a] + 1) * (2 * sh.l[b] + 1) for a, b in pairs]
    nP = [2 * aux.l[k] + 1 for k in auxidx]
    ro, co = np.concatenate([[0], np.cumsum(nab)]), np.concatenate([[0], np.cumsum(nP)])
    B = np.zeros((ro[-1], co[-1]))
    for i, pr in enumerate(pairs):
        for k, ak in enumerate(auxidx):
            v = oracle.eri3(ob, oa, pr.reshape(1, 2), [ak])  # [1, nab, nP, 1]
            B[ro[i]:ro[i + 1], co[k]:co[k + 1]] = v[0, :, :, 0]
    return B


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_eri3_batch_mixed_classes(ctx, flags):
    """Task-list batch over all classes l_a, l_b <= 3 x l_P <= 6 in one call;
    with the graph flag the call is repeated and every replay checked."""
    import torch
    from paper_2405_01834_amd.mderi import FLAG_GRAPH
    sh, aux, pairs, auxidx = _mixed(70 + flags, 18, 14)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    a = ctx.basis(aux.l, aux.nprim, aux.exps, aux.coefs, aux.centers)
    ref = _batch_ref(sh, aux, pairs, auxidx)
    nrep = 3 if flags & FLAG_GRAPH else 2
    out = None
    for rep in range(nrep):
        if out is not None:
            out.zero_()
        Bm = ctx.eri3_batch(b, a, pairs, auxidx, flags=flags, out=out)
        out = Bm.t().view(-1) if out is None else out  # the call's buffer, reused
        torch.cuda.synchronize()
        got = Bm.cpu().numpy()
        err = np.abs(got - ref)
        bad = err > ATOL + RTOL * np.abs(ref)
        assert not bad.any(), f"rep {rep}: {bad.sum()} of {bad.size} outside tolerance; max err {err.max():.3e}"


def _class_batch_matrix(sh, aux, pairs, auxidx):
    """Oracle batch matrix for pairs of one class and aux shells of one l."""
    ob = oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1)
    oa = oracle.Basis(aux.l, aux.nprim, aux.exps, aux.coefs, aux.centers, 1)
    V = oracle.eri3(ob, oa, pairs, auxidx)  # [ij, ab, mP, k]
    npair, nab, nP, naux = V.shape
    return np.transpose(V, (0, 1, 3, 2)).reshape(npair * nab, naux * nP)


@pytest.mark.parametrize("la,lb,lP,npair,naux", [(1, 0, 1, 80, 80), (2, 1, 3, 72, 64)])
def test_eri3_batch_workgroups_loop(ctx, la, lb, lP, npair, naux):
    """One class block of more triplets (6,400 and 4,608) than the persistent
    launch has workgroups, so every workgroup runs several tasks and reuses
    its LDS; against the oracle, plain and with the graph flag."""
    import torch
    from paper_2405_01834_amd.mderi import FLAG_GRAPH
    rng = np.random.default_rng(90 + la + lP)
    sh = inputs.random_shells(rng, [la, lb] * npair, [1, 2] * npair, 8.0, 0.05, 200.0)
    aux = inputs.random_shells(rng, [lP] * naux, 1, 8.0, 0.05, 200.0)
    pairs = np.arange(2 * npair, dtype=np.int32).reshape(-1, 2)
    auxidx = np.arange(naux, dtype=np.int32)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    a = ctx.basis(aux.l, aux.nprim, aux.exps, aux.coefs, aux.centers)
    ref = _class_batch_matrix(sh, aux, pairs, auxidx)
    for flags in (0, FLAG_GRAPH, FLAG_GRAPH):
        Bm = ctx.eri3_batch(b, a, pairs, auxidx, flags=flags)
        torch.cuda.synchronize()
        got = Bm.cpu().numpy()
        err = np.abs(got - ref)
        bad = err > ATOL + RTOL * np.abs(ref)
        assert not bad.any(), f"flags {flags}: {bad.sum()} of {bad.size} outside; max err {err.max():.3e}"
