"""GPU density-fitted Coulomb and exchange matrices (mderi_dfj, mderi_dfk:
(ab|P) task list, metric class batches, Cholesky factor of the Coulomb
metric, solves and contractions) against the oracle's dense assemblies
(oracle.dfj, oracle.dfk): max |d| <= 1e-10 of the largest element (the solve
carries the metric's condition number, below 1e2 for these fitting sets, on
top of the 1e-12 integral parity), exact symmetry; and the exact J and K
(the oracle's brute force) when the fitting set holds the pair products of s
shells."""
import numpy as np
import pytest

import oracle
from paper_2405_01834_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(need_gpu):
    from paper_2405_01834_amd import Context
    return Context(0)


def _obasis(sh):
    return oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1)


@pytest.mark.parametrize("seed,ls,Ks,lx", [(1, [0, 1, 2, 0, 1], [2, 1, 1, 3, 2], [0, 1, 2, 0, 1, 2, 3]),
                                           (2, [2, 3, 1, 1], [1, 1, 2, 1], [0, 0, 1, 2, 2, 3, 4, 1])])
def test_dfj_matches_oracle(ctx, seed, ls, Ks, lx):
    import torch
    rng = np.random.default_rng(seed)
    sh = inputs.random_shells(rng, ls, Ks, 3.0, 0.3, 5.0)
    ax = inputs.random_shells(rng, lx, 1, 3.0, 0.2, 4.0)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    a = ctx.basis(ax.l, ax.nprim, ax.exps, ax.coefs, ax.centers)
    nao = b.nao()
    C = rng.normal(size=(nao, 3))
    D = C @ C.T
    J = ctx.dfj(b, a, torch.tensor(D, device="cuda"))
    torch.cuda.synchronize()
    got = J.cpu().numpy()
    ref = oracle.dfj(_obasis(sh), _obasis(ax), D)
    assert np.array_equal(got, got.T)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_dfj_exact_with_product_fitting_set(ctx):
    """s shells of single primitives with their pair products (exponent
    a_i + a_j at P_ij) as the fitting set: the fit is exact, J equals the
    brute-force J."""
    import torch
    rng = np.random.default_rng(31)
    n = 4
    ex = np.exp(rng.uniform(np.log(0.3), np.log(3.0), n))
    cen = rng.uniform(-1.0, 1.0, (n, 3))
    b = ctx.basis(np.zeros(n, np.int32), np.ones(n, np.int32), ex, np.ones(n), cen)
    pe, pc = [], []
    for i in range(n):
        for j in range(i, n):
            pe.append(ex[i] + ex[j])
            pc.append((ex[i] * cen[i] + ex[j] * cen[j]) / (ex[i] + ex[j]))
    m = len(pe)
    a = ctx.basis(np.zeros(m, np.int32), np.ones(m, np.int32), np.array(pe), np.ones(m), np.array(pc))
    C = rng.normal(size=(n, n))
    D = C @ C.T
    J = ctx.dfj(b, a, torch.tensor(D, device="cuda"))
    torch.cuda.synchronize()
    ref = oracle.jbuild(oracle.Basis([0] * n, [1] * n, ex, np.ones(n), cen, 1), D)
    assert np.max(np.abs(J.cpu().numpy() - ref)) <= 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed,ls,Ks,lx", [(1, [0, 1, 2, 0, 1], [2, 1, 1, 3, 2], [0, 1, 2, 0, 1, 2, 3]),
                                           (2, [2, 3, 1, 1], [1, 1, 2, 1], [0, 0, 1, 2, 2, 3, 4, 1])])
def test_dfk_matches_oracle(ctx, seed, ls, Ks, lx):
    """Density-fitted K against the oracle's dense assembly (1e-10 of max |K|,
    the solve's condition number on top of the integral parity); exactly
    symmetric."""
    import torch
    rng = np.random.default_rng(seed)
    sh = inputs.random_shells(rng, ls, Ks, 3.0, 0.3, 5.0)
    ax = inputs.random_shells(rng, lx, 1, 3.0, 0.2, 4.0)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    a = ctx.basis(ax.l, ax.nprim, ax.exps, ax.coefs, ax.centers)
    nao = b.nao()
    C = rng.normal(size=(nao, 3))
    D = C @ C.T
    K = ctx.dfk(b, a, torch.tensor(D, device="cuda"))
    torch.cuda.synchronize()
    got = K.cpu().numpy()
    ref = oracle.dfk(_obasis(sh), _obasis(ax), D)
    assert np.array_equal(got, got.T)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_dfk_exact_with_product_fitting_set(ctx):
    """s shells of single primitives with their pair products as the fitting
    set: the fitted integrals are exact, K equals the brute-force K; an
    unsymmetric-looking but symmetric D of mixed signs."""
    import torch
    rng = np.random.default_rng(35)
    n = 4
    ex = np.exp(rng.uniform(np.log(0.3), np.log(3.0), n))
    cen = rng.uniform(-1.0, 1.0, (n, 3))
    b = ctx.basis(np.zeros(n, np.int32), np.ones(n, np.int32), ex, np.ones(n), cen)
    pe, pc = [], []
    for i in range(n):
        for j in range(i, n):
            pe.append(ex[i] + ex[j])
            pc.append((ex[i] * cen[i] + ex[j] * cen[j]) / (ex[i] + ex[j]))
    m = len(pe)
    a = ctx.basis(np.zeros(m, np.int32), np.ones(m, np.int32), np.array(pe), np.ones(m), np.array(pc))
    X = rng.normal(size=(n, n))
    D = X + X.T
    K = ctx.dfk(b, a, torch.tensor(D, device="cuda"))
    torch.cuda.synchronize()
    ref = oracle.kbuild(oracle.Basis([0] * n, [1] * n, ex, np.ones(n), cen, 1), D)
    assert np.max(np.abs(K.cpu().numpy() - ref)) <= 1e-9 * np.max(np.abs(ref))

