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



def test_kept_factors_follow_bases_and_geometry(need_gpu):
    """The factors a context keeps between density-fitting calls: repeated
    mderi_dfj / mderi_dfk calls on the same bases (taking the kept (ab|P),
    the metric's factor, B L^-T after a K build, and B L^-T spread over the
    AO pairs) give the oracle's J and K; moving either basis, switching to
    another basis pair and mderi_set_workspace_limit each compute them
    again (a stale factor would give the old geometry's values)."""
    import torch
    from paper_2405_01834_amd import Context
    rng = np.random.default_rng(61)
    ls, Ks, lx = [0, 1, 2, 0, 1], [2, 1, 1, 3, 2], [0, 1, 2, 0, 1, 2, 3]
    sh = inputs.random_shells(rng, ls, Ks, 3.0, 0.3, 5.0)
    ax = inputs.random_shells(rng, lx, 1, 3.0, 0.2, 4.0)
    ctx = Context(0)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    a = ctx.basis(ax.l, ax.nprim, ax.exps, ax.coefs, ax.centers)
    nao = b.nao()
    C = rng.normal(size=(nao, 3))
    Dh = C @ C.T
    D = torch.tensor(Dh, device="cuda")

    def check(got, ref):
        got = got.cpu().numpy()
        assert np.array_equal(got, got.T)
        assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))

    def refs(bsh, ash):
        ob, oa = _obasis(bsh), _obasis(ash)
        return oracle.dfj(ob, oa, Dh), oracle.dfk(ob, oa, Dh)

    Jr, Kr = refs(sh, ax)
    J1 = ctx.dfj(b, a, D)           # computes the factors
    J2 = ctx.dfj(b, a, D)           # kept (ab|P) and Cholesky factor
    K1 = ctx.dfk(b, a, D)           # B L^-T in place, spread over the AO pairs
    K2 = ctx.dfk(b, a, D)           # the two GEMMs alone
    J3 = ctx.dfj(b, a, D)           # J from B L^-T, no solve
    torch.cuda.synchronize()
    for J in (J1, J2, J3):
        check(J, Jr)
    for K in (K1, K2):
        check(K, Kr)
    assert float((J2 - J1).abs().max()) <= 1e-13 * float(J1.abs().max())
    assert float((K2 - K1).abs().max()) <= 1e-13 * float(K1.abs().max())

    # the primary basis moved
    moved = sh.centers + rng.normal(scale=0.3, size=sh.centers.shape)
    cb = torch.tensor(moved, device="cuda")
    b.set_centers(cb)
    sh_m = inputs.Shells(sh.l, sh.nprim, sh.exps, sh.coefs, moved)
    Jm_r, Km_r = refs(sh_m, ax)
    check(ctx.dfk(b, a, D), Km_r)
    check(ctx.dfj(b, a, D), Jm_r)
    # the fitting basis moved as well
    amoved = ax.centers + rng.normal(scale=0.3, size=ax.centers.shape)
    ca = torch.tensor(amoved, device="cuda")
    a.set_centers(ca)
    ax_m = inputs.Shells(ax.l, ax.nprim, ax.exps, ax.coefs, amoved)
    Jmm_r, Kmm_r = refs(sh_m, ax_m)
    check(ctx.dfj(b, a, D), Jmm_r)
    check(ctx.dfk(b, a, D), Kmm_r)
    # another basis pair, then this one again
    b2 = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    a2 = ctx.basis(ax.l, ax.nprim, ax.exps, ax.coefs, ax.centers)
    check(ctx.dfk(b2, a2, D), Kr)
    check(ctx.dfj(b, a, D), Jmm_r)
    # kept factors used from another stream (the library's calls move to it)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    Js = ctx.dfj(b, a, D, stream=side)
    Ks = ctx.dfk(b, a, D, stream=side)
    Js2 = ctx.dfj(b, a, D, stream=side)
    side.synchronize()
    check(Js, Jmm_r)
    check(Ks, Kmm_r)
    check(Js2, Jmm_r)
    # the work space (and the factors in it) freed
    ctx.set_workspace_limit(0)
    check(ctx.dfk(b, a, D), Kmm_r)
    torch.cuda.synchronize()
    del cb, ca
