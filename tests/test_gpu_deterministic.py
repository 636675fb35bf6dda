"""The deterministic mode of the J and K builds (opts.deterministic = 1:
fixed-point images added by 64-bit integer atomics, whose sums do not depend
on the order in which the waves add them):
  * two runs on the 12-atom synthetic cluster (per atom s4 p3 d2 f1 g1,
    hundreds of thousands of quartets racing on shared elements) give the
    same bits, J and K exactly symmetric;
  * they agree with the FP64-atomic path within 1e-13 of max |K| / max |J|
    (the fixed-point rounding, B 2^-95 per image, is far below that);
  * on a small molecule they match the oracle's brute force at 1e-12;
  * a density of zeros gives zeros; values other than 0 and 1 are rejected;
  * the gradient in the same mode (four-digit fixed point): bitwise
    repeatable and within 1e-12 of the FP64-atomic gradient.
Also the workspace cap (mderi_set_workspace_limit), the way to make the
library's allocation failures (MDERI_ENOMEM) happen on purpose."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2405_01834_amd import inputs

pytestmark = pytest.mark.gpu

TAU = 1e-12


@pytest.fixture(scope="module")
def ctx(need_gpu):
    from paper_2405_01834_amd import Context
    return Context(0)


@pytest.fixture(scope="module")
def cluster(ctx):
    import torch
    sh, atom, pos, D = inputs.cluster(7, 12)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, atom=atom)
    return b, torch.tensor(D, device="cuda")


def test_deterministic_repeats_bitwise(ctx, cluster):
    import torch
    b, D = cluster
    J1, K1 = ctx.jkbuild(b, D, tau=TAU, deterministic=True)
    J2, K2 = ctx.jkbuild(b, D, tau=TAU, deterministic=True)
    K3 = ctx.kbuild(b, D, tau=TAU, deterministic=True)
    J3, _ = ctx.jkbuild(b, D, want_k=False, tau=TAU, deterministic=True)  # J alone: its own buffer layout
    torch.cuda.synchronize()
    assert torch.equal(K1, K2) and torch.equal(J1, J2) and torch.equal(K1, K3) and torch.equal(J1, J3)
    assert torch.equal(K1, K1.T) and torch.equal(J1, J1.T)


def test_deterministic_agrees_with_atomic(ctx, cluster):
    import torch
    b, D = cluster
    Jd, Kd = ctx.jkbuild(b, D, tau=TAU, deterministic=True)
    Ja, Ka = ctx.jkbuild(b, D, tau=TAU)
    torch.cuda.synchronize()
    for got, ref in ((Kd, Ka), (Jd, Ja)):
        scale = float(ref.abs().max())
        assert scale > 0.0
        assert float((got - ref).abs().max()) <= 1e-13 * scale


def test_deterministic_matches_oracle(ctx):
    import torch
    rng = np.random.default_rng(41)
    ls, Ks = [0, 1, 2, 3, 0, 2, 1], [2, 1, 1, 1, 3, 2, 1]
    sh = inputs.random_shells(rng, ls, Ks, 3.0, 0.1, 30.0)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    nao = b.nao()
    C = rng.normal(size=(nao, 4))
    D = C @ C.T
    J, K = ctx.jkbuild(b, torch.tensor(D, device="cuda"), tau=TAU, deterministic=True)
    torch.cuda.synchronize()
    ob = oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1)
    for got, ref in ((K.cpu().numpy(), oracle.kbuild(ob, D)), (J.cpu().numpy(), oracle.jbuild(ob, D))):
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_deterministic_zero_density(ctx, cluster):
    import torch
    b, D = cluster
    J, K = ctx.jkbuild(b, torch.zeros_like(D), tau=TAU, deterministic=True)
    torch.cuda.synchronize()
    assert not bool(J.any()) and not bool(K.any())


def test_deterministic_refused_where_unsupported(ctx, cluster):
    import torch
    from paper_2405_01834_amd.mderi import MderiError, Opts, load_library, _check
    b, D = cluster
    nao = b.nao()
    K = torch.empty_like(D)
    g = torch.empty((12, 3), dtype=torch.float64, device="cuda")
    lib = load_library()
    vp = ctypes.c_void_p
    with pytest.raises(MderiError):
        _check(lib.mderi_kbuild(ctx._h, b._h, vp(D.data_ptr()), vp(K.data_ptr()), nao,
                                ctypes.byref(Opts(0, TAU, 0, 0, 0, 2)), None))
    with pytest.raises(MderiError):
        _check(lib.mderi_kbuild_grad(ctx._h, b._h, 0, vp(D.data_ptr()), vp(D.data_ptr()), nao,
                                     ctypes.c_double(1.0), vp(g.data_ptr()), 12, 0,
                                     ctypes.byref(Opts(0, TAU, 0, 0, 0, 5)), None))


def test_deterministic_gradient(ctx, cluster):
    """The exchange gradient in the deterministic mode: two runs give the
    same bits; it agrees with the FP64-atomic gradient within 1e-12 of max |g|
    (the 2^-80 steps of the fixed point are far below that), and a Coulomb
    pattern with unsymmetric weights and accumulate as well."""
    import torch
    b, D = cluster
    g1 = ctx.kbuild_grad(b, D, 12, tau=TAU, deterministic=True)
    g2 = ctx.kbuild_grad(b, D, 12, tau=TAU, deterministic=True)
    ga = ctx.kbuild_grad(b, D, 12, tau=TAU)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    assert float((g1 - ga).abs().max()) <= 1e-12 * float(ga.abs().max())
    rng = np.random.default_rng(44)
    W = torch.tensor(rng.normal(size=tuple(D.shape)), device="cuda")
    base = torch.tensor(rng.normal(size=(12, 3)), device="cuda")
    outs = []
    for det in (True, True, False):
        o = base.clone()
        ctx.kbuild_grad(b, D, 12, Wr=W, pattern=1, scale=0.5, tau=TAU, out=o, accumulate=True, deterministic=det)
        outs.append(o)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    scale = float((outs[2] - base).abs().max())
    assert float((outs[0] - outs[2]).abs().max()) <= 1e-12 * scale


def test_workspace_limit_gives_enomem_and_recovers(need_gpu):
    """A workspace cap below what a call needs: MDERI_ENOMEM (status -2) from
    the K build, the 4-centre batch and the gradient; after the cap is lifted
    the same context gives the results of an uncapped one."""
    import torch
    from paper_2405_01834_amd import Context
    from paper_2405_01834_amd.mderi import MderiError
    rng = np.random.default_rng(43)
    sh = inputs.random_shells(rng, [0, 1, 2, 1, 0], [2, 1, 1, 2, 1], 3.0, 0.1, 30.0)
    nao = int(np.sum(2 * sh.l + 1))
    C = rng.normal(size=(nao, 3))
    D = torch.tensor(C @ C.T, device="cuda")
    ref_ctx = Context(0)
    rb = ref_ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    K_ref = ref_ctx.kbuild(rb, D, tau=TAU)
    V_ref = ref_ctx.eri4(rb, [[2, 2], [2, 2]], [[3, 1]])
    ctx = Context(0)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    ctx.set_workspace_limit(256)
    for call in (lambda: ctx.kbuild(b, D, tau=TAU), lambda: ctx.eri4(b, [[2, 2], [2, 2]], [[3, 1]]),
                 lambda: ctx.kbuild_grad(b, D, len(sh.l), tau=TAU)):
        with pytest.raises(MderiError) as e:
            call()
        assert e.value.status == -2 and "limit" in str(e.value)
    torch.cuda.synchronize()
    ctx.set_workspace_limit(0)
    K = ctx.kbuild(b, D, tau=TAU)
    V = ctx.eri4(b, [[2, 2], [2, 2]], [[3, 1]])
    torch.cuda.synchronize()
    assert float((K - K_ref).abs().max()) <= 1e-13 * float(K_ref.abs().max())
    assert torch.equal(V, V_ref)
