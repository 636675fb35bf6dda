"""GPU nuclear gradient of the exchange energy E = tr(D K[D]) (the adjoint of
the exchange build) against the FP64 oracle, which differentiates every
ordered quartet on all four centres: max |dg| <= 1e-11 max |g|.  Also
checked: translational invariance (sum over atoms vanishes), the autograd
wrapper (dE/dR from the gradient call, dE/dD = 2K) and central finite
differences of the GPU energy."""
import numpy as np
import pytest

import oracle
from paper_2405_01834_amd import inputs

pytestmark = pytest.mark.gpu

CASES = [
    (11, 2, ((0, 2), (1, 1), (2, 1)), 2.5),
    (12, 3, ((0, 1), (1, 2), (2, 1), (3, 1)), 3.0),
    (13, 2, ((1, 1), (4, 1), (2, 2)), 2.0),
]


@pytest.fixture(scope="module")
def ctx(need_gpu):
    from paper_2405_01834_amd import Context
    return Context(0)


def _molecule(seed, natom, shells, spread):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, spread, (natom, 3))
    ls, Ks, atom = [], [], []
    for a in range(natom):
        for l, k in shells:
            ls.append(l)
            Ks.append(k)
            atom.append(a)
    sh = inputs.random_shells(rng, ls, Ks, 1.0, 0.1, 30.0)
    atom = np.array(atom, dtype=np.int32)
    sh.centers = pos[atom]
    return sh, pos, atom


def _density(seed, nao):
    rng = np.random.default_rng(seed + 100)
    C = rng.normal(size=(nao, 4)) / np.sqrt(nao)
    return C @ C.T


@pytest.mark.parametrize("seed,natom,shells,spread", CASES)
def test_kgrad_parity(ctx, seed, natom, shells, spread):
    import torch
    sh, pos, atom = _molecule(seed, natom, shells, spread)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, atom=atom)
    D = _density(seed, b.nao())
    g = ctx.kbuild_grad(b, torch.tensor(D, device="cuda"), natom, tau=1e-12)
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    ref = oracle.exchange_grad(oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1), atom, natom, D,
                               tau=1e-12)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-11 * scale, (got, ref)
    assert np.max(np.abs(got.sum(axis=0))) <= 1e-11 * scale


def test_kgrad_autograd_and_fd(ctx):
    import torch
    from paper_2405_01834_amd.mderi import exchange_energy
    seed, natom, shells, spread = CASES[1]
    sh, pos, atom = _molecule(seed, natom, shells, spread)
    # the autograd function moves the shells of its own basis to the
    # coordinates on the device (mderi_basis_set_centers)
    spec = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers + 1.0, atom=atom)
    nao = spec.nao()
    D0 = _density(seed, nao)
    coords = torch.tensor(pos, device="cuda", requires_grad=True)
    D = torch.tensor(D0, device="cuda", requires_grad=True)
    E = exchange_energy(ctx, coords, D, spec)
    E.backward()
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, atom=atom)
    K = ctx.kbuild(b, torch.tensor(D0, device="cuda"))
    g = ctx.kbuild_grad(b, torch.tensor(D0, device="cuda"), natom)
    torch.cuda.synchronize()
    assert abs(E.item() - float((D0 * K.cpu().numpy()).sum())) <= 1e-13 * abs(E.item())
    # same kernels; FP64 atomics may sum in another order
    gn = g.cpu().numpy()
    assert np.max(np.abs(coords.grad.cpu().numpy() - gn)) <= 1e-13 * np.max(np.abs(gn))
    assert np.max(np.abs(D.grad.cpu().numpy() - 2.0 * K.cpu().numpy())) <= 1e-14 * np.max(np.abs(K.cpu().numpy()))
    # central differences of the GPU energy, error O(h^2)
    h = 1e-4
    gd = g.cpu().numpy()
    for a, x in ((0, 0), (1, 2), (2, 1)):
        e = []
        for sgn in (1.0, -1.0):
            p = pos.copy()
            p[a, x] += sgn * h
            cp = torch.tensor(p, device="cuda")
            e.append(exchange_energy(ctx, cp, torch.tensor(D0, device="cuda"), spec).item())
        fd = (e[0] - e[1]) / (2 * h)
        assert abs(fd - gd[a, x]) <= 1e-6 * np.max(np.abs(gd)), (a, x, fd, gd[a, x])
