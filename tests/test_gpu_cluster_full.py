"""The synthetic cluster at its full size, 150 atoms (per atom s4 p3 d2 f1 g1,
K = 1, exponents geometric 0.08-2000, atoms >= 2 bohr apart in a 30-bohr
box, rank-100 PSD density, Schwarz 1e-12): the K build, the J+K build and
the exchange gradient end to end on the GPU, checked
  * on sampled shell blocks of K and J against the oracle's brute force
    restricted to the quartets feeding them (1e-12 of max |K| / max |J|),
    blocks on one atom, on neighbouring atoms and at random;
  * by translational invariance of the gradient (1e-10 of max |g|);
  * by a central difference of tr(D K) along a random direction
    (h = 1e-4, 1e-6 of max |g|).
The run takes minutes of GPU time and about a minute of oracle time, so it is
collected only with MDERI_FULL_CLUSTER=1; the default GPU suite checks the
same paths on the 24-atom cluster (test_gpu_jk.py)."""
import os
import time

import numpy as np
import pytest

import oracle
from paper_2405_01834_amd import inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("MDERI_FULL_CLUSTER") != "1",
                                 reason="full-size cluster run (minutes); set MDERI_FULL_CLUSTER=1")]

TAU = 1e-12
NATOM = int(os.environ.get("MDERI_CLUSTER_ATOMS", "150"))


def _log(msg):
    print(msg, flush=True)


def _blocks(sh, atom, pos, rng):
    """Shell blocks (s0, s1): three on one atom, three on nearest-neighbour
    atoms, two at random."""
    by_atom = [np.flatnonzero(atom == a) for a in range(len(pos))]
    out = []
    for _ in range(3):
        a = rng.integers(len(pos))
        s0, s1 = rng.choice(by_atom[a], 2)
        out.append((int(s0), int(s1)))
    for _ in range(3):
        a = rng.integers(len(pos))
        d = np.linalg.norm(pos - pos[a], axis=1)
        d[a] = np.inf
        b = int(np.argmin(d))
        out.append((int(rng.choice(by_atom[a])), int(rng.choice(by_atom[b]))))
    for _ in range(2):
        s0, s1 = rng.choice(sh.n, 2)
        out.append((int(s0), int(s1)))
    return out


def test_full_cluster_k_j_gradient(need_gpu):
    import torch
    from paper_2405_01834_amd import Context
    ctx = Context(0)
    ctx.progress(True)
    sh, atom, pos, D = inputs.cluster(7, NATOM)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, atom=atom)
    Dd = torch.tensor(D, device="cuda")
    _log(f"cluster {NATOM} atoms, {sh.n} shells, {b.nao()} AOs")

    def timed(label, fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        _log(f"{label}: {time.perf_counter() - t:.1f} s")
        return r

    K = timed("K build", lambda: ctx.kbuild(b, Dd, tau=TAU))
    g = timed("exchange gradient", lambda: ctx.kbuild_grad(b, Dd, NATOM, tau=TAU))
    J, K2, E = timed("J+K build with energies", lambda: ctx.jkbuild(b, Dd, tau=TAU, energies=True))
    Kn, Jn, gn = K.cpu().numpy(), J.cpu().numpy(), g.cpu().numpy()
    e0 = float(E[1].item())
    kscale = np.max(np.abs(Kn))
    assert np.max(np.abs(K2.cpu().numpy() - Kn)) <= 1e-13 * kscale
    assert abs(e0 - float(np.sum(D * Kn))) <= 1e-12 * abs(e0)

    res = np.max(np.abs(gn.sum(axis=0))) / np.max(np.abs(gn))
    _log(f"translational residual {res:.2e}")
    assert res <= 1e-10

    direction = np.random.default_rng(6).normal(size=(NATOM, 3))
    direction /= np.linalg.norm(direction)
    h = 1e-4
    e = []
    for sgn in (1.0, -1.0):
        p = pos + sgn * h * direction
        b.set_centers(torch.tensor(p[atom], device="cuda"))
        _, _, Ep = timed(f"K build at {'+' if sgn > 0 else '-'}h", lambda: ctx.jkbuild(
            b, Dd, want_j=False, tau=TAU, energies=True))
        e.append(float(Ep[1].item()))
    b.set_centers(torch.tensor(pos[atom], device="cuda"))
    fd = (e[0] - e[1]) / (2 * h)
    an = float(np.sum(gn * direction))
    _log(f"directional derivative: analytic {an:.12e} central difference {fd:.12e} "
         f"(diff {abs(fd - an):.2e}, max |g| {np.max(np.abs(gn)):.3e})")
    assert abs(fd - an) <= 1e-6 * np.max(np.abs(gn))

    ao = np.concatenate([[0], np.cumsum(2 * sh.l + 1)])
    blocks = _blocks(sh, atom, pos, np.random.default_rng(5))
    ob = oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1)
    for which, M in (("K", Kn), ("J", Jn)):
        t = time.perf_counter()
        ref = oracle.fock_blocks(ob, D, blocks, which=which, tau=TAU)
        scale = np.max(np.abs(M))
        worst = 0.0
        for (s0, s1), r in zip(blocks, ref):
            got = M[ao[s0]:ao[s0 + 1], ao[s1]:ao[s1 + 1]]
            worst = max(worst, float(np.max(np.abs(got - r))) / scale)
        _log(f"{which}: {len(blocks)} sampled shell blocks against the oracle in {time.perf_counter() - t:.1f} s, "
             f"max |d| / max |{which}| = {worst:.2e}")
        assert worst <= 1e-12
