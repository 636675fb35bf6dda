"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  This module draws random numbers only; it contains none of the
integral arithmetic (screening, which needs integrals, is done by whichever
side consumes the candidates).

Workloads (stand-ins for the random shells of Sec. 5 and the molecules of
Sec. 6, none of which ship with the paper):
  * pp_quartets  -- 16 bra x 32 ket [pp] pairs, K=1, centres U[0,10)^3,
                    exponents log-uniform in [0.1, 100], seed 0.
  * class_pairs  -- candidate shell pairs of one class for the l-class batches:
                    centres U[0,20)^3, exponents log-uniform in [0.05, 500],
                    coefficients U[0.1, 1], K primitives per shell.
  * eri3_batch   -- 3-centre task list: `npair` primary pairs with l_a, l_b
                    uniform in 0..3 and K uniform in 1..5 per shell, `naux`
                    auxiliary shells with l_P uniform in 0..6 and K=1; centres
                    U[0,20)^3, exponents log-uniform in [0.05, 500],
                    coefficients U[0.1, 1].
  * cluster      -- atoms at least 2 bohr apart, drawn uniformly in a box
                    whose side scales as 30 bohr x (natom / 150)^(1/3) (the
                    density of a 150-atom cluster in a 30-bohr box); per atom
                    the shells s4 p3 d2 f1 g1, K=1, exponents of the n shells
                    of one l geometric from 0.08 to 2000 (a single shell takes
                    the geometric mean); symmetric PSD density of rank 100
                    (or nao if smaller), D = C C^T with C ~ N(0, 1/nao).
Draw order per shell: centre (3 uniforms), K exponents, K coefficients.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Shells:
    l: np.ndarray        # int32 [n]
    nprim: np.ndarray    # int32 [n]
    exps: np.ndarray     # float64 [sum nprim]
    coefs: np.ndarray    # float64 [sum nprim]
    centers: np.ndarray  # float64 [n, 3]

    @property
    def n(self):
        return len(self.l)

    def concat(self, other: "Shells") -> "Shells":
        return Shells(np.concatenate([self.l, other.l]), np.concatenate([self.nprim, other.nprim]),
                      np.concatenate([self.exps, other.exps]), np.concatenate([self.coefs, other.coefs]),
                      np.concatenate([self.centers, other.centers]))

    def subset(self, idx) -> "Shells":
        idx = np.asarray(idx)
        off = np.concatenate([[0], np.cumsum(self.nprim)])
        sel = np.concatenate([np.arange(off[i], off[i + 1]) for i in idx]) if len(idx) else np.zeros(0, int)
        return Shells(self.l[idx].copy(), self.nprim[idx].copy(), self.exps[sel].copy(), self.coefs[sel].copy(),
                      self.centers[idx].copy())


def random_shells(rng: np.random.Generator, ls, K, box, exp_lo, exp_hi, coef_lo=0.1, coef_hi=1.0) -> Shells:
    """One shell per entry of `ls` (K int or per-shell list)."""
    ls = np.asarray(ls, dtype=np.int32)
    Ks = np.full(len(ls), K, dtype=np.int32) if np.isscalar(K) else np.asarray(K, dtype=np.int32)
    cen, ex, co = [], [], []
    for i in range(len(ls)):
        cen.append(rng.uniform(0.0, box, 3))
        ex.append(np.exp(rng.uniform(np.log(exp_lo), np.log(exp_hi), Ks[i])))
        co.append(rng.uniform(coef_lo, coef_hi, Ks[i]) if Ks[i] > 1 else np.ones(1))
    return Shells(ls, Ks, np.concatenate(ex), np.concatenate(co), np.array(cen).reshape(-1, 3))


def pp_quartets(seed: int = 0, nbra: int = 16, nket: int = 32):
    """[pp|pp] K=1: returns (shells, bra_pairs, ket_pairs)."""
    rng = np.random.default_rng(seed)
    n = 2 * (nbra + nket)
    sh = random_shells(rng, [1] * n, 1, 10.0, 0.1, 100.0)
    pairs = np.arange(n, dtype=np.int32).reshape(-1, 2)
    return sh, pairs[:nbra].copy(), pairs[nbra:].copy()


def class_pairs(seed: int, la: int, lb: int, K: int, npairs: int, box: float = 20.0, exp_lo: float = 0.05,
                exp_hi: float = 500.0):
    """`npairs` candidate pairs (shell 2i, shell 2i+1) of class (la, lb) with K
    primitives per shell.  Returns (shells, pairs)."""
    rng = np.random.default_rng(seed)
    ls = [la, lb] * npairs
    sh = random_shells(rng, ls, K, box, exp_lo, exp_hi)
    return sh, np.arange(2 * npairs, dtype=np.int32).reshape(-1, 2)


def near_pairs(seed: int, la: int, lb: int, K: int, npairs: int, box: float = 20.0, sep: float = 1.5,
               exp_lo: float = 0.05, exp_hi: float = 500.0):
    """Candidate pairs whose second shell sits within `sep` bohr of the first
    (cheap way to draw pairs most of which survive screening)."""
    rng = np.random.default_rng(seed)
    cen, ex, co, ls, Ks = [], [], [], [], []
    for _ in range(npairs):
        c0 = rng.uniform(0.0, box, 3)
        d = rng.normal(size=3)
        d *= rng.uniform(0.0, sep) / max(np.linalg.norm(d), 1e-12)
        for l, c in ((la, c0), (lb, c0 + d)):
            cen.append(c)
            ex.append(np.exp(rng.uniform(np.log(exp_lo), np.log(exp_hi), K)))
            co.append(rng.uniform(0.1, 1.0, K) if K > 1 else np.ones(1))
            ls.append(l)
            Ks.append(K)
    sh = Shells(np.array(ls, np.int32), np.array(Ks, np.int32), np.concatenate(ex), np.concatenate(co),
                np.array(cen))
    return sh, np.arange(2 * npairs, dtype=np.int32).reshape(-1, 2)


CLUSTER_SHELLS = ((0, 4), (1, 3), (2, 2), (3, 1), (4, 1))  # (l, shells per atom)


def cluster(seed: int, natom: int, min_dist: float = 2.0, rank: int = 100):
    """Synthetic molecular cluster.  Returns (shells, atom_of_shell, positions, D)."""
    rng = np.random.default_rng(seed)
    box = 30.0 * (natom / 150.0) ** (1.0 / 3.0)
    pos = []
    while len(pos) < natom:
        x = rng.uniform(0.0, box, 3)
        if all(np.linalg.norm(x - y) >= min_dist for y in pos):
            pos.append(x)
    pos = np.array(pos)
    ls, ex, atom = [], [], []
    for a in range(natom):
        for l, n in CLUSTER_SHELLS:
            e = [np.sqrt(0.08 * 2000.0)] if n == 1 else np.geomspace(0.08, 2000.0, n)
            for z in e:
                ls.append(l)
                ex.append(z)
                atom.append(a)
    ls = np.array(ls, np.int32)
    atom = np.array(atom, np.int32)
    sh = Shells(ls, np.ones(len(ls), np.int32), np.array(ex), np.ones(len(ls)), pos[atom])
    nao = int(np.sum(2 * ls + 1))
    C = rng.normal(size=(nao, min(rank, nao))) / np.sqrt(nao)
    return sh, atom, pos, C @ C.T


def eri3_batch(seed: int, npair: int = 512, naux: int = 512):
    """Mixed-class 3-centre workload.  Returns (primary shells, aux shells, pairs, aux indices)."""
    rng = np.random.default_rng(seed)
    ls = rng.integers(0, 4, 2 * npair)
    Ks = rng.integers(1, 6, 2 * npair)
    prim = random_shells(rng, ls, Ks, 20.0, 0.05, 500.0)
    aux = random_shells(rng, rng.integers(0, 7, naux), 1, 20.0, 0.05, 500.0)
    return prim, aux, np.arange(2 * npair, dtype=np.int32).reshape(-1, 2), np.arange(naux, dtype=np.int32)
