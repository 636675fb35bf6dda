"""FP64 CPU oracle for McMurchie-Davidson 3-/4-centre Coulomb integrals.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2405_01834_amd``) and the GPU library never
imports it.

This module is a thin ctypes wrapper around ``liboracle.so`` (built from
``oracle.c`` by :func:`build`); every function of the method lives in the C
source, which cites the equations of Sec. 2 of the paper that it follows.

Basis arrays use the same plain convention as the GPU boundary: ``l[nshell]``,
``nprim[nshell]``, concatenated ``exps`` / ``coefs`` and ``centers[nshell, 3]``
in bohr.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

ORACLE_LMAX = 8  # public shells; derivatives use l+1 internally


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-shared", "-fPIC", "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_SO)
        _setup(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _setup(L):
    L.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
    L.oracle_E2.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, _dp]
    L.oracle_E1.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
    L.oracle_R.argtypes = [ctypes.c_int, ctypes.c_double, _dp, ctypes.c_double, _dp]
    L.oracle_solid.argtypes = [ctypes.c_int, _dp]
    L.oracle_norm_coefs.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp]
    basis = [ctypes.c_int, _ip, _ip, _dp, _dp, _dp, ctypes.c_int]
    L.oracle_eri4_cart.argtypes = basis + [ctypes.c_int] * 4 + [_dp]
    L.oracle_eri4_deriv.argtypes = basis + [ctypes.c_int] * 4 + [_dp]
    L.oracle_eri4.argtypes = basis + [ctypes.c_int, _ip, ctypes.c_int, _ip, _dp, ctypes.c_int]
    L.oracle_eri3.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, _dp, ctypes.c_int, _ip, _ip, _dp, _dp, _dp,
                              ctypes.c_int, ctypes.c_int, _ip, ctypes.c_int, _ip, _dp, ctypes.c_int]
    L.oracle_schwarz.argtypes = basis + [ctypes.c_int, _ip, _dp, ctypes.c_int]
    L.oracle_eri2.argtypes = basis + [ctypes.c_int, _ip, ctypes.c_int, _ip, _dp, ctypes.c_int]
    L.oracle_kbuild.argtypes = basis + [_dp, ctypes.c_double, _dp, ctypes.c_int]
    L.oracle_exchange_grad.argtypes = basis + [_ip, ctypes.c_int, _dp, ctypes.c_double, _dp, ctypes.c_int]
    L.oracle_jbuild.argtypes = basis + [_dp, ctypes.c_double, _dp, ctypes.c_int]
    L.oracle_fock_blocks.argtypes = basis + [_dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _ip, _dp,
                                             ctypes.c_int]
    L.oracle_grad_pattern.argtypes = basis + [_ip, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_double, _dp,
                                              ctypes.c_int]
    for name in ("oracle_jbuild", "oracle_fock_blocks", "oracle_grad_pattern", "oracle_eri2"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("oracle_eri4_cart", "oracle_eri4_deriv", "oracle_eri4", "oracle_eri3", "oracle_schwarz",
                 "oracle_kbuild", "oracle_exchange_grad"):
        getattr(L, name).restype = ctypes.c_int


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def nsph(l):
    return 2 * l + 1


def ncart(l):
    return (l + 1) * (l + 2) // 2


class Basis:
    """Plain container for a shell list (host arrays)."""

    def __init__(self, l, nprim, exps, coefs, centers, normalize=1):
        self.l = np.ascontiguousarray(l, dtype=np.int32)
        self.nprim = np.ascontiguousarray(nprim, dtype=np.int32)
        self.exps = np.ascontiguousarray(exps, dtype=np.float64)
        self.coefs = np.ascontiguousarray(coefs, dtype=np.float64)
        self.centers = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        self.normalize = int(normalize)
        assert self.l.shape == self.nprim.shape == (self.centers.shape[0],)
        assert self.exps.shape == self.coefs.shape == (int(self.nprim.sum()),)

    @property
    def nshell(self):
        return int(self.l.shape[0])

    def args(self):
        return (self.nshell, self.l.ctypes.data_as(_ip), self.nprim.ctypes.data_as(_ip),
                self.exps.ctypes.data_as(_dp), self.coefs.ctypes.data_as(_dp),
                self.centers.ctypes.data_as(_dp), self.normalize)

    def nao(self):
        return int(np.sum(2 * self.l + 1))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with code {rc}")


def boys(mmax: int, T: float) -> np.ndarray:
    F = np.zeros(mmax + 1)
    lib().oracle_boys(mmax, float(T), F.ctypes.data_as(_dp))
    return F


def E2(la, lb, za, zb, Ax, Bx) -> np.ndarray:
    E = np.zeros((la + 1, lb + 1, la + lb + 1))
    lib().oracle_E2(la, lb, za, zb, Ax, Bx, E.ctypes.data_as(_dp))
    return E


def E1(la, za) -> np.ndarray:
    E = np.zeros((la + 1, la + 1))
    lib().oracle_E1(la, za, E.ctypes.data_as(_dp))
    return E


def R(L, rho, PQ, pref=1.0) -> np.ndarray:
    out = np.zeros((L + 1, L + 1, L + 1))
    pq, pqp = _d(PQ)
    lib().oracle_R(L, rho, pqp, pref, out.ctypes.data_as(_dp))
    return out


def solid(l) -> np.ndarray:
    C = np.zeros((nsph(l), ncart(l)))
    lib().oracle_solid(l, C.ctypes.data_as(_dp))
    return C


def cart_list(l):
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


def norm_coefs(l, exps, coefs, normalize=1) -> np.ndarray:
    z, zp = _d(exps)
    c, cp = _d(coefs)
    out = np.zeros(len(z))
    lib().oracle_norm_coefs(l, len(z), zp, cp, normalize, out.ctypes.data_as(_dp))
    return out


def eri4_cart(basis: Basis, i, j, k, m) -> np.ndarray:
    ls = [int(basis.l[x]) for x in (i, j, k, m)]
    out = np.zeros([ncart(x) for x in ls])
    _check(lib().oracle_eri4_cart(*basis.args(), i, j, k, m, out.ctypes.data_as(_dp)), "oracle_eri4_cart")
    return out


def eri4_deriv(basis: Basis, i, j, k, m) -> np.ndarray:
    """out[centre, xyz, ma, mb, mc, md]."""
    ls = [int(basis.l[x]) for x in (i, j, k, m)]
    out = np.zeros([4, 3] + [nsph(x) for x in ls])
    _check(lib().oracle_eri4_deriv(*basis.args(), i, j, k, m, out.ctypes.data_as(_dp)), "oracle_eri4_deriv")
    return out


def eri4(basis: Basis, bra, ket, nthreads=0) -> np.ndarray:
    """Class batch, returned as V[ij, ab, cd, kl] (numpy shape (nbra, Nab, Ncd, nket), Fortran order)."""
    bra, brap = _i(np.asarray(bra).reshape(-1, 2))
    ket, ketp = _i(np.asarray(ket).reshape(-1, 2))
    la, lb = int(basis.l[bra[0, 0]]), int(basis.l[bra[0, 1]])
    lc, ld = int(basis.l[ket[0, 0]]), int(basis.l[ket[0, 1]])
    nab, ncd = nsph(la) * nsph(lb), nsph(lc) * nsph(ld)
    V = np.zeros(len(bra) * nab * ncd * len(ket))
    _check(lib().oracle_eri4(*basis.args(), len(bra), brap, len(ket), ketp, V.ctypes.data_as(_dp), nthreads),
           "oracle_eri4")
    return V.reshape((len(bra), nab, ncd, len(ket)), order="F")


def eri4_shellset(basis: Basis, i, j, k, m) -> np.ndarray:
    """One shell quartet as [ma, mb, mc, md]."""
    V = eri4(basis, [[i, j]], [[k, m]], nthreads=1)
    ls = [int(basis.l[x]) for x in (i, j, k, m)]
    return V[0, :, :, 0].reshape([nsph(x) for x in ls])


def eri3(basis: Basis, aux: Basis, pairs, auxidx, nthreads=0) -> np.ndarray:
    """(ab|P) batch as V[ij, ab, mP, k] (shape (npair, Nab, NP, naux), Fortran order)."""
    pairs, pp = _i(np.asarray(pairs).reshape(-1, 2))
    auxidx, ap = _i(np.asarray(auxidx).reshape(-1))
    la, lb = int(basis.l[pairs[0, 0]]), int(basis.l[pairs[0, 1]])
    lc = int(aux.l[auxidx[0]])
    nab, nc = nsph(la) * nsph(lb), nsph(lc)
    V = np.zeros(len(pairs) * nab * nc * len(auxidx))
    assert basis.normalize == aux.normalize
    a = aux.args()
    _check(lib().oracle_eri3(*basis.args()[:6], a[0], a[1], a[2], a[3], a[4], a[5], basis.normalize, len(pairs), pp,
                             len(auxidx), ap, V.ctypes.data_as(_dp), nthreads), "oracle_eri3")
    return V.reshape((len(pairs), nab, nc, len(auxidx)), order="F")


def eri2(basis: Basis, shells_a, shells_c, nthreads=0) -> np.ndarray:
    """2-centre Coulomb integrals (a|c) of single shells of one basis (one l per
    list) as V[i, ma, mc, k] (shape (na, Na, Nc, nc), Fortran order)."""
    sa, ap = _i(np.asarray(shells_a).reshape(-1))
    sc, cp = _i(np.asarray(shells_c).reshape(-1))
    na_, nc_ = nsph(int(basis.l[sa[0]])), nsph(int(basis.l[sc[0]]))
    V = np.zeros(len(sa) * na_ * nc_ * len(sc))
    _check(lib().oracle_eri2(*basis.args(), len(sa), ap, len(sc), cp, V.ctypes.data_as(_dp), nthreads), "oracle_eri2")
    return V.reshape((len(sa), na_, nc_, len(sc)), order="F")


def schwarz(basis: Basis, pairs, nthreads=0) -> np.ndarray:
    pairs, pp = _i(np.asarray(pairs).reshape(-1, 2))
    Q = np.zeros(len(pairs))
    _check(lib().oracle_schwarz(*basis.args(), len(pairs), pp, Q.ctypes.data_as(_dp), nthreads), "oracle_schwarz")
    return Q


def kbuild(basis: Basis, D, tau=1e-12, nthreads=0) -> np.ndarray:
    nao = basis.nao()
    D, Dp = _d(D)
    assert D.shape == (nao, nao)
    K = np.zeros((nao, nao))
    _check(lib().oracle_kbuild(*basis.args(), Dp, float(tau), K.ctypes.data_as(_dp), nthreads), "oracle_kbuild")
    return K


def exchange_grad(basis: Basis, atom_of_shell, natom, D, tau=1e-12, nthreads=0) -> np.ndarray:
    nao = basis.nao()
    D, Dp = _d(D)
    assert D.shape == (nao, nao)
    aos, aop = _i(atom_of_shell)
    g = np.zeros((natom, 3))
    _check(lib().oracle_exchange_grad(*basis.args(), aop, int(natom), Dp, float(tau), g.ctypes.data_as(_dp),
                                      nthreads), "oracle_exchange_grad")
    return g


def jbuild(basis: Basis, D, tau=1e-12, nthreads=0) -> np.ndarray:
    """J_ab = sum_cd (ab|cd) D_cd by brute force over every screened ordered quartet."""
    nao = basis.nao()
    D, Dp = _d(D)
    assert D.shape == (nao, nao)
    J = np.zeros((nao, nao))
    _check(lib().oracle_jbuild(*basis.args(), Dp, float(tau), J.ctypes.data_as(_dp), nthreads), "oracle_jbuild")
    return J


def three_index(basis: Basis, aux: Basis, nthreads=0) -> np.ndarray:
    """Dense (ab|P) over all AO pairs of `basis` and all AOs of `aux`:
    T[a, b, P] (shape (nao, nao, naux_ao)), assembled from eri3 shell by shell."""
    ao = np.concatenate([[0], np.cumsum(2 * basis.l + 1)])
    xo = np.concatenate([[0], np.cumsum(2 * aux.l + 1)])
    T = np.zeros((ao[-1], ao[-1], xo[-1]))
    for i in range(basis.nshell):
        for j in range(basis.nshell):
            for k in range(aux.nshell):
                V = eri3(basis, aux, [[i, j]], [k], nthreads)[0]  # [ab, mP]
                T[ao[i]:ao[i + 1], ao[j]:ao[j + 1], xo[k]:xo[k + 1]] = V.reshape(ao[i + 1] - ao[i], ao[j + 1] - ao[j], -1)
    return T


def metric(aux: Basis, nthreads=0) -> np.ndarray:
    """Dense Coulomb metric M_PQ = (P|Q) over all AOs of `aux`."""
    xo = np.concatenate([[0], np.cumsum(2 * aux.l + 1)])
    M = np.zeros((xo[-1], xo[-1]))
    for i in range(aux.nshell):
        for k in range(aux.nshell):
            M[xo[i]:xo[i + 1], xo[k]:xo[k + 1]] = eri2(aux, [i], [k], nthreads)[0, :, :, 0]
    return M


def dfj(basis: Basis, aux: Basis, D, nthreads=0) -> np.ndarray:
    """Density-fitted Coulomb matrix (the use of 3-centre integrals that Sec. 1
    motivates): the pair density sum_cd D_cd (cd| is fitted in the Coulomb
    metric, c = M^{-1} gamma with gamma_Q = sum_cd (Q|cd) D_cd and
    M_PQ = (P|Q), and J_ab = sum_P (ab|P) c_P.  Dense assembly; numpy solves."""
    assert basis.normalize == aux.normalize
    T = three_index(basis, aux, nthreads)
    M = metric(aux, nthreads)
    gamma = np.einsum("abP,ab->P", T, np.asarray(D, dtype=np.float64))
    c = np.linalg.solve(M, gamma)
    return T @ c


def dfk(basis: Basis, aux: Basis, D, nthreads=0) -> np.ndarray:
    """Density-fitted exchange matrix: every pair product is fitted in the
    Coulomb metric, (ab|cd) ~ sum_PQ (ab|P) [M^{-1}]_PQ (Q|cd) with
    M_PQ = (P|Q), and K_ac = sum_bd (ab|cd)_fit D_bd (the exchange operator of
    Sec. 6 over the fitted integrals).  Dense assembly; numpy solves."""
    assert basis.normalize == aux.normalize
    T = three_index(basis, aux, nthreads)
    M = metric(aux, nthreads)
    nao, naux = T.shape[0], T.shape[2]
    F = np.linalg.solve(M, T.reshape(nao * nao, naux).T).T.reshape(T.shape)  # sum_P [M^-1]_QP (P|cd)
    return np.einsum("abQ,cdQ,bd->ac", T, F, np.asarray(D, dtype=np.float64), optimize=True)


def fock_blocks(basis: Basis, D, blocks, which="K", tau=1e-12, nthreads=0):
    """Shell blocks of K (which="K", block (s0, s1) = K[AOs of s0, AOs of s1])
    or J (which="J") by the brute force restricted to the quartets feeding
    them.  Returns a list of [N(l_s0), N(l_s1)] arrays."""
    nao = basis.nao()
    D, Dp = _d(D)
    assert D.shape == (nao, nao)
    blk, bp = _i(np.asarray(blocks).reshape(-1, 2))
    sizes = [(nsph(int(basis.l[a])), nsph(int(basis.l[b]))) for a, b in blk]
    out = np.zeros(max(1, sum(x * y for x, y in sizes)))
    _check(lib().oracle_fock_blocks(*basis.args(), Dp, float(tau), {"K": 0, "J": 1}[which], len(blk), bp,
                                    out.ctypes.data_as(_dp), nthreads), "oracle_fock_blocks")
    res, o = [], 0
    for x, y in sizes:
        res.append(out[o:o + x * y].reshape(x, y).copy())
        o += x * y
    return res


def grad_pattern(basis: Basis, atom_of_shell, natom, pattern, Wl, Wr, tau=1e-12, nthreads=0) -> np.ndarray:
    """dE/dR of E = sum W_abcd (ab|cd), W = Wl_ac Wr_bd (pattern "exchange")
    or Wl_ab Wr_cd (pattern "coulomb")."""
    nao = basis.nao()
    Wl, Wlp = _d(Wl)
    Wr, Wrp = _d(Wr)
    assert Wl.shape == Wr.shape == (nao, nao)
    aos, aop = _i(atom_of_shell)
    g = np.zeros((natom, 3))
    _check(lib().oracle_grad_pattern(*basis.args(), aop, int(natom), {"exchange": 0, "coulomb": 1}[pattern], Wlp,
                                     Wrp, float(tau), g.ctypes.data_as(_dp), nthreads), "oracle_grad_pattern")
    return g
