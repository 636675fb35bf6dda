"""Independent reference for Cartesian two-electron integrals: the
Obara-Saika vertical recurrence (Obara & Saika, J. Chem. Phys. 84, 3963
(1986)) followed by the Head-Gordon-Pople horizontal recurrence
(J. Chem. Phys. 89, 5777 (1988)) -- the OS/HGP scheme the paper compares
against (Sec. 5, Performance).  Written from the published recurrences; it
shares nothing with the MD oracle except the integral it computes.

Arithmetic is done in a caller-chosen number type (mpmath mpf at 30+ digits,
or Python float); the Boys function comes from mpmath's incomplete gamma
function.  Only meant for tiny inputs (l <= 3) in the CPU test suite.
"""
from __future__ import annotations

from functools import lru_cache

import mpmath as mp


def boys_mp(m: int, T):
    T = mp.mpf(T)
    if T == 0:
        return mp.mpf(1) / (2 * m + 1)
    return mp.gammainc(m + mp.mpf(1) / 2, 0, T) / (2 * T ** (m + mp.mpf(1) / 2))


def cart_list(l):
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


def prim_eri_cart(la, lb, lc, ld, za, A, zb, B, zc, C, zd, D, dps=30):
    """Primitive [ab|cd] over bare Cartesian Gaussians for all components.

    Returns a dict {(a, b, c, d): value} with a..d Cartesian exponent triples;
    values are mpmath numbers at `dps` digits.
    """
    with mp.workdps(dps):
        za, zb, zc, zd = (mp.mpf(x) for x in (za, zb, zc, zd))
        A, B, C, D = ([mp.mpf(x) for x in v] for v in (A, B, C, D))
        p, q = za + zb, zc + zd
        P = [(za * A[i] + zb * B[i]) / p for i in range(3)]
        Q = [(zc * C[i] + zd * D[i]) / q for i in range(3)]
        W = [(p * P[i] + q * Q[i]) / (p + q) for i in range(3)]
        rho = p * q / (p + q)
        AB2 = sum((A[i] - B[i]) ** 2 for i in range(3))
        CD2 = sum((C[i] - D[i]) ** 2 for i in range(3))
        PQ2 = sum((P[i] - Q[i]) ** 2 for i in range(3))
        Kab = mp.exp(-za * zb / p * AB2)
        Kcd = mp.exp(-zc * zd / q * CD2)
        base = 2 * mp.pi ** mp.mpf(2.5) / (p * q * mp.sqrt(p + q)) * Kab * Kcd
        T = rho * PQ2
        L = la + lb + lc + ld
        F = [boys_mp(m, T) for m in range(L + 1)]

        @lru_cache(maxsize=None)
        def vrr(a, c, m):
            # [a0|c0]^(m) with a, c exponent triples
            if min(a) < 0 or min(c) < 0:
                return mp.mpf(0)
            if sum(a) == 0 and sum(c) == 0:
                return base * F[m]
            if sum(a) > 0:
                i = next(k for k in range(3) if a[k] > 0)
                am = list(a); am[i] -= 1; am = tuple(am)
                amm = list(am); amm[i] -= 1; amm = tuple(amm)
                cm = list(c); cm[i] -= 1; cm = tuple(cm)
                v = (P[i] - A[i]) * vrr(am, c, m) + (W[i] - P[i]) * vrr(am, c, m + 1)
                if am[i] > 0:
                    v += am[i] / (2 * p) * (vrr(amm, c, m) - rho / p * vrr(amm, c, m + 1))
                if c[i] > 0:
                    v += c[i] / (2 * (p + q)) * vrr(am, cm, m + 1)
                return v
            i = next(k for k in range(3) if c[k] > 0)
            cm = list(c); cm[i] -= 1; cm = tuple(cm)
            cmm = list(cm); cmm[i] -= 1; cmm = tuple(cmm)
            v = (Q[i] - C[i]) * vrr(a, cm, m) + (W[i] - Q[i]) * vrr(a, cm, m + 1)
            if cm[i] > 0:
                v += cm[i] / (2 * q) * (vrr(a, cmm, m) - rho / q * vrr(a, cmm, m + 1))
            return v

        @lru_cache(maxsize=None)
        def hrr_ket(a, c, d):
            # (a0|cd) from (a0|e0), d moved onto c
            if sum(d) == 0:
                return vrr(a, c, 0)
            i = next(k for k in range(3) if d[k] > 0)
            dm = list(d); dm[i] -= 1; dm = tuple(dm)
            cp = list(c); cp[i] += 1; cp = tuple(cp)
            return hrr_ket(a, cp, dm) + (C[i] - D[i]) * hrr_ket(a, c, dm)

        @lru_cache(maxsize=None)
        def hrr_bra(a, b, c, d):
            if sum(b) == 0:
                return hrr_ket(a, c, d)
            i = next(k for k in range(3) if b[k] > 0)
            bm = list(b); bm[i] -= 1; bm = tuple(bm)
            ap = list(a); ap[i] += 1; ap = tuple(ap)
            return hrr_bra(ap, bm, c, d) + (A[i] - B[i]) * hrr_bra(a, bm, c, d)

        out = {}
        for a in cart_list(la):
            for b in cart_list(lb):
                for c in cart_list(lc):
                    for d in cart_list(ld):
                        out[(a, b, c, d)] = hrr_bra(a, b, c, d)
        return out


def contracted_eri_cart(shells, dps=30):
    """Contracted Cartesian (ab|cd) over four raw shells.

    shells: 4 tuples (l, exps, coefs, centre); primitives are bare
    x^a y^b z^c exp(-z r^2) times the raw coefficients.  Returns a float
    array [ncart(la), ncart(lb), ncart(lc), ncart(ld)] in the component order
    lx descending then ly descending.
    """
    import numpy as np
    (la, ea, ca, A), (lb, eb, cb, B), (lc, ec, cc, C), (ld, ed, cd, D) = shells
    dims = [len(cart_list(x)) for x in (la, lb, lc, ld)]
    with mp.workdps(dps):
        acc = {}
        for za, wa in zip(ea, ca):
            for zb, wb in zip(eb, cb):
                for zc, wc in zip(ec, cc):
                    for zd, wd in zip(ed, cd):
                        prim = prim_eri_cart(la, lb, lc, ld, za, A, zb, B, zc, C, zd, D, dps)
                        w = mp.mpf(wa) * wb * wc * wd
                        for k, v in prim.items():
                            acc[k] = acc.get(k, mp.mpf(0)) + w * v
        out = np.zeros(dims)
        for ia, a in enumerate(cart_list(la)):
            for ib, b in enumerate(cart_list(lb)):
                for ic, c in enumerate(cart_list(lc)):
                    for id_, d in enumerate(cart_list(ld)):
                        out[ia, ib, ic, id_] = float(acc[(a, b, c, d)])
    return out
