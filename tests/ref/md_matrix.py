"""Matrix-form McMurchie-Davidson reference for high angular momentum.

The sum-form oracle evaluates every Cartesian integral as a double sum over
bra and ket Hermite indices, which is out of reach at l = 5, 6 (about 1e6
terms per Cartesian integral).  This module assembles the same integral as
dense products of the oracle's own pinned building blocks -- the 1-D
Hermite coefficients E (oracle.E2), the Hermite integrals R (oracle.R,
which includes the Boys function) and the solid-harmonic coefficients
(oracle.solid) -- over the full (l+1)^3 Hermite grids:

    (ab|cd) = sum_{tuv} sum_{tau nu phi} E^{ab}_{tuv} (-1)^{tau+nu+phi}
              E^{cd}_{tau nu phi} R_{t+tau, u+nu, v+phi}            (Sec. 2)

contracted with the oracle's normalised coefficients and transformed to
real solid harmonics.  It shares no code with the GPU path; the CPU tests
pin it against oracle.eri4 on classes the sum form can reach.
"""
from __future__ import annotations

import numpy as np

import oracle


def _hermite_grid(la, lb, za, zb, A, B):
    """E^{ab}_{tuv} for all Cartesian (a, b) as [ncart_a * ncart_b, n, n, n], n = la+lb+1."""
    n = la + lb + 1
    E = [oracle.E2(la, lb, za, zb, A[x], B[x]) for x in range(3)]  # [i][j][t]
    ca, cb = oracle.cart_list(la), oracle.cart_list(lb)
    out = np.zeros((len(ca) * len(cb), n, n, n))
    for ia, a in enumerate(ca):
        for ib, b in enumerate(cb):
            out[ia * len(cb) + ib] = np.einsum("t,u,v->tuv", E[0][a[0], b[0]], E[1][a[1], b[1]], E[2][a[2], b[2]])
    return out


def shellset(shells, i, j, k, m):
    """Contracted solid-harmonic (ab|cd) of shells i, j, k, m as [Na*Nb, Nc*Nd]
    (ab = m_a N(l_b) + m_b), unit-normalised shells (normalize=1)."""
    ls = [int(shells.l[x]) for x in (i, j, k, m)]
    off = np.concatenate([[0], np.cumsum(shells.nprim)])
    prim = []
    for x, l in zip((i, j, k, m), ls):
        z = shells.exps[off[x]:off[x + 1]]
        c = oracle.norm_coefs(l, z, shells.coefs[off[x]:off[x + 1]], 1)
        prim.append((z, c, shells.centers[x]))
    la, lb, lc, ld = ls
    nb, nk = la + lb + 1, lc + ld + 1
    L = la + lb + lc + ld
    # index grids of R[t+tau, u+nu, v+phi] and the ket sign (-1)^{tau+nu+phi}
    tb = np.indices((nb, nb, nb)).reshape(3, -1)
    tk = np.indices((nk, nk, nk)).reshape(3, -1)
    sgn = (-1.0) ** tk.sum(axis=0)
    Vc = 0.0
    (za, ca, A), (zb, cb, B), (zc, cc, C), (zd, cd, D) = prim
    for ia in range(len(za)):
        for ib in range(len(zb)):
            p = za[ia] + zb[ib]
            P = (za[ia] * A + zb[ib] * B) / p
            Eb = _hermite_grid(la, lb, za[ia], zb[ib], A, B).reshape(-1, nb ** 3) * (ca[ia] * cb[ib])
            for ic in range(len(zc)):
                for idd in range(len(zd)):
                    q = zc[ic] + zd[idd]
                    Q = (zc[ic] * C + zd[idd] * D) / q
                    Ek = _hermite_grid(lc, ld, zc[ic], zd[idd], C, D).reshape(-1, nk ** 3) * (cc[ic] * cd[idd])
                    rho = p * q / (p + q)
                    pref = 2.0 * np.pi ** 2.5 / (p * q * np.sqrt(p + q))
                    R = oracle.R(L, rho, P - Q, pref)
                    M = R[tb[0][:, None] + tk[0][None, :], tb[1][:, None] + tk[1][None, :],
                          tb[2][:, None] + tk[2][None, :]] * sgn[None, :]
                    Vc = Vc + Eb @ M @ Ek.T
    Ca, Cb, Cc, Cd = (oracle.solid(x) for x in ls)
    Vc = Vc.reshape(Ca.shape[1], Cb.shape[1], Cc.shape[1], Cd.shape[1])
    V = np.einsum("ai,bj,ck,dl,ijkl->abcd", Ca, Cb, Cc, Cd, Vc, optimize=True)
    return V.reshape(Ca.shape[0] * Cb.shape[0], Cc.shape[0] * Cd.shape[0])
