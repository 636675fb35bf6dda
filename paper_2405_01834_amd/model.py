"""Sizes and the roofline cost model of the MD scheme (Table md-scheme, Sec. 2).

Per primitive shellset [bra|ket] with L = l_bra + l_ket:
  [0]^(m) -> [r]^(0)      (Eq. r):   A_in = L+1,        A_out = Ñ(L),          N_F = R_L
  [r]     -> [p|q]        (Eq. pq):  A_in = Ñ(L),       A_out = Ñ_b Ñ_k,      N_F = Ñ_b Ñ_k / 2
  [p|q]   -> [p|ket]      (ket):     A_in = Ñ_b Ñ_k,   A_out = Ñ_b N_k,      N_F = 2 Ñ_b Ñ_k N_k
  [p|ket] -> [bra|ket]    (bra):     A_in = Ñ_b N_k,   A_out = N_b N_k,      N_F = 2 N_b Ñ_b N_k
with R_L = (2+L)(7+L)(12+5L+L^2)/8, Ñ(l) = (l+1)(l+2)(l+3)/6, Ñ_b = Ñ(l_a+l_b),
N_b = N(l_a) N(l_b), N(l) = 2l+1 (the table's 81 = 9^2 for [11|11] fixes
N_b as the product).  With contraction, the ket step runs once per primitive
quartet and the bra step once per bra primitive pair (ket transformed first).
"""
from __future__ import annotations


def ntil(l: int) -> int:
    return (l + 1) * (l + 2) * (l + 3) // 6


def nsph(l: int) -> int:
    return 2 * l + 1


def R_L(L: int) -> int:
    return (2 + L) * (7 + L) * (12 + 5 * L + L * L) // 8


def md_scheme(la: int, lb: int, lc: int, ld: int) -> dict:
    """The four rows of Table md-scheme for one primitive shellset."""
    L = la + lb + lc + ld
    Nhb, Nhk = ntil(la + lb), ntil(lc + ld)
    Nb, Nk = nsph(la) * nsph(lb), nsph(lc) * nsph(ld)
    return {
        "r": (L + 1, ntil(L), R_L(L)),
        "pq": (ntil(L), Nhb * Nhk, Nhb * Nhk / 2),
        "ket": (Nhb * Nhk, Nhb * Nk, 2 * Nhb * Nhk * Nk),
        "bra": (Nhb * Nk, Nb * Nk, 2 * Nb * Nhb * Nk),
    }


def eri4_flops(la: int, lb: int, lc: int, ld: int, kbra: int, kket: int) -> float:
    """Model FLOPs of one contracted shellset: K (R_L + Ñ_b Ñ_k/2 + 2 Ñ_b Ñ_k N_k)
    + K_bra 2 N_b Ñ_b N_k with K = K_bra K_ket (pair-level contraction degrees)."""
    t = md_scheme(la, lb, lc, ld)
    K = kbra * kket
    return K * (t["r"][2] + t["pq"][2] + t["ket"][2]) + kbra * t["bra"][2]


def top_degree(l: int) -> int:
    """T(l) = (l+1)(l+2)/2 Hermite functions of degree exactly l: by Hobson's
    theorem the only ones a single solid-harmonic Gaussian expands into."""
    return (l + 1) * (l + 2) // 2


def eri3_flops(la: int, lb: int, lP: int, kbra: int, kaux: int) -> float:
    """Model FLOPs of one contracted 3-centre shellset (ab|P) in the order the
    kernel runs it, auxiliary side first: per primitive triple R_L plus the
    auxiliary transform over the T_P top-degree rows, [p|P] = sum_q [p|q] H_P
    (2 Ñ_ab T_P N_P); per pair primitive the pair transform (2 N_ab Ñ_ab N_P):
        K_ab K_P (R_L + 2 Ñ_ab T_P N_P) + K_ab 2 N_ab Ñ_ab N_P,
    L = l_a + l_b + l_P.  The pair-first order would count
    K_ab K_P (R_L + 2 N_ab Ñ_ab T_P) + K_P 2 N_ab T_P N_P instead."""
    L = la + lb + lP
    Nhab, Nab, TP, NP = ntil(la + lb), nsph(la) * nsph(lb), top_degree(lP), nsph(lP)
    return kbra * kaux * (R_L(L) + 2 * Nhab * TP * NP) + kbra * 2 * Nab * Nhab * NP


def eri3_flops_pair_first(la: int, lb: int, lP: int, kbra: int, kaux: int) -> float:
    """The pair-first count of the same shellset (see eri3_flops)."""
    L = la + lb + lP
    Nhab, Nab, TP, NP = ntil(la + lb), nsph(la) * nsph(lb), top_degree(lP), nsph(lP)
    return kbra * kaux * (R_L(L) + 2 * Nab * Nhab * TP) + kaux * 2 * Nab * TP * NP


def eri4_outputs(la: int, lb: int, lc: int, ld: int) -> int:
    return nsph(la) * nsph(lb) * nsph(lc) * nsph(ld)


FP64_PEAK_TFLOPS = 78.6   # MI355X, vector and matrix
HBM_PEAK_GBS = 8000.0
