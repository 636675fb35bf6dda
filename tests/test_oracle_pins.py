"""Pins of the FP64 CPU oracle against facts that do not come from the oracle
itself: closed forms, mpmath evaluations of the defining formulas, an
independent Obara-Saika/Head-Gordon-Pople evaluation, exact polynomial facts
about solid harmonics, symmetries and invariances of the Coulomb integral.

Each test names the passage of the paper (Asadchev & Valeev, Sec. 2
"Formalism" unless stated) or the mathematical fact it pins.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from tests.ref.os_hgp import boys_mp, contracted_eri_cart

# ---------------------------------------------------------------------------
# Boys function, Eq. (boys)
# ---------------------------------------------------------------------------

T_GRID = [0.0, 1e-12, 1e-6, 1e-3, 0.1, 0.5, 1.0, 2.5, 5.0, 9.9, 15.0, 29.9, 30.1, 37.5, 45.0, 59.9, 60.1,
          79.9, 80.1, 100.0, 250.0, 1e3, 3e4, 3e5, 1e6]


@pytest.mark.parametrize("mmax", [0, 1, 4, 8, 12, 16, 25, 36])
def test_boys_matches_incomplete_gamma(mmax):
    """F_m(T) = gamma(m+1/2, T) / (2 T^{m+1/2}) evaluated by mpmath at 40 digits."""
    worst = 0.0
    with mp.workdps(40):
        for T in T_GRID:
            F = oracle.boys(mmax, T)
            for m in range(mmax + 1):
                ref = float(boys_mp(m, T))
                worst = max(worst, abs(F[m] - ref) / ref)
    assert worst < 1e-15, worst


def test_boys_closed_forms():
    # F_m(0) = 1/(2m+1)
    F = oracle.boys(30, 0.0)
    assert np.allclose(F, 1.0 / (2 * np.arange(31) + 1), rtol=1e-16, atol=0)
    # F_0(T) = (1/2) sqrt(pi/T) erf(sqrt T)
    for T in [1e-4, 0.3, 2.0, 17.0, 64.0, 500.0]:
        ref = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
        assert abs(oracle.boys(0, T)[0] - ref) <= 2e-16 * ref
    # large-T asymptote Gamma(m+1/2)/(2 T^{m+1/2}) with exponentially small error
    T = 2000.0
    F = oracle.boys(10, T)
    for m in range(11):
        ref = math.gamma(m + 0.5) / (2 * T ** (m + 0.5))
        assert abs(F[m] - ref) <= 1e-15 * ref


def test_boys_downward_identity():
    """F_m = (2T F_{m+1} + e^{-T}) / (2m+1) on both sides of the method switch."""
    for T in [0.7, 12.0, 45.0, 71.0, 120.0]:
        F = oracle.boys(20, T)
        for m in range(20):
            lhs = F[m]
            rhs = (2 * T * F[m + 1] + math.exp(-T)) / (2 * m + 1)
            assert abs(lhs - rhs) <= 4e-16 * lhs


# ---------------------------------------------------------------------------
# Hermite expansion coefficients, Eqs. (cart2herm-1/2), (E1rr)-(E2-abab)
# ---------------------------------------------------------------------------

def _lam(t, p, P, x):
    """Hermite Gaussian (d/dP)^t exp(-p (x-P)^2) = p^{t/2} H_t(sqrt(p)(x-P)) e^{-p(x-P)^2}."""
    y = mp.sqrt(p) * (x - P)
    return p ** (mp.mpf(t) / 2) * mp.hermite(t, y) * mp.exp(-y * y)


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (0, 2), (2, 3), (4, 4), (6, 5), (9, 8)])
def test_E2_pointwise_expansion(la, lb):
    """x_A^i x_B^j e^{-a x_A^2 - b x_B^2} = sum_t E_t^{ij} Lambda_t(x), Eq. (cart2herm-2)."""
    a, b, A, B = 0.73, 1.9, -0.4, 0.85
    E = oracle.E2(la, lb, a, b, A, B)
    p = a + b
    P = (a * A + b * B) / p
    with mp.workdps(30):
        for x in [-1.3, -0.2, 0.1, 0.55, 1.7]:
            x = mp.mpf(x)
            for i in range(la + 1):
                for j in range(lb + 1):
                    lhs = (x - A) ** i * (x - B) ** j * mp.exp(-a * (x - A) ** 2 - b * (x - B) ** 2)
                    terms = [E[i, j, t] * _lam(t, p, P, x) for t in range(i + j + 1)]
                    scale = max([abs(lhs)] + [abs(tm) for tm in terms]) + 1e-300
                    assert abs(lhs - sum(terms)) / scale < 1e-13


@pytest.mark.parametrize("la,lb", [(1, 1), (3, 2), (6, 6)])
def test_E2_top_degree(la, lb):
    """Eq. (E2-abab): E_{ab}^{a+b} = E^0_00 / (2 zeta_p)^{a+b}."""
    a, b, A, B = 0.4, 2.2, 0.3, -1.1
    E = oracle.E2(la, lb, a, b, A, B)
    p = a + b
    E0 = math.exp(-a * b / p * (A - B) ** 2)
    for i in range(la + 1):
        for j in range(lb + 1):
            assert abs(E[i, j, i + j] - E0 / (2 * p) ** (i + j)) <= 1e-15 * abs(E0 / (2 * p) ** (i + j))
            # parity structure of a 2-centre product is absent: nothing else forced to zero
    assert E.shape == (la + 1, lb + 1, la + lb + 1)


@pytest.mark.parametrize("la", [0, 1, 2, 5, 7, 9])
def test_E1_pointwise_expansion(la):
    """x_A^i e^{-a x_A^2} = sum_t E_t^i Lambda_t(x), Eq. (cart2herm-1), and the
    parity zeros of Eq. (E1-aa)."""
    a, A = 1.3, 0.2
    E = oracle.E1(la, a)
    with mp.workdps(30):
        for x in [-0.9, 0.05, 0.6, 1.4]:
            x = mp.mpf(x)
            for i in range(la + 1):
                lhs = (x - A) ** i * mp.exp(-a * (x - A) ** 2)
                terms = [E[i, t] * _lam(t, a, A, x) for t in range(i + 1)]
                scale = max([abs(lhs)] + [abs(tm) for tm in terms]) + 1e-300
                assert abs(lhs - sum(terms)) / scale < 1e-13
    for i in range(la + 1):
        for t in range(la + 1):
            if t > i or (t + i) % 2 == 1:
                assert E[i, t] == 0.0


# ---------------------------------------------------------------------------
# Auxiliary integrals, Eqs. (0m) and (r)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("L", [1, 3, 5])
def test_R_is_derivative_of_F0(L):
    """[t u v]^(0) = d^t/dX^t d^u/dY^u d^v/dZ^v [0]^(0)(X, Y, Z), with
    [0]^(0) = F_0(rho |P-Q|^2) (prefactor 1), by mpmath differentiation."""
    rho = 0.9
    PQ = np.array([0.35, -0.6, 0.8])
    R = oracle.R(L, rho, PQ)

    def f0(X, Y, Z):
        T = rho * (X * X + Y * Y + Z * Z)
        return mp.sqrt(mp.pi / T) * mp.erf(mp.sqrt(T)) / 2

    scale = np.max(np.abs(R))
    with mp.workdps(30):
        for t in range(L + 1):
            for u in range(L + 1 - t):
                for v in range(L + 1 - t - u):
                    ref = mp.diff(f0, (mp.mpf(PQ[0]), mp.mpf(PQ[1]), mp.mpf(PQ[2])), (t, u, v))
                    assert abs(R[t, u, v] - float(ref)) < 1e-13 * scale, (t, u, v)


# ---------------------------------------------------------------------------
# Solid harmonics (coefficients C of Eqs. (solid2herm-1/2))
# ---------------------------------------------------------------------------

def _sphere_monomial(a, b, c):
    """Integral of x^a y^b z^c over the unit sphere."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    return 2.0 * math.gamma((a + 1) / 2) * math.gamma((b + 1) / 2) * math.gamma((c + 1) / 2) / math.gamma(
        (a + b + c + 3) / 2)


@pytest.mark.parametrize("l", range(0, 10))
def test_solid_harmonics_harmonic_and_orthonormal(l):
    C = oracle.solid(l)
    comps = oracle.cart_list(l)
    # Laplacian of sum_k C[m,k] x^a y^b z^c must vanish identically
    for m in range(2 * l + 1):
        lap = {}
        for k, (a, b, c) in enumerate(comps):
            for ax, e in enumerate((a, b, c)):
                if e >= 2:
                    key = [a, b, c]
                    key[ax] -= 2
                    key = tuple(key)
                    lap[key] = lap.get(key, 0.0) + C[m, k] * e * (e - 1)
        assert all(abs(v) < 1e-12 * np.max(np.abs(C)) for v in lap.values())
    # Orthogonal on the sphere with the norm of x^l: 4 pi / (2l+1)
    G = np.zeros((2 * l + 1, 2 * l + 1))
    for i, ci in enumerate(comps):
        for j, cj in enumerate(comps):
            s = _sphere_monomial(ci[0] + cj[0], ci[1] + cj[1], ci[2] + cj[2])
            G += np.outer(C[:, i], C[:, j]) * s
    assert np.allclose(G, np.eye(2 * l + 1) * 4 * math.pi / (2 * l + 1), rtol=0, atol=1e-12)


def test_solid_harmonics_order_and_phase():
    """m = -l..l ordering with standard phases: p = (y, z, x);
    d: m=0 is z^2 - (x^2+y^2)/2, m=2 is sqrt(3)/2 (x^2 - y^2), m=-2 is sqrt(3) xy."""
    C1 = oracle.solid(1)  # Cartesian order x, y, z
    assert np.allclose(C1, [[0, 1, 0], [0, 0, 1], [1, 0, 0]])
    C2 = oracle.solid(2)  # xx, xy, xz, yy, yz, zz
    assert np.allclose(C2[2], [-0.5, 0, 0, -0.5, 0, 1])
    assert np.allclose(C2[4], [math.sqrt(3) / 2, 0, 0, -math.sqrt(3) / 2, 0, 0])
    assert np.allclose(C2[0], [0, math.sqrt(3), 0, 0, 0, 0])
    assert np.allclose(C2[1], [0, 0, 0, 0, math.sqrt(3), 0])
    assert np.allclose(C2[3], [0, 0, math.sqrt(3), 0, 0, 0])


@pytest.mark.parametrize("l", [0, 1, 2, 4, 6, 8])
def test_hobson_top_degree_only(l):
    """A 1-centre solid-harmonic Gaussian expands in Hermite Gaussians of degree
    exactly l (Hobson's theorem): H_P^q = sum_c C_c E_c^q (Eq. (solid2herm-1))
    vanishes for |q| < l and equals C_q / (2 zeta)^l for |q| = l."""
    a = 0.77
    C = oracle.solid(l)
    E = oracle.E1(l, a)
    comps = oracle.cart_list(l)
    for m in range(2 * l + 1):
        for t in range(l + 1):
            for u in range(l + 1 - t):
                for v in range(l + 1 - t - u):
                    terms = [C[m, k] * E[c[0], t] * E[c[1], u] * E[c[2], v] for k, c in enumerate(comps)]
                    h = sum(terms)
                    if t + u + v < l:
                        # zero up to the rounding of its terms (large at l = 8)
                        assert abs(h) < 1e-14 * max(1.0, sum(abs(x) for x in terms))
                    else:
                        k = comps.index((t, u, v))
                        assert abs(h - C[m, k] / (2 * a) ** l) < 1e-14 * max(1.0, abs(C[m, k] / (2 * a) ** l))


@pytest.mark.parametrize("l,K", [(0, 1), (1, 3), (2, 2), (4, 3), (6, 1), (8, 2)])
def test_normalised_shell_has_unit_norm(l, K):
    """Closed-form self-overlap of every normalised solid-harmonic AO is 1:
    sum_kk' c~_k c~_k' (4 pi/(2l+1)) Gamma(l+3/2) / (2 (z_k+z_k')^{l+3/2})."""
    rng = np.random.default_rng(11 + l)
    z = np.exp(rng.uniform(np.log(0.05), np.log(500), K))
    c = rng.uniform(0.1, 1.0, K)
    ct = oracle.norm_coefs(l, z, c, 1)
    S = 0.0
    for i in range(K):
        for j in range(K):
            S += ct[i] * ct[j] * 4 * math.pi / (2 * l + 1) * math.gamma(l + 1.5) / (2 * (z[i] + z[j]) ** (l + 1.5))
    assert abs(S - 1.0) < 1e-14


# ---------------------------------------------------------------------------
# Whole integrals
# ---------------------------------------------------------------------------

def _rand_basis(ls, K, rng, box=2.0, lo=0.2, hi=3.0, normalize=1):
    ex = [np.exp(rng.uniform(np.log(lo), np.log(hi), k)) for k in K]
    co = [rng.uniform(0.2, 1.0, k) for k in K]
    cen = rng.uniform(-box / 2, box / 2, (len(ls), 3))
    return oracle.Basis(ls, K, np.concatenate(ex), np.concatenate(co), cen, normalize), ex, co, cen


def test_ssss_closed_form():
    """(ss|ss) over contracted normalised s shells:
    sum c~c~c~c~ 2 pi^{5/2}/(pq sqrt(p+q)) e^{-mu_ab AB^2} e^{-mu_cd CD^2} F_0(rho PQ^2),
    with F_0 from erf and the contraction normalisation done here."""
    rng = np.random.default_rng(3)
    K = [2, 1, 3, 2]
    b, ex, co, cen = _rand_basis([0, 0, 0, 0], K, rng)
    v = oracle.eri4_shellset(b, 0, 1, 2, 3).ravel()[0]
    ct = []
    for z, c in zip(ex, co):
        S = sum(ci * cj * (2 * math.sqrt(zi * zj) / (zi + zj)) ** 1.5 for zi, ci in zip(z, c) for zj, cj in zip(z, c))
        ct.append([ci * (2 * zi / math.pi) ** 0.75 / math.sqrt(S) for zi, ci in zip(z, c)])
    ref = 0.0
    for ia, za in enumerate(ex[0]):
        for ib, zb in enumerate(ex[1]):
            for ic, zc in enumerate(ex[2]):
                for id_, zd in enumerate(ex[3]):
                    p, q = za + zb, zc + zd
                    P = (za * cen[0] + zb * cen[1]) / p
                    Q = (zc * cen[2] + zd * cen[3]) / q
                    rho = p * q / (p + q)
                    T = rho * np.sum((P - Q) ** 2)
                    F0 = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
                    ref += (ct[0][ia] * ct[1][ib] * ct[2][ic] * ct[3][id_] * 2 * math.pi ** 2.5 /
                            (p * q * math.sqrt(p + q)) * math.exp(-za * zb / p * np.sum((cen[0] - cen[1]) ** 2)) *
                            math.exp(-zc * zd / q * np.sum((cen[2] - cen[3]) ** 2)) * F0)
    assert abs(v - ref) <= 1e-14 * abs(ref)


OS_CASES = [((0, 0, 0, 0), (1, 1, 1, 1), 30), ((1, 0, 0, 0), (2, 1, 1, 2), 30), ((1, 1, 0, 0), (1, 2, 2, 1), 30),
            ((1, 1, 1, 1), (1, 1, 2, 1), 30), ((2, 0, 1, 0), (2, 1, 1, 1), 30), ((2, 1, 2, 0), (1, 1, 1, 1), 25),
            ((2, 2, 1, 1), (1, 1, 1, 1), 25), ((0, 2, 2, 0), (1, 2, 1, 1), 25), ((3, 1, 0, 2), (1, 1, 1, 1), 20),
            ((3, 3, 1, 0), (1, 1, 1, 1), 20)]


@pytest.mark.parametrize("ls,K,dps", OS_CASES)
def test_against_obara_saika_hgp(ls, K, dps):
    """Contracted Cartesian integrals agree with an independent OS-VRR + HGP-HRR
    evaluation (the comparison method of Sec. 5) on raw, unnormalised shells."""
    rng = np.random.default_rng(100 + sum(ls) * 7 + sum(K))
    b, ex, co, cen = _rand_basis(ls, K, rng, normalize=0)
    ref = contracted_eri_cart([(ls[i], ex[i], co[i], cen[i]) for i in range(4)], dps=dps)
    v = oracle.eri4_cart(b, 0, 1, 2, 3)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(v - ref)) <= 1e-13 * scale + 1e-300


def test_three_centre_against_obara_saika():
    """(ab|c) equals the 4-centre (ab|c s0) with an s function of exponent 0
    and coefficient 1 (the 1-centre Hermite expansion of Eqs. (E1rr)-(E1-aa)),
    evaluated independently by OS/HGP."""
    rng = np.random.default_rng(7)
    ls = [2, 1, 3]
    K = [2, 1, 1]
    ex = [np.exp(rng.uniform(np.log(0.3), np.log(3), k)) for k in K]
    co = [rng.uniform(0.2, 1.0, k) for k in K]
    cen = rng.uniform(-1, 1, (3, 3))
    prim = oracle.Basis(ls[:2], K[:2], np.concatenate(ex[:2]), np.concatenate(co[:2]), cen[:2], 0)
    aux = oracle.Basis(ls[2:], K[2:], np.concatenate(ex[2:]), np.concatenate(co[2:]), cen[2:], 0)
    # raw Cartesian comparison needs the Cartesian path: undo the solid transform of the oracle
    # by comparing solid results with OS results transformed by the (separately pinned) C.
    V = oracle.eri3(prim, aux, [[0, 1]], [0])[0, :, :, 0]
    ref_c = contracted_eri_cart([(ls[0], ex[0], co[0], cen[0]), (ls[1], ex[1], co[1], cen[1]),
                                 (ls[2], ex[2], co[2], cen[2]), (0, [0.0], [1.0], cen[2])], dps=25)[..., 0]
    Ca, Cb, Cc = oracle.solid(ls[0]), oracle.solid(ls[1]), oracle.solid(ls[2])
    ref = np.einsum("ai,bj,ck,ijk->abk", Ca, Cb, np.eye(Cc.shape[1]), ref_c)
    ref = np.einsum("ck,abk->abc", Cc, ref).reshape(V.shape)
    assert np.max(np.abs(V - ref)) <= 1e-13 * np.max(np.abs(ref))


def _perm_check(V, W, axes):
    np.testing.assert_allclose(V, np.transpose(W, axes), rtol=1e-12, atol=1e-15 * np.max(np.abs(V)))


@pytest.mark.parametrize("ls", [(2, 3, 1, 4), (1, 1, 0, 2), (4, 4, 3, 2)])
def test_eight_fold_symmetry(ls):
    rng = np.random.default_rng(sum(ls))
    b, *_ = _rand_basis(ls, [2, 1, 2, 1], rng)
    V = oracle.eri4_shellset(b, 0, 1, 2, 3)
    _perm_check(V, oracle.eri4_shellset(b, 1, 0, 2, 3), (1, 0, 2, 3))
    _perm_check(V, oracle.eri4_shellset(b, 0, 1, 3, 2), (0, 1, 3, 2))
    _perm_check(V, oracle.eri4_shellset(b, 2, 3, 0, 1), (2, 3, 0, 1))
    _perm_check(V, oracle.eri4_shellset(b, 3, 2, 1, 0), (3, 2, 1, 0))


def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@pytest.mark.parametrize("ls", [(1, 1, 1, 1), (2, 0, 3, 1), (4, 2, 2, 3)])
def test_rotational_invariance(ls):
    """Real solid harmonics of one l transform by an orthogonal matrix under
    rotation, so each shellset's Frobenius norm is rotation invariant (a
    wrong Cartesian -> solid coefficient breaks this)."""
    rng = np.random.default_rng(40 + sum(ls))
    b, ex, co, cen = _rand_basis(ls, [1, 2, 1, 1], rng)
    V = oracle.eri4_shellset(b, 0, 1, 2, 3)
    for _ in range(3):
        Rm = _rotation(rng)
        b2 = oracle.Basis(b.l, b.nprim, b.exps, b.coefs, cen @ Rm.T + rng.normal(size=3), 1)
        V2 = oracle.eri4_shellset(b2, 0, 1, 2, 3)
        assert abs(np.linalg.norm(V2) - np.linalg.norm(V)) <= 1e-12 * np.linalg.norm(V)
    # the invariant is not trivially satisfied: permuting centres changes it
    b3 = oracle.Basis(b.l, b.nprim, b.exps, b.coefs, cen[[0, 2, 1, 3]], 1)
    assert abs(np.linalg.norm(oracle.eri4_shellset(b3, 0, 1, 2, 3)) - np.linalg.norm(V)) > 1e-6 * np.linalg.norm(V)


def test_translation_invariance():
    rng = np.random.default_rng(9)
    b, ex, co, cen = _rand_basis((3, 1, 2, 2), [2, 1, 1, 2], rng)
    V = oracle.eri4_shellset(b, 0, 1, 2, 3)
    b2 = oracle.Basis(b.l, b.nprim, b.exps, b.coefs, cen + np.array([3.3, -1.2, 7.0]), 1)
    np.testing.assert_allclose(oracle.eri4_shellset(b2, 0, 1, 2, 3), V, rtol=1e-11, atol=1e-13 * np.max(np.abs(V)))


def test_schwarz_inequality():
    rng = np.random.default_rng(21)
    b, *_ = _rand_basis((2, 1, 3, 2), [1, 2, 1, 1], rng, box=3.0)
    V = oracle.eri4_shellset(b, 0, 1, 2, 3).reshape(15, 35)
    Vab = oracle.eri4_shellset(b, 0, 1, 0, 1).reshape(15, 15)
    Vcd = oracle.eri4_shellset(b, 2, 3, 2, 3).reshape(35, 35)
    bound = np.sqrt(np.outer(np.diag(Vab), np.diag(Vcd)))
    assert np.all(np.abs(V) <= bound * (1 + 1e-12))
    Q = oracle.schwarz(b, [[0, 1], [2, 3]])
    assert np.isclose(Q[0], math.sqrt(np.max(np.abs(np.diag(Vab)))), rtol=1e-14)
    assert np.isclose(Q[1], math.sqrt(np.max(np.abs(np.diag(Vcd)))), rtol=1e-14)


@pytest.mark.parametrize("la,lc", [(0, 0), (1, 2), (3, 4), (6, 5)])
def test_far_field_monopole(la, lc):
    """A normalised AO's square carries unit charge, so (a_m a_m | c_n c_n)
    tends to 1/R for far-apart centres (relative error O(1/(zeta R^2)))."""
    R = 2000.0
    b = oracle.Basis([la, la, lc, lc], [2, 2, 1, 1], [0.6, 2.5, 0.6, 2.5, 0.9, 0.9], [0.4, 0.7, 0.4, 0.7, 1, 1],
                     [[0, 0, 0], [0, 0, 0], [R / math.sqrt(3)] * 3, [R / math.sqrt(3)] * 3], 1)
    V = oracle.eri4_shellset(b, 0, 1, 2, 3)
    for m in range(2 * la + 1):
        for n in range(2 * lc + 1):
            assert abs(V[m, m, n, n] * R - 1.0) < 1e-5


# ---------------------------------------------------------------------------
# Exchange operator (Sec. 6) and nuclear derivatives
# ---------------------------------------------------------------------------

def _tiny_molecule(rng, shells_per_atom=((0, 2), (1, 1), (2, 1)), natom=2, spread=2.5):
    ls, K, ex, co, cen, atom = [], [], [], [], [], []
    pos = rng.uniform(0, spread, (natom, 3))
    for a in range(natom):
        for l, k in shells_per_atom:
            ls.append(l)
            K.append(k)
            ex.append(np.exp(rng.uniform(np.log(0.3), np.log(4.0), k)))
            co.append(rng.uniform(0.3, 1.0, k))
            cen.append(pos[a])
            atom.append(a)
    return (ls, K, np.concatenate(ex), np.concatenate(co), np.array(cen), np.array(atom, dtype=np.int32), pos)


def _full_eri(b):
    n = b.nshell
    off = np.concatenate([[0], np.cumsum(2 * b.l + 1)])
    nao = off[-1]
    G = np.zeros((nao, nao, nao, nao))
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for m in range(n):
                    G[off[i]:off[i + 1], off[j]:off[j + 1], off[k]:off[k + 1], off[m]:off[m + 1]] = \
                        oracle.eri4_shellset(b, i, j, k, m)
    return G


def test_kbuild_matches_explicit_contraction():
    """K_ac = sum_bd (ab|cd) D_bd (Sec. 6), against an einsum over the full
    ERI tensor; K is symmetric for symmetric D and tr(DK) >= 0."""
    rng = np.random.default_rng(5)
    ls, K, ex, co, cen, atom, pos = _tiny_molecule(rng)
    b = oracle.Basis(ls, K, ex, co, cen, 1)
    nao = b.nao()
    C = rng.normal(size=(nao, 3))
    D = C @ C.T
    G = _full_eri(b)
    Kref = np.einsum("abcd,bd->ac", G, D)
    Kor = oracle.kbuild(b, D, tau=0.0)
    np.testing.assert_allclose(Kor, Kref, rtol=1e-12, atol=1e-13 * np.max(np.abs(Kref)))
    np.testing.assert_allclose(Kor, Kor.T, rtol=1e-12, atol=1e-13 * np.max(np.abs(Kref)))
    Dn = rng.normal(size=(nao, nao))
    # the definition does not need a symmetric D: an unsymmetric one catches a transposed operand
    np.testing.assert_allclose(oracle.kbuild(b, Dn, tau=0.0), np.einsum("abcd,bd->ac", G, Dn), rtol=1e-12,
                               atol=1e-13 * np.max(np.abs(Kref)))
    Dn = Dn + Dn.T
    assert np.trace(Dn @ oracle.kbuild(b, Dn, tau=0.0)) > 0


def test_derivative_integrals_finite_difference():
    """d(ab|cd)/dA_x from 2 zeta (a+1_x ...) - a_x (a-1_x ...) matches central
    differences; the four centre derivatives sum to zero (translation)."""
    rng = np.random.default_rng(8)
    ls = (1, 2, 0, 3)
    b, ex, co, cen = _rand_basis(ls, [2, 1, 1, 1], rng)
    d = oracle.eri4_deriv(b, 0, 1, 2, 3)
    scale = np.max(np.abs(d))
    np.testing.assert_allclose(d.sum(axis=0), 0.0, atol=1e-12 * scale)
    h = 1e-4
    for w in range(4):
        for x in range(3):
            cp, cm = cen.copy(), cen.copy()
            cp[w, x] += h
            cm[w, x] -= h
            Vp = oracle.eri4_shellset(oracle.Basis(b.l, b.nprim, b.exps, b.coefs, cp, 1), 0, 1, 2, 3)
            Vm = oracle.eri4_shellset(oracle.Basis(b.l, b.nprim, b.exps, b.coefs, cm, 1), 0, 1, 2, 3)
            fd = (Vp - Vm) / (2 * h)
            assert np.max(np.abs(fd - d[w, x])) < 1e-7 * scale


def test_exchange_gradient_finite_difference():
    """dE/dR for E = tr(D K) = sum D_ac D_bd (ab|cd) against central
    differences of the oracle's own K (h = 1e-4 bohr) and translational
    invariance of the analytic gradient."""
    rng = np.random.default_rng(12)
    ls, K, ex, co, cen, atom, pos = _tiny_molecule(rng, shells_per_atom=((0, 1), (1, 1), (2, 1)))
    b = oracle.Basis(ls, K, ex, co, cen, 1)
    nao = b.nao()
    C = rng.normal(size=(nao, 2))
    D = C @ C.T
    g = oracle.exchange_grad(b, atom, len(pos), D, tau=0.0)
    assert np.max(np.abs(g.sum(axis=0))) < 1e-11 * np.max(np.abs(g))
    h = 1e-4

    def energy(p):
        bb = oracle.Basis(ls, K, ex, co, p[atom], 1)
        return float(np.sum(D * oracle.kbuild(bb, D, tau=0.0)))

    for a in range(len(pos)):
        for x in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[a, x] += h
            pm[a, x] -= h
            fd = (energy(pp) - energy(pm)) / (2 * h)
            assert abs(fd - g[a, x]) < 1e-6 * np.max(np.abs(g)), (a, x, fd, g[a, x])


def test_matrix_form_reference_matches_oracle():
    """The matrix-form assembly used for l = 5, 6 parity (tests/ref/md_matrix)
    equals the sum-form oracle where both run: contracted, mixed classes."""
    from paper_2405_01834_amd import inputs
    from tests.ref import md_matrix
    rng = np.random.default_rng(31)
    sh = inputs.random_shells(rng, [2, 1, 3, 0, 2, 2], [2, 1, 1, 3, 1, 2], 3.0, 0.1, 20.0)
    ob = oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1)
    for q in ((0, 1, 2, 3), (4, 5, 0, 2), (2, 0, 5, 1)):
        ref = oracle.eri4(ob, [q[:2]], [q[2:]])[0, :, :, 0]
        got = md_matrix.shellset(sh, *q)
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))), q


def test_jbuild_matches_explicit_contraction():
    """J_ab = sum_cd (ab|cd) D_cd against an einsum over the full ERI tensor,
    with an unsymmetric D (catches a transposed operand); tr(DJ) >= 0 for a
    symmetric D (the Coulomb self-energy of a charge distribution)."""
    rng = np.random.default_rng(15)
    ls, K, ex, co, cen, atom, pos = _tiny_molecule(rng)
    b = oracle.Basis(ls, K, ex, co, cen, 1)
    nao = b.nao()
    G = _full_eri(b)
    Dn = rng.normal(size=(nao, nao))
    Jref = np.einsum("abcd,cd->ab", G, Dn)
    np.testing.assert_allclose(oracle.jbuild(b, Dn, tau=0.0), Jref, rtol=1e-12, atol=1e-13 * np.max(np.abs(Jref)))
    Ds = Dn + Dn.T
    assert np.sum(Ds * oracle.jbuild(b, Ds, tau=0.0)) > 0


def test_fock_blocks_match_full_builds():
    """Shell blocks of K and J from the restricted brute force equal the same
    blocks of the full builds, with screening active (tau = 1e-4 drops the
    quartets of distant pairs here, so both must apply the same rule)."""
    rng = np.random.default_rng(16)
    ls, K, ex, co, cen, atom, pos = _tiny_molecule(rng, natom=3, spread=9.0)
    b = oracle.Basis(ls, K, ex, co, cen, 1)
    nao = b.nao()
    D = rng.normal(size=(nao, nao))
    off = np.concatenate([[0], np.cumsum(2 * np.asarray(ls) + 1)])
    tau = 1e-4
    Kf, Jf = oracle.kbuild(b, D, tau=tau), oracle.jbuild(b, D, tau=tau)
    assert np.max(np.abs(Kf - oracle.kbuild(b, D, tau=0.0))) > 0  # screening is active
    blocks = [(0, 0), (1, 4), (4, 1), (2, len(ls) - 1), (len(ls) - 1, 3)]
    for which, full in (("K", Kf), ("J", Jf)):
        got = oracle.fock_blocks(b, D, blocks, which=which, tau=tau)
        for (s0, s1), blk in zip(blocks, got):
            ref = full[off[s0]:off[s0 + 1], off[s1]:off[s1 + 1]]
            np.testing.assert_allclose(blk, ref, rtol=1e-12, atol=1e-14 * np.max(np.abs(full)))


@pytest.mark.parametrize("pattern", ["exchange", "coulomb"])
def test_pattern_gradient_finite_difference(pattern):
    """dE/dR for E = tr(Wl K[Wr]) (exchange weights Wl_ac Wr_bd) and
    E = tr(Wl J[Wr]) (Coulomb weights Wl_ab Wr_cd), Wl != Wr and both
    unsymmetric, against central differences of the oracle's own K and J
    (h = 1e-4 bohr); translational invariance of the analytic gradient."""
    rng = np.random.default_rng(21 if pattern == "exchange" else 22)
    ls, K, ex, co, cen, atom, pos = _tiny_molecule(rng, shells_per_atom=((0, 1), (1, 1), (2, 1)))
    b = oracle.Basis(ls, K, ex, co, cen, 1)
    nao = b.nao()
    Wl, Wr = rng.normal(size=(nao, nao)), rng.normal(size=(nao, nao))
    g = oracle.grad_pattern(b, atom, len(pos), pattern, Wl, Wr, tau=0.0)
    scale = np.max(np.abs(g))
    assert np.max(np.abs(g.sum(axis=0))) < 1e-11 * scale
    build = oracle.kbuild if pattern == "exchange" else oracle.jbuild

    def energy(p):
        bb = oracle.Basis(ls, K, ex, co, p[atom], 1)
        return float(np.sum(Wl * build(bb, Wr, tau=0.0)))

    h = 1e-4
    for a in range(len(pos)):
        for x in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[a, x] += h
            pm[a, x] -= h
            fd = (energy(pp) - energy(pm)) / (2 * h)
            assert abs(fd - g[a, x]) < 1e-6 * scale, (a, x, fd, g[a, x])


def test_exchange_pattern_is_the_exchange_gradient():
    """With Wl = Wr = D the exchange-pattern gradient is dE/dR of tr(D K[D])."""
    rng = np.random.default_rng(23)
    ls, K, ex, co, cen, atom, pos = _tiny_molecule(rng, shells_per_atom=((0, 1), (1, 1), (2, 1)))
    b = oracle.Basis(ls, K, ex, co, cen, 1)
    C = rng.normal(size=(b.nao(), 2))
    D = C @ C.T
    g1 = oracle.grad_pattern(b, atom, len(pos), "exchange", D, D, tau=0.0)
    g0 = oracle.exchange_grad(b, atom, len(pos), D, tau=0.0)
    np.testing.assert_allclose(g1, g0, rtol=1e-12, atol=1e-13 * np.max(np.abs(g0)))


# ---------------------------------------------------------------------------
# 2-centre Coulomb metric (a|c)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("la,lc,K", [(0, 0, (2, 1)), (1, 2, (1, 2)), (3, 1, (2, 2)), (4, 4, (1, 1)), (6, 2, (1, 1)),
                                     (8, 3, (1, 1)), (7, 7, (1, 1))])
def test_two_centre_against_obara_saika(la, lc, K):
    """(a|c) equals the 4-centre (a s0|c s0) with s functions of exponent 0 and
    coefficient 1 (a Gaussian times the constant 1), evaluated independently
    by OS/HGP on raw shells; compared after the (separately pinned) solid
    transform."""
    rng = np.random.default_rng(40 + 7 * la + lc)
    ls = [la, lc]
    ex = [np.exp(rng.uniform(np.log(0.3), np.log(3), k)) for k in K]
    co = [rng.uniform(0.2, 1.0, k) for k in K]
    cen = rng.uniform(-1, 1, (2, 3))
    b = oracle.Basis(ls, list(K), np.concatenate(ex), np.concatenate(co), cen, 0)
    V = oracle.eri2(b, [0], [1])[0, :, :, 0]
    ref_c = contracted_eri_cart([(la, ex[0], co[0], cen[0]), (0, [0.0], [1.0], cen[0]),
                                 (lc, ex[1], co[1], cen[1]), (0, [0.0], [1.0], cen[1])], dps=25)[:, 0, :, 0]
    ref = oracle.solid(la) @ ref_c @ oracle.solid(lc).T
    # 1e-12 of the largest element (the parity bar): the solid transform of
    # the raw (4|4) block cancels about two digits in double precision
    assert np.max(np.abs(V - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_two_centre_ss_closed_form():
    """Normalised primitive s shells: (s_a|s_c) = N_a N_c 2 pi^{5/2} /
    (a c sqrt(a+c)) F_0(a c R^2 / (a+c)), N = (2 z / pi)^{3/4}, with F_0 from
    erf in mpmath."""
    a, c = 0.7, 2.3
    cen = np.array([[0.1, -0.2, 0.3], [0.9, 0.4, -0.5]])
    b = oracle.Basis([0, 0], [1, 1], np.array([a, c]), np.array([1.0, 1.0]), cen, 1)
    v = oracle.eri2(b, [0], [1]).ravel()[0]
    with mp.workdps(30):
        R2 = mp.mpf(float(np.sum((cen[0] - cen[1]) ** 2)))
        x = mp.mpf(a) * c / (a + c) * R2
        F0 = mp.sqrt(mp.pi / x) / 2 * mp.erf(mp.sqrt(x))
        ref = (2 * mp.mpf(a) / mp.pi) ** 0.75 * (2 * mp.mpf(c) / mp.pi) ** 0.75 * 2 * mp.pi ** 2.5 / (
            mp.mpf(a) * c * mp.sqrt(mp.mpf(a) + c)) * F0
    assert abs(v - float(ref)) <= 1e-14 * abs(float(ref))


def test_two_centre_metric_symmetric_positive_definite():
    """The Coulomb metric of a set of shells (mixed l, contracted, several
    centres) is symmetric, (a|c) = (c|a)^T, and positive definite (the Coulomb
    operator is a positive kernel)."""
    rng = np.random.default_rng(11)
    ls = [0, 1, 2, 3, 0, 2, 4, 1]
    K = [2, 1, 1, 2, 1, 2, 1, 1]
    b, *_ = _rand_basis(ls, K, rng, box=3.0)
    n = sum(2 * l + 1 for l in ls)
    off = np.concatenate([[0], np.cumsum([2 * l + 1 for l in ls])])
    M = np.zeros((n, n))
    for i in range(len(ls)):
        for k in range(len(ls)):
            M[off[i]:off[i + 1], off[k]:off[k + 1]] = oracle.eri2(b, [i], [k])[0, :, :, 0]
    assert np.max(np.abs(M - M.T)) <= 1e-14 * np.max(np.abs(M))
    assert np.min(np.linalg.eigvalsh(M)) > 0.0


@pytest.mark.parametrize("la,lb,lP", [(2, 1, 8), (0, 0, 7), (3, 3, 8)])
def test_three_centre_high_aux_l_against_obara_saika(la, lb, lP):
    """(ab|P) with an auxiliary shell of l = 7, 8 against OS/HGP on (ab|P s0)
    (raw single primitives), solid transforms in double."""
    rng = np.random.default_rng(60 + la + 3 * lb + 7 * lP)
    ls = [la, lb, lP]
    ex = [np.exp(rng.uniform(np.log(0.3), np.log(3), 1)) for _ in ls]
    cen = rng.uniform(-1, 1, (3, 3))
    prim = oracle.Basis(ls[:2], [1, 1], np.concatenate(ex[:2]), np.ones(2), cen[:2], 0)
    aux = oracle.Basis(ls[2:], [1], ex[2], np.ones(1), cen[2:], 0)
    V = oracle.eri3(prim, aux, [[0, 1]], [0])[0, :, :, 0]
    ref_c = contracted_eri_cart([(la, ex[0], [1.0], cen[0]), (lb, ex[1], [1.0], cen[1]),
                                 (lP, ex[2], [1.0], cen[2]), (0, [0.0], [1.0], cen[2])], dps=30)[..., 0]
    ref = np.einsum("ai,bj,ck,ijk->abc", oracle.solid(la), oracle.solid(lb), oracle.solid(lP), ref_c).reshape(V.shape)
    assert np.max(np.abs(V - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_dfj_exact_when_products_are_in_the_fitting_set():
    """s shells of single primitives: phi_i phi_j is one s Gaussian of exponent
    a_i + a_j at P_ij, so with those products as the fitting set the pair
    density lies in its span and density-fitted J equals the exact J (the
    oracle's brute force)."""
    rng = np.random.default_rng(31)
    n = 3
    ex = np.exp(rng.uniform(np.log(0.3), np.log(3.0), n))
    cen = rng.uniform(-1.0, 1.0, (n, 3))
    b = oracle.Basis([0] * n, [1] * n, ex, np.ones(n), cen, 1)
    pe, pc = [], []
    for i in range(n):
        for j in range(i, n):
            pe.append(ex[i] + ex[j])
            pc.append((ex[i] * cen[i] + ex[j] * cen[j]) / (ex[i] + ex[j]))
    aux = oracle.Basis([0] * len(pe), [1] * len(pe), np.array(pe), np.ones(len(pe)), np.array(pc), 1)
    C = rng.normal(size=(n, n))
    D = C @ C.T
    J = oracle.jbuild(b, D)
    Jdf = oracle.dfj(b, aux, D)
    assert np.max(np.abs(Jdf - J)) <= 1e-10 * np.max(np.abs(J))


def test_dfj_energy_is_variational():
    """The fitted Coulomb energy never exceeds the exact one:
    tr(D J_df) = gamma^T M^{-1} gamma <= tr(D J), the fitting error being
    non-negative in the Coulomb norm (mixed l, incomplete fitting set)."""
    rng = np.random.default_rng(32)
    ls = [0, 1, 0, 2]
    b = oracle.Basis(ls, [1] * 4, np.exp(rng.uniform(np.log(0.3), np.log(3), 4)), np.ones(4),
                     rng.uniform(-1, 1, (4, 3)), 1)
    aux = oracle.Basis([0, 1, 2, 0, 1], [1] * 5, np.exp(rng.uniform(np.log(0.2), np.log(4), 5)), np.ones(5),
                       rng.uniform(-1, 1, (5, 3)), 1)
    nao = b.nao()
    C = rng.normal(size=(nao, 3))
    D = C @ C.T
    J = oracle.jbuild(b, D)
    Jdf = oracle.dfj(b, aux, D)
    E, Edf = float(np.sum(D * J)), float(np.sum(D * Jdf))
    assert 0.0 < Edf <= E * (1 + 1e-12)


def test_dfk_exact_when_products_are_in_the_fitting_set():
    """With the pair products of single-primitive s shells as the fitting set
    every (ab| lies in its span, the fitted integrals are exact and the
    density-fitted K equals the exact K (the oracle's brute force)."""
    rng = np.random.default_rng(33)
    n = 3
    ex = np.exp(rng.uniform(np.log(0.3), np.log(3.0), n))
    cen = rng.uniform(-1.0, 1.0, (n, 3))
    b = oracle.Basis([0] * n, [1] * n, ex, np.ones(n), cen, 1)
    pe, pc = [], []
    for i in range(n):
        for j in range(i, n):
            pe.append(ex[i] + ex[j])
            pc.append((ex[i] * cen[i] + ex[j] * cen[j]) / (ex[i] + ex[j]))
    aux = oracle.Basis([0] * len(pe), [1] * len(pe), np.array(pe), np.ones(len(pe)), np.array(pc), 1)
    C = rng.normal(size=(n, n))
    D = C @ C.T
    K = oracle.kbuild(b, D)
    Kdf = oracle.dfk(b, aux, D)
    assert np.max(np.abs(Kdf - K)) <= 1e-10 * np.max(np.abs(K))


def test_dfk_exchange_energy_is_variational():
    """For D = sum_k c_k c_k^T, tr(D K) = sum_kl (phi_k phi_l | phi_k phi_l) is a
    sum of Coulomb self-energies of pair densities, and fitting each in the
    Coulomb metric can only lower it: 0 < tr(D K_df) <= tr(D K) (mixed l,
    incomplete fitting set); K_df is symmetric."""
    rng = np.random.default_rng(34)
    ls = [0, 1, 0, 2]
    b = oracle.Basis(ls, [1] * 4, np.exp(rng.uniform(np.log(0.3), np.log(3), 4)), np.ones(4),
                     rng.uniform(-1, 1, (4, 3)), 1)
    aux = oracle.Basis([0, 1, 2, 0, 1, 3], [1] * 6, np.exp(rng.uniform(np.log(0.2), np.log(4), 6)), np.ones(6),
                       rng.uniform(-1, 1, (6, 3)), 1)
    nao = b.nao()
    C = rng.normal(size=(nao, 3))
    D = C @ C.T
    K = oracle.kbuild(b, D)
    Kdf = oracle.dfk(b, aux, D)
    E, Edf = float(np.sum(D * K)), float(np.sum(D * Kdf))
    assert 0.0 < Edf <= E * (1 + 1e-12)
    assert Edf < 0.999 * E  # the set is incomplete: the fit loses something
    assert np.max(np.abs(Kdf - Kdf.T)) <= 1e-13 * np.max(np.abs(Kdf))

