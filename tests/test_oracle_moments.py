"""Pins of the oracle's transformation matrices against what the paper prints
and what the mathematics fixes (exact rational arithmetic throughout)."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import moments
from tests.golden_io import paper_values, read_matrix

Q = 19


def test_velocity_set_eq2():
    # Eq. (2): rest, 6 axis and 12 diagonal velocities, opposites adjacent.
    E = moments.VELOCITIES
    assert len(set(E)) == 19
    assert sorted(sum(c * c for c in e) for e in E) == [0] + [1] * 6 + [2] * 12
    for a in range(1, 19, 2):
        assert moments.opposite(a) == a + 1


def test_M_equals_printed_eq12():
    M = moments.nonorth_M()
    printed = read_matrix("eq12_M.txt")
    assert [[Fr(v) for v in r] for r in M] == printed
    assert moments.nnz(M) == paper_values()["nnz_M"]["value"]


def test_exact_inverse_identity_and_nnz():
    M = moments.nonorth_M()
    Mi = moments.exact_inverse(M)
    I = moments.matmul_exact(M, Mi)
    assert all(I[i][j] == (1 if i == j else 0) for i in range(Q) for j in range(Q))
    I2 = moments.matmul_exact(Mi, M)
    assert all(I2[i][j] == (1 if i == j else 0) for i in range(Q) for j in range(Q))
    # The text claims 96 non-zeros; the exact inverse has 99.
    assert moments.nnz(Mi) == 99
    assert paper_values()["nnz_Minv_printed_claim"]["value"] == 96


def test_exact_inverse_vs_printed_appendix_a():
    """Appendix A agrees with the exact inverse except in rows 13 and 14, where
    the printed -1/4 sits in column 7 (m_7 = e_x e_y) instead of column 8
    (m_8 = e_x e_z); velocities 13, 14 = (1,0,-1), (-1,0,1) have e_x e_y = 0."""
    Mi = moments.exact_inverse(moments.nonorth_M())
    printed = read_matrix("appA_Minv.txt")
    diffs = [(a, k) for a in range(Q) for k in range(Q) if Mi[a][k] != printed[a][k]]
    assert sorted(diffs) == [(13, 7), (13, 8), (14, 7), (14, 8)]
    for a in (13, 14):
        assert printed[a][7] == Fr(-1, 4) and printed[a][8] == 0
        assert Mi[a][7] == 0 and Mi[a][8] == Fr(-1, 4)
    # As printed, the table is not an inverse and breaks mass conservation:
    # column 7 of a valid inverse must sum to zero (sum_a Minv[a][k] = delta_k0).
    M = moments.nonorth_M()
    bad = moments.matmul_exact(M, printed)
    assert any(bad[i][j] != (1 if i == j else 0) for i in range(Q) for j in range(Q))
    assert sum(printed[a][7] for a in range(Q)) == Fr(-1, 2)
    assert sum(printed[a][8] for a in range(Q)) == Fr(1, 2)
    for k in range(Q):
        assert sum(Mi[a][k] for a in range(Q)) == (1 if k == 0 else 0)


def _row(**coef):
    r = [Fr(0)] * Q
    for k, v in coef.items():
        r[int(k[1:])] = Fr(v)
    return r


def test_chapman_enskog_C_rows():
    """C_i = M E_i M^-1 (after Eq. (22)) reproduces the flux coefficients printed
    in Eqs. (24)-(27) and (36)-(41)."""
    M = moments.nonorth_M()
    Cx, Cy, Cz = moments.c_matrices(M, moments.exact_inverse(M))
    third, sixth, half = Fr(1, 3), Fr(1, 6), Fr(1, 2)
    expect = {
        # Eq. (24)
        0: (_row(k1=1), _row(k2=1), _row(k3=1)),
        # Eq. (25)
        1: (_row(k4=third, k5=third), _row(k7=1), _row(k8=1)),
        # Eq. (26)
        2: (_row(k7=1), _row(k4=third, k5=-sixth, k6=half), _row(k9=1)),
        # Eq. (27)
        3: (_row(k8=1), _row(k9=1), _row(k4=third, k5=-sixth, k6=-half)),
        # Eq. (36)
        4: (_row(k1=1, k11=1, k13=1), _row(k2=1, k10=1, k15=1), _row(k3=1, k12=1, k14=1)),
        # Eq. (37)
        5: (_row(k1=2, k11=-1, k13=-1), _row(k2=-1, k10=2, k15=-1), _row(k3=-1, k12=2, k14=-1)),
        # Eq. (38)
        6: (_row(k11=1, k13=-1), _row(k2=1, k15=-1), _row(k3=-1, k14=1)),
        # Eqs. (39)-(41)
        7: (_row(k10=1), _row(k11=1), _row()),
        8: (_row(k12=1), _row(), _row(k13=1)),
        9: (_row(), _row(k14=1), _row(k15=1)),
    }
    for k, (ex, ey, ez) in expect.items():
        assert Cx[k] == ex, k
        assert Cy[k] == ey, k
        assert Cz[k] == ez, k


def test_orthogonal_basis_counts_and_orthogonality():
    Mo = moments.orth_M()
    assert moments.nnz(Mo) == paper_values()["nnz_orthogonal_M_and_inverse"]["value"]
    Moi = moments.exact_inverse(Mo)
    assert moments.nnz(Moi) == 213
    D = [sum(v * v for v in r) for r in Mo]
    for i in range(Q):
        for j in range(Q):
            dot = sum(a * b for a, b in zip(Mo[i], Mo[j]))
            assert dot == (D[i] if i == j else 0)
    # Inverse of an orthogonal-row matrix is M^T D^-1.
    for a in range(Q):
        for k in range(Q):
            assert Moi[a][k] == Fr(Mo[k][a], D[k])
    # First rows are the conserved moments and their standard energy polynomials.
    E = moments.VELOCITIES
    assert Mo[0] == [1] * Q
    assert Mo[1] == [19 * sum(c * c for c in e) - 30 for e in E]
    assert Mo[3] == [e[0] for e in E]


def test_orth_sigma_rows_image_of_eq16_vector():
    # The velocity-space vector through which Eq. (16) acts (column 4 of M^-1)
    # maps onto the e and eps rows of the orthogonal basis only.
    assert moments.orth_sigma_rows() == (19, -16)


def test_to_f64_is_correctly_rounded():
    Mi = moments.exact_inverse(moments.nonorth_M())
    A = moments.to_f64(Mi)
    assert A[3, 5] == -1.0 / 12.0 and A[1, 4] == 1.0 / 6.0
    assert np.all(np.isin(np.unique(A), [0.0, 1.0, -1.0, 0.5, -0.5, 0.25, -0.25, 1 / 6, -1 / 12]))


@pytest.mark.parametrize("op", ["nonorth", "orth"])
def test_rates_layout(op):
    if op == "nonorth":
        r = moments.nonorth_rates(1.1, 1.0, 1.2, 1.4)
        assert r == [1, 1, 1, 1, 1.1, 1, 1, 1, 1, 1, 1.2, 1.2, 1.2, 1.2, 1.2, 1.2, 1.4, 1.4, 1.4]
    else:
        r = moments.orth_rates(1.1, 1.0, 1.2, 1.4, 1.5, 1.6)
        names = moments.ORTH_ROW_NAMES
        d = dict(zip(names, r))
        assert d["e"] == 1.1 and d["eps"] == 1.5 and d["mx"] == 1.6 and d["qy"] == 1.2
        assert d["pxy"] == d["3pxx"] == d["pww"] == 1.0 and d["3pixx"] == d["piww"] == 1.4


def test_orth_equilibrium_rows_in_closed_form():
    """The orthogonal model's default equilibrium and forcing moments
    (M_orth f_eq with the textbook D3Q19 f_eq, M_orth G with Guo's G) have the
    closed forms that the kernel evaluates with free parameters:
    eps_eq = rho (3 - 11/2 |u|^2), 3pi_xx = -(1/2) 3p_xx, pi_ww = -(1/2) p_ww,
    S_eps = -11 F.u, and the pi source rows -1/2 of the p source rows.  The
    other reading of the model (orth_meq = 1) changes exactly these three
    rows (and their sources) to w_eps = 0, w_epsj = -475/63, w_xx = 0."""
    M = np.array(moments.orth_M(), dtype=float)
    E = np.array(moments.VELOCITIES, dtype=float)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    names = moments.ORTH_ROW_NAMES
    ie, ipxx, iixx, ipww, iiww = (names.index(n) for n in ("eps", "3pxx", "3pixx", "pww", "piww"))
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho = rng.uniform(0.1, 2.0)
        u = rng.uniform(-0.1, 0.1, 3)
        F = rng.uniform(-1e-2, 1e-2, 3)
        eu, eF = E @ u, E @ F
        feq = w * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * u @ u)
        G = w * (3 * (eF - F @ u) + 9 * eu * eF)
        m, S = M @ feq, M @ G
        assert abs(m[ie] - rho * (3 - 5.5 * (u @ u))) < 1e-13
        assert abs(m[iixx] + 0.5 * m[ipxx]) < 1e-13 and abs(m[iiww] + 0.5 * m[ipww]) < 1e-13
        assert abs(S[ie] - 2 * (-5.5) * (F @ u)) < 1e-15
        assert abs(S[iixx] + 0.5 * S[ipxx]) < 1e-15 and abs(S[iiww] + 0.5 * S[ipww]) < 1e-15
