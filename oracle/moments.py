"""Exact construction of the D3Q19 velocity set and both MRT moment bases.

Test infrastructure (see ``oracle/__init__``).  Everything here is rational
arithmetic with :class:`fractions.Fraction`; the FP64 arrays handed to the C
step are the correctly rounded images of the exact entries.

Pins (tests/test_oracle_moments.py):
  * ``nonorth_M`` equals the matrix printed as Eq. (12) (golden fixture) and
    has 145 non-zeros (text after Eq. (12)).
  * ``exact_inverse`` gives M M^-1 = I exactly; it equals the matrix printed
    in Appendix A except for the two entries the printed table misplaces
    (rows 13 and 14, column 7 vs 8); 99 non-zeros.
  * C_i = M E_i M^-1 reproduces every coefficient of Eqs. (24)-(27) and
    (36)-(41) (Sec. III).
  * ``orth_M`` has 213 non-zeros and so does its inverse (text after
    Eq. (12)); its rows are mutually orthogonal.
  * equilibria recover rho and rho*u; rest state gives the textbook weights.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr

import numpy as np

# Eq. (2): the 19 velocities, columns of the printed 3x19 matrix, in order.
VELOCITIES = (
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
)
Q = 19


def opposite(a: int) -> int:
    """Index of -e_a (Eq. (2) lists opposite velocities as neighbours)."""
    ex, ey, ez = VELOCITIES[a]
    return VELOCITIES.index((-ex, -ey, -ez))


def nonorth_basis(e) -> list[int]:
    """Row values M_{k,alpha} for one velocity, Eqs. (7)-(10) in order k=0..18."""
    x, y, z = e
    n2 = x * x + y * y + z * z
    return [
        1, x, y, z,                                   # Eq. (7)
        n2, 3 * x * x - n2, y * y - z * z,            # Eq. (8)
        x * y, x * z, y * z,
        x * x * y, x * y * y, x * x * z,              # Eq. (9)
        x * z * z, y * y * z, y * z * z,
        x * x * y * y, x * x * z * z, y * y * z * z,  # Eq. (10)
    ]


def nonorth_M() -> list[list[int]]:
    """Transformation matrix of Eq. (12), built from the basis (rows = moments)."""
    cols = [nonorth_basis(e) for e in VELOCITIES]
    return [[cols[a][k] for a in range(Q)] for k in range(Q)]


def exact_inverse(M) -> list[list[Fr]]:
    """Gauss-Jordan inverse in exact rationals (raises if singular)."""
    n = len(M)
    A = [[Fr(M[i][j]) for j in range(n)] + [Fr(int(i == j)) for j in range(n)]
         for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        piv = A[c][c]
        A[c] = [v / piv for v in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                k = A[r][c]
                A[r] = [a - k * b for a, b in zip(A[r], A[c])]
    return [row[n:] for row in A]


def matmul_exact(A, B):
    return [[sum(Fr(A[i][k]) * Fr(B[k][j]) for k in range(len(B)))
             for j in range(len(B[0]))] for i in range(len(A))]


# ---------------------------------------------------------------------------
# Orthogonal comparison model.  The paper constructs it by Gram-Schmidt
# orthogonalisation of polynomials of the velocity components (Sec. I) and
# cites the usual D3Q19 ordering; the seed polynomials below, taken in order,
# give the rho, e, epsilon, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww,
# pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z rows.
# ---------------------------------------------------------------------------
ORTH_ROW_NAMES = ("rho", "e", "eps", "jx", "qx", "jy", "qy", "jz", "qz",
                  "3pxx", "3pixx", "pww", "piww", "pxy", "pyz", "pxz",
                  "mx", "my", "mz")


def _orth_seed(e) -> list[int]:
    x, y, z = e
    n = x * x + y * y + z * z
    return [1, n, n * n, x, n * x, y, n * y, z, n * z,
            3 * x * x - n, n * (3 * x * x - n), y * y - z * z, n * (y * y - z * z),
            x * y, y * z, x * z,
            (y * y - z * z) * x, (z * z - x * x) * y, (x * x - y * y) * z]


def orth_M() -> list[list[int]]:
    """Gram-Schmidt over the 19 velocities; each row scaled to coprime integers
    by a positive factor (so the sign follows its seed polynomial)."""
    seeds = [[Fr(_orth_seed(e)[k]) for e in VELOCITIES] for k in range(Q)]
    rows: list[list[Fr]] = []
    for s in seeds:
        r = list(s)
        for q in rows:
            c = sum(a * b for a, b in zip(r, q)) / sum(b * b for b in q)
            r = [a - c * b for a, b in zip(r, q)]
        den = 1
        for v in r:
            den = den * v.denominator // math.gcd(den, v.denominator)
        iv = [int(v * den) for v in r]
        g = 0
        for v in iv:
            g = math.gcd(g, abs(v))
        rows.append([Fr(v // g) for v in iv])
    return [[int(v) for v in r] for r in rows]


def to_f64(A) -> np.ndarray:
    """Correctly rounded FP64 image of an exact matrix."""
    return np.array([[float(Fr(v)) for v in row] for row in A], dtype=np.float64)


def nnz(A) -> int:
    return sum(1 for row in A for v in row if v != 0)


# Relaxation-rate vectors (diagonal of Lambda).
def nonorth_rates(s_e, s_nu, s_q, s_pi) -> list[float]:
    """Eq. (11): conserved moments at 1, then s_e, s_nu x5, s_q x6, s_pi x3."""
    return [1.0, 1.0, 1.0, 1.0, s_e] + [s_nu] * 5 + [s_q] * 6 + [s_pi] * 3


def orth_rates(s_e, s_nu, s_q, s_pi, s_eps, s_m) -> list[float]:
    """Rates by row of ``orth_M``: conserved rows (rho, j) at 1, e -> s_e,
    eps -> s_eps, q -> s_q, the five second-order stress rows -> s_nu, the two
    pi rows -> s_pi, the three cubic m rows -> s_m."""
    r = {"rho": 1.0, "jx": 1.0, "jy": 1.0, "jz": 1.0, "e": s_e, "eps": s_eps,
         "qx": s_q, "qy": s_q, "qz": s_q,
         "3pxx": s_nu, "pww": s_nu, "pxy": s_nu, "pyz": s_nu, "pxz": s_nu,
         "3pixx": s_pi, "piww": s_pi, "mx": s_m, "my": s_m, "mz": s_m}
    return [r[n] for n in ORTH_ROW_NAMES]


# Rows relaxed at s_nu (the five second-order stress moments).
NONORTH_NU_ROWS = (5, 6, 7, 8, 9)


def orth_nu_rows() -> tuple[int, ...]:
    return tuple(ORTH_ROW_NAMES.index(n) for n in ("3pxx", "pww", "pxy", "pyz", "pxz"))


def orth_sigma_rows() -> tuple[int, int]:
    """Rows of the orthogonal basis that receive the thermodynamic-consistency
    correction: the image under ``orth_M`` of the velocity-space vector that
    Eq. (16) adds through row 4 of the non-orthogonal model, i.e. column 4 of
    the exact non-orthogonal inverse.  Returns the (e, eps) coefficients.
    Parity unpinned against the paper beyond the equal-rate limit."""
    Mi = exact_inverse(nonorth_M())
    col4 = [Mi[a][4] for a in range(Q)]
    Mo = orth_M()
    img = [sum(Fr(Mo[k][a]) * col4[a] for a in range(Q)) for k in range(Q)]
    assert all(v == 0 for i, v in enumerate(img) if i not in (1, 2))
    return int(img[1]), int(img[2])


def c_matrices(M, Minv):
    """C_i = M E_i M^-1 for i = x, y, z (Sec. III, definition after Eq. (22))."""
    out = []
    for i in range(3):
        Ei = [[Fr(VELOCITIES[a][i]) if a == b else Fr(0) for b in range(Q)]
              for a in range(Q)]
        out.append(matmul_exact(matmul_exact(M, Ei), Minv))
    return out
