"""D3Q19 lattice constants transcribed from the paper (oracle side).

Test infrastructure only (see ``oracle/__init__.py``).

Index convention: the paper numbers the velocities 1..19 with the rest
velocity last (App. B, Fig. d3q19_table).  Here index ``a`` (0-based) is the
paper's index ``a + 1``; opposite pairs are (0,1), (2,3), ..., (16,17) and the
rest velocity is 18.
"""
import numpy as np

# App. B, Fig. d3q19_table: velocities c_alpha (paper indices 1..19).
C = np.array([
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 0, 0),
], dtype=np.int64)

# App. B, Fig. d3q19_table: weights w_alpha.
W = np.array([1 / 18] * 6 + [1 / 36] * 12 + [1 / 3], dtype=np.float64)

# Opposite direction of each velocity (c_opp = -c).
OPP = np.array([1, 0, 3, 2, 5, 4, 7, 6, 9, 8, 11, 10, 13, 12, 15, 14, 17, 16, 18])

# App. B, eq. moment-matrix: the 19x19 orthogonal moment matrix M, row by row
# as printed; columns follow the velocity order above.
M = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, -30],
    [-4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 12],
    [1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0],
    [-4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0],
    [0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0, 0],
    [0, 0, -4, 4, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0],
    [0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0],
    [2, 2, -1, -1, -1, -1, 1, 1, 1, 1, -2, -2, -2, -2, 1, 1, 1, 1, 0],
    [-4, -4, 2, 2, 2, 2, 1, 1, 1, 1, -2, -2, -2, -2, 1, 1, 1, 1, 0],
    [0, 0, 1, 1, -1, -1, 1, 1, 1, 1, 0, 0, 0, 0, -1, -1, -1, -1, 0],
    [0, 0, -2, -2, 2, 2, 1, 1, 1, 1, 0, 0, 0, 0, -1, -1, -1, -1, 0],
    [0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0],
    [0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, -1, 1, -1, 1, 0],
    [0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 1, -1, -1, 1, 0],
], dtype=np.float64)

# M^{-1}, taken literally as the numerical inverse of M.
MINV = np.linalg.inv(M)

# App. B, eq. relaxation-matrix: the fixed rates of S.  The entries at rows
# 9, 11, 13, 14, 15 are s_nu (set per cell by the LES closure, Sec. 2.3).
S_RHO, S_E, S_EPS, S_J, S_Q, S_PI, S_M = 1.0, 1.19, 1.4, 1.0, 1.2, 1.4, 1.98
SHEAR_ROWS = (9, 11, 13, 14, 15)


def relaxation_diagonal(s_nu, s_e=S_E, s_eps=S_EPS, s_q=S_Q, s_pi=S_PI, s_m=S_M):
    """Diagonal of S (eq. relaxation-matrix) with s_nu broadcast per cell.

    Returns an array of shape (19,) + shape(s_nu).
    """
    s_nu = np.asarray(s_nu, dtype=np.float64)
    one = np.ones_like(s_nu)
    rows = [S_RHO * one, s_e * one, s_eps * one,
            S_J * one, s_q * one, S_J * one, s_q * one, S_J * one, s_q * one,
            s_nu, s_pi * one, s_nu, s_pi * one, s_nu, s_nu, s_nu,
            s_m * one, s_m * one, s_m * one]
    return np.stack(rows)
