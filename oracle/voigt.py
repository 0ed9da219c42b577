"""Voigt <-> fourth-order tensor maps of the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Convention (the one the stiffness tables of the cells use): Voigt index I of the
symmetric pair (i, j) is 0, 1, 2 for (0,0), (1,1), (2,2) and 3, 4, 5 for (1,2),
(0,2), (0,1); the 6x6 matrix multiplies the strain with engineering shear
[e11, e22, e33, 2 e23, 2 e13, 2 e12] (Sec. 2.2: the stiffness has the minor and
major symmetries, so 21 numbers describe it).  The 21-entry form is the upper
triangle of the 6x6 matrix, row by row.

Pins (tests/test_oracle_operators.py): the isotropic tensor
lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk) from its Lame constants, the
minor and major symmetries, and the 21 <-> 6x6 round trip.
"""
from __future__ import annotations

import numpy as np


def voigt_index(i: int, j: int) -> int:
    """Voigt index of the symmetric index pair (i, j)."""
    return i if i == j else 6 - i - j


_VI = np.array([[voigt_index(i, j) for j in range(3)] for i in range(3)])


def voigt_to_tensor(C6: np.ndarray) -> np.ndarray:
    """C_ijkl = C6[I(i,j), I(k,l)]."""
    C6 = np.asarray(C6, dtype=np.float64)
    return C6[_VI[:, :, None, None], _VI[None, None, :, :]]


def c21_to_voigt(c21: np.ndarray) -> np.ndarray:
    """Symmetric 6x6 Voigt matrix from its upper triangle listed row by row."""
    C6 = np.zeros((6, 6))
    C6[np.triu_indices(6)] = np.asarray(c21, dtype=np.float64)
    return C6 + np.triu(C6, 1).T
