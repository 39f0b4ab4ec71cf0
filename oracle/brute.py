"""Arbitrary-precision brute force of Eq. (gravity) for tiny N (mpmath).

TEST INFRASTRUCTURE ONLY.  Used to pin the FP64 reference on inputs of a few
particles, with every operation carried at ``dps`` decimal digits.
"""

from __future__ import annotations

import mpmath


def forces(x, m, eps2, dps: int = 50):
    """Lists (a [n][3], p [n]) of mpf values, paper sign, j != i."""
    with mpmath.workdps(dps):
        X = [[mpmath.mpf(float(c)) for c in row] for row in x]
        M = [mpmath.mpf(float(v)) for v in m]
        e2 = mpmath.mpf(float(eps2))
        n = len(X)
        A, P = [], []
        for i in range(n):
            acc = [mpmath.mpf(0)] * 3
            pot = mpmath.mpf(0)
            for j in range(n):
                if i == j:
                    continue
                d = [X[i][c] - X[j][c] for c in range(3)]
                s = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + e2
                pot += M[j] / mpmath.sqrt(s)
                for c in range(3):
                    acc[c] += M[j] * d[c] / s ** mpmath.mpf(1.5)
            A.append(acc)
            P.append(pot)
        return A, P
