"""Exact rational Taylor series of exp(A) 1 for tiny integer graphs (brute force pin).

exp(A) 1 = sum_l A^l 1 / l!, and (A^l 1)_i is the number of walks of length l starting at node i
(the walk reading of communicability in "The total communicability"). For a 0/1 matrix these are
integers, so the partial sums are exact fractions; the series is cut where the remainder is below
`tail` (remainder of sum_{l>L} rho^l/l! * ||1||, rho <= max row sum).
"""
from __future__ import annotations

from fractions import Fraction
import math

import numpy as np


def ebtc_taylor_exact(A_int: np.ndarray, tail: float = 1e-30) -> list[Fraction]:
    A = [[int(x) for x in row] for row in np.asarray(A_int)]
    n = len(A)
    rho = max((sum(abs(x) for x in row) for row in A), default=0)
    walks = [1] * n
    acc = [Fraction(1)] * n
    l = 0
    fact = 1
    while True:
        l += 1
        fact *= l
        walks = [sum(A[i][j] * walks[j] for j in range(n)) for i in range(n)]
        acc = [acc[i] + Fraction(walks[i], fact) for i in range(n)]
        # remainder bound: sum_{k>l} rho^k / k! <= rho^(l+1)/(l+1)! * e^rho
        if rho == 0 or (rho ** (l + 1)) / math.factorial(l + 1) * math.exp(rho) < tail:
            return acc
