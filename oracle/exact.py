"""Exact-rational recomputation of tiny cases (TEST INFRASTRUCTURE).

Pure Python with ``fractions.Fraction``: decodes bytes arithmetically, forms
the per-input sums, the normaliser window, the normalised array cumulants and
the estimator with no rounding at all. It is used to bound the FP64 oracle's
rounding error on tiny N, M, and to decide flags exactly. Paper equations as
in ``sk_oracle.c`` (Sec. 2.2.1, Eq. singlesums, discreteMean, normedSum1/2,
avgSK, final).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Optional


def decode(byte: int):
    return (byte >> 4) - 8, (byte & 15) - 8


def exact_sk(x, M: int, L: int, est: int = 0, mask=None):
    """x: nested [T][F][N] ints (bytes). Returns V[f][b] as Fraction or None (invalid)."""
    T = len(x)
    F = len(x[0])
    N = len(x[0][0])
    B = T // M
    S1 = [[[0] * N for _ in range(B)] for _ in range(F)]
    S2 = [[[0] * N for _ in range(B)] for _ in range(F)]
    for t in range(B * M):
        b = t // M
        for f in range(F):
            for i in range(N):
                re, im = decode(int(x[t][f][i]))
                p = re * re + im * im
                S1[f][b][i] += p
                S2[f][b][i] += p * p
    out: List[List[Optional[Fraction]]] = []
    for f in range(F):
        row = []
        for b in range(B):
            A = Fraction(0)
            Bq = Fraction(0)
            R1 = 0
            R2 = 0
            n = 0
            for i in range(N):
                if mask is not None and not mask[f][i]:
                    continue
                P = S1[f][b][i] if L == 0 else sum(S1[f][bb][i] for bb in range(max(0, b - L + 1), b + 1))
                if P <= 0:
                    continue
                n += 1
                R1 += S1[f][b][i]
                R2 += S2[f][b][i]
                A += Fraction(S1[f][b][i], P)
                Bq += Fraction(S2[f][b][i], P * P)
            K = n * M
            if K < 2 or (L == 0 and R1 == 0) or (L != 0 and A == 0):
                row.append(None)
                continue
            if L == 0:
                V = Fraction(K + 1, K - 1) * (Fraction(K * R2, R1 * R1) - 1)
            elif est == 1:
                V = Fraction(M + 1, M - 1) * (Fraction(M) * Bq / n - 1)
            else:
                V = Fraction(K + 1, K - 1) * (K * Bq / (A * A) - 1)
            row.append(V)
        out.append(row)
    return out
