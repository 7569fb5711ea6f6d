"""Plain Python-integer definitions of the RNS quantities -- test infrastructure.

These follow the paper's Sec. 3.1: a bignum X is represented by its residues
x_i = X mod m_i over pairwise-coprime moduli, and the Montgomery product with
R = M = prod(m_i) computes X*Y*M^-1 mod N channel by channel (the cited RNS
Montgomery algorithm of Bajard et al. 2001).  Each function below is the
closed-form definition of one quantity of that algorithm, written with Python
integers; none of them shares code with the GPU library.

Notation: B = (m_1..m_k) is the first base, M its product, M_i = M / m_i.
"""
from __future__ import annotations

from math import prod


def residues(x: int, moduli) -> list:
    """RNS representation of x (Sec. 3.1)."""
    return [x % m for m in moduli]


def crt(res, moduli) -> int:
    """The unique X < prod(moduli) with the given residues (CRT, Sec. 3.1)."""
    M = prod(moduli)
    x = 0
    for r, m in zip(res, moduli):
        Mi = M // m
        x += r * Mi * pow(Mi, -1, m)
    return x % M


def mont_quotient_digits(X: int, Y: int, N: int, B) -> list:
    """xi_i = |x_i y_i (-N^-1) M_i^-1|_{m_i}: the first step of the RNS
    Montgomery product, computed independently in each channel of B."""
    M = prod(B)
    out = []
    for m in B:
        Mi = M // m
        out.append((X * Y) % m * (-pow(N, -1, m)) % m * pow(Mi, -1, m) % m)
    return out


def mont_qhat(X: int, Y: int, N: int, B) -> int:
    """q^ = sum_i xi_i M_i: the first base extension's value, an integer
    congruent to -X*Y*N^-1 modulo M and lying in [0, k*M)."""
    M = prod(B)
    return sum(x * (M // m) for x, m in zip(mont_quotient_digits(X, Y, N, B), B))


def mont_mul(X: int, Y: int, N: int, B) -> int:
    """The integer r = (X*Y + q^*N) / M produced by the RNS Montgomery
    product over base B; r == X*Y*M^-1 (mod N)."""
    M = prod(B)
    t = X * Y + mont_qhat(X, Y, N, B) * N
    if t % M:
        raise ArithmeticError("X*Y + q^*N is not divisible by M")
    return t // M
