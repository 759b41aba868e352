"""Exact densities of states g(E) for the periodic 2D Ising and q-state Potts models.

TEST INFRASTRUCTURE ONLY (part of the oracle).  These exact counts pin the REWL
oracle and measure the accuracy of its estimates; the product never imports them.

Three independent routes, each exact in integer arithmetic:

* ``brute_force``      -- enumerate all q^N configurations (N <= 16).
* ``transfer_matrix``  -- Z(v) = Tr T(v)^L with T the row-to-row transfer matrix,
  v marking one broken bond; evaluated at 2N+1 points modulo several primes,
  interpolated, and lifted by the Chinese remainder theorem (Ising L <= 8,
  Potts q^L <= ~1000).
* ``kaufman_ising``    -- Kaufman's closed form of the torus partition function
  (Phys. Rev. 76, 1232 (1949)), which is a rational function of y = e^{2K}.
  It is evaluated exactly modulo primes p = 1 (mod 2n) on a coset of the n-th
  roots of unity, turned into coefficients by an inverse number-theoretic
  transform, and lifted by CRT: the exact integer DOS at any even L.

Energy bins follow the REWL code: Ising E = -sum s_i s_j, bin (E + 2N)/4;
Potts E = -sum delta(q_i, q_j) (Eq. (2) of the paper), bin E + 2N.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np


def n_bins(model: str, L: int) -> int:
    N = L * L
    return N + 1 if model == "ising" else 2 * N + 1


def _bin_of_broken(model: str, broken):
    """Broken (unsatisfied) bond count -> energy bin.  Ising E = -2N + 2*broken."""
    return broken // 2 if model == "ising" else broken


# --------------------------------------------------------------------------------------
# brute force
# --------------------------------------------------------------------------------------
def brute_force(model: str, q: int, L: int) -> list[int]:
    """Count every configuration of the L x L torus.  Returns g per energy bin."""
    N = L * L
    qq = 2 if model == "ising" else q
    if qq ** N > 2 ** 26:
        raise ValueError("too many states for brute force")
    idx = np.arange(qq ** N, dtype=np.int64)
    spins = np.empty((qq ** N, N), dtype=np.int8)
    for i in range(N):
        spins[:, i] = idx % qq
        idx //= qq
    grid = spins.reshape(-1, L, L)
    broken = (grid != np.roll(grid, 1, axis=2)).sum(axis=(1, 2)) + \
             (grid != np.roll(grid, 1, axis=1)).sum(axis=(1, 2))
    bins = _bin_of_broken(model, broken)
    counts = np.bincount(bins, minlength=n_bins(model, L))
    return [int(v) for v in counts]


# --------------------------------------------------------------------------------------
# modular helpers
# --------------------------------------------------------------------------------------
def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _primes(count: int, below: int, modulus: int = 2) -> list[int]:
    """`count` distinct primes p < below with p = 1 (mod modulus), largest first."""
    out = []
    p = ((below - 2) // modulus) * modulus + 1
    while len(out) < count:
        if p < modulus:
            raise ValueError("ran out of primes")
        if _is_prime(p):
            out.append(p)
        p -= modulus
    return out


def _crt(residues: list[list[int]], primes: list[int]) -> list[int]:
    """Lift residues (one list per prime) of non-negative integers < prod(primes)."""
    M = 1
    for p in primes:
        M *= p
    basis = []
    for p in primes:
        Mi = M // p
        basis.append(Mi * pow(Mi % p, -1, p))
    n = len(residues[0])
    out = []
    for k in range(n):
        x = 0
        for r, e in zip(residues, basis):
            x += int(r[k]) * e
        out.append(x % M)
    return out


def _interpolate_mod(xs: list[int], ys: list[int], p: int) -> list[int]:
    """Coefficients (low to high) of the polynomial through (xs, ys) over GF(p)."""
    n = len(xs)
    coef = [y % p for y in ys]
    for j in range(1, n):                      # Newton divided differences
        for i in range(n - 1, j - 1, -1):
            coef[i] = (coef[i] - coef[i - 1]) * pow(xs[i] - xs[i - j], -1, p) % p
    poly = [0] * n                             # expand the Newton form
    for i in range(n - 1, -1, -1):
        new = [0] * n
        for d in range(n - 1):
            new[d + 1] = (new[d + 1] + poly[d]) % p
            new[d] = (new[d] - xs[i] * poly[d]) % p
        new[0] = (new[0] + coef[i]) % p
        poly = new
    return poly


# --------------------------------------------------------------------------------------
# transfer matrix
# --------------------------------------------------------------------------------------
def transfer_matrix(model: str, q: int, L: int) -> list[int]:
    """Exact DOS via Z(v) = Tr T(v)^L, v^broken-bonds, mod primes + CRT."""
    qq = 2 if model == "ising" else q
    R = qq ** L
    if R > 1024:
        raise ValueError("row space too large")
    N = L * L
    rows = np.array([[(s // qq ** x) % qq for x in range(L)] for s in range(R)], dtype=np.int64)
    horiz = (rows != np.roll(rows, 1, axis=1)).sum(axis=1)             # broken bonds in a row
    vert = (rows[:, None, :] != rows[None, :, :]).sum(axis=2)          # broken between rows
    expo = vert + horiz[None, :]                                        # T[s, s'] exponent
    deg = 2 * N
    bits = N * math.log2(qq) + 2
    primes = _primes(int(bits // 19) + 2, 1 << 20)
    res = []
    for p in primes:
        xs = list(range(1, deg + 2))
        ys = []
        for v in xs:
            powtab = np.array([pow(v, e, p) for e in range(deg + 1)], dtype=np.float64)
            T = powtab[expo]
            acc = None
            base = T
            e = L
            while e:
                if e & 1:
                    acc = base.copy() if acc is None else np.mod(acc @ base, p)
                e >>= 1
                if e:
                    base = np.mod(base @ base, p)
            ys.append(int(np.diag(acc).sum()) % p)
        res.append(_interpolate_mod(xs, ys, p))
    coeffs = _crt(res, primes)                                           # by broken bonds
    out = [0] * n_bins(model, L)
    for broken, c in enumerate(coeffs):
        if c:
            if model == "ising" and broken % 2:
                raise AssertionError("odd broken-bond count on the torus")
            out[_bin_of_broken(model, broken)] += c
    return out


# --------------------------------------------------------------------------------------
# Kaufman's torus formula, exact modulo primes
# --------------------------------------------------------------------------------------
def _ntt(a: np.ndarray, root: int, p: int) -> np.ndarray:
    """In-order radix-2 transform A_j = sum_i a_i root^(i j) mod p (len power of 2)."""
    n = len(a)
    a = a.copy() % p
    j = 0
    for i in range(1, n):                       # bit reversal
        bit = n >> 1
        while j & bit:
            j ^= bit
            bit >>= 1
        j |= bit
        if i < j:
            a[i], a[j] = a[j], a[i]
    length = 2
    while length <= n:
        w = pow(root, n // length, p)
        half = length // 2
        tw = np.array([pow(w, i, p) for i in range(half)], dtype=np.int64)
        a = a.reshape(-1, length)
        u = a[:, :half].copy()
        v = a[:, half:] * tw % p
        a[:, :half] = (u + v) % p
        a[:, half:] = (u - v) % p
        a = a.reshape(-1)
        length *= 2
    return a


def _primitive_root_of_order(order: int, p: int) -> int:
    """An element of exact multiplicative order `order` (which divides p-1)."""
    fac = []
    m, d = order, 2
    while d * d <= m:
        if m % d == 0:
            fac.append(d)
            while m % d == 0:
                m //= d
        d += 1
    if m > 1:
        fac.append(m)
    for g in range(2, p):
        x = pow(g, (p - 1) // order, p)
        if all(pow(x, order // f, p) != 1 for f in fac):
            return x
    raise ValueError("no root")


def _chebyshev_T(n: int, c: np.ndarray, p: int) -> np.ndarray:
    """T_n(c) mod p elementwise, via the doubling pair (T_k, T_{k+1})."""
    a = np.ones_like(c)            # T_0
    b = c % p                      # T_1
    for bit in bin(n)[2:]:
        if bit == "1":             # (T_k, T_{k+1}) -> (T_{2k+1}, T_{2k+2})
            a, b = (2 * a % p * b - c) % p, (2 * b % p * b - 1) % p
        else:                      # (T_k, T_{k+1}) -> (T_{2k}, T_{2k+1})
            a, b = (2 * a % p * a - 1) % p, (2 * a % p * b - c) % p
    return a


def _kaufman_mod(L: int, p: int, n: int):
    """g_b c^b mod p, b = 0..n-1, for the L x L Ising torus (n >= N+1)."""
    N = L * L
    zeta = _primitive_root_of_order(2 * n, p)            # order 2n
    zL = _primitive_root_of_order(2 * L, p)              # order 2L
    t = 3
    while pow(t, 2 * n, p) == 1:                         # t outside <zeta>: avoids y = +-1
        t += 1
    inv2 = pow(2, -1, p)
    zinv = pow(zeta, -1, p)
    # evaluation points y_i = t * zeta^{-i}; u_i = y_i^{-2} = t^{-2} omega^i, omega = zeta^2
    y = np.empty(n, dtype=np.int64)
    cur = t % p
    for i in range(n):
        y[i] = cur
        cur = cur * zinv % p

    def inv(v):
        return np.array([pow(int(e), -1, p) for e in v], dtype=np.int64)

    y2m1 = (y * y - 1) % p
    yinv = inv(y)
    # A = cosh2K coth2K = (y^2+1)^2 / (2 y (y^2-1))
    A = (y * y + 1) % p
    A = A * A % p * inv(2 * y % p * y2m1 % p) % p
    two_T = {}
    for l in range(1, L):
        cosl = (pow(zL, l, p) + pow(zL, 2 * L - l, p)) * inv2 % p
        c = (A - cosl) % p
        two_T[l] = 2 * _chebyshev_T(L, c, p) % p
    Z1 = np.ones(n, dtype=np.int64)
    Z2 = np.ones(n, dtype=np.int64)
    Z3 = np.ones(n, dtype=np.int64)
    Z4 = np.ones(n, dtype=np.int64)
    for l in range(1, L):
        cp = (two_T[l] + 2) % p          # (2 cosh(L gamma_l / 2))^2
        sp = (two_T[l] - 2) % p          # (2 sinh(L gamma_l / 2))^2
        if l % 2:
            Z1 = Z1 * cp % p
            Z2 = Z2 * sp % p
        else:
            Z3 = Z3 * cp % p
            Z4 = Z4 * sp % p
    # unpaired gamma_0 (e^{gamma_0} = y (y-1)/(y+1)) and gamma_L (e^{gamma_L} = y (y+1)/(y-1))
    g0 = y * ((y - 1) % p) % p * inv((y + 1) % p) % p
    gL = y * ((y + 1) % p) % p * inv((y - 1) % p) % p
    h = L // 2
    g0h = np.array([pow(int(v), h, p) for v in g0], dtype=np.int64)
    gLh = np.array([pow(int(v), h, p) for v in gL], dtype=np.int64)
    g0hi, gLhi = inv(g0h), inv(gLh)
    Z3 = Z3 * ((g0h + g0hi) % p) % p * ((gLh + gLhi) % p) % p
    Z4 = Z4 * ((g0h - g0hi) % p) % p * ((gLh - gLhi) % p) % p
    S = (Z1 + Z2 + Z3 + Z4) % p
    # Z = 1/2 (2 sinh 2K)^{N/2} S with 2 sinh 2K = (y^2-1)/y; P(u) = Z y^{-N}
    pre = y2m1 * yinv % p
    pre = np.array([pow(int(v), N // 2, p) for v in pre], dtype=np.int64)
    yN = np.array([pow(int(v), N, p) for v in yinv], dtype=np.int64)
    P = S * pre % p * inv2 % p * yN % p
    # inverse transform over omega = zeta^2: coefficient b holds g_b (t^{-2})^b
    omega = zeta * zeta % p
    coef = _ntt(P, pow(omega, -1, p), p) * pow(n, -1, p) % p
    cinv = t * t % p                                 # undo (t^{-2})^b
    scale = np.empty(n, dtype=np.int64)
    cur = 1
    for b in range(n):
        scale[b] = cur
        cur = cur * cinv % p
    return coef * scale % p


def _kaufman_residues(args):
    L, p, n, N = args
    return [int(v) for v in _kaufman_mod(L, p, n)[: N + 1]]


def kaufman_ising(L: int, processes: int = 1) -> list[int]:
    """Exact integer DOS of the L x L periodic Ising model (L even), by bin.
    processes > 1 evaluates the primes in a process pool (same result)."""
    if L % 2 or L < 2:
        raise ValueError("even L required")
    N = L * L
    n = 1
    while n < N + 1:
        n *= 2
    modulus = (2 * n) * (2 * L) // math.gcd(2 * n, 2 * L)
    count = (N + 8) // 29 + 2
    primes = _primes(count, 1 << 30, modulus)
    jobs = [(L, p, n, N) for p in primes]
    if processes > 1:
        import multiprocessing as mp
        with mp.Pool(processes) as pool:
            res = pool.map(_kaufman_residues, jobs)
    else:
        res = [_kaufman_residues(j) for j in jobs]
    g = _crt(res, primes)
    if sum(g) != 2 ** N:
        raise AssertionError("sum of g differs from 2^N")
    return g


def ln_g(counts: list[int]) -> np.ndarray:
    """Natural log of exact counts; -inf where the level does not occur."""
    return np.array([math.log(c) if c > 0 else -math.inf for c in counts], dtype=np.float64)


@lru_cache(maxsize=None)
def exact_ln_g(model: str, q: int, L: int) -> tuple:
    """Exact ln g by the cheapest applicable route (cached)."""
    if model == "ising":
        return tuple(ln_g(kaufman_ising(L)))
    return tuple(ln_g(transfer_matrix(model, q, L)))
