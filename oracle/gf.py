"""CPU oracle for the Q-adic transform path (TEST INFRASTRUCTURE ONLY).

This module is the checker, not the product.  Only the test suite, the
smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py``
may import it.  It shares no code with the HIP library: no tables, no
helpers, no constants.  Everything is plain Python integers (arbitrary
precision) plus, for the larger GEMM cases, numpy int64 matrix products
used as a library step.

Source: J.-G. Dumas, "Q-adic Transform Revisited" (arXiv 0710.0510).

Conventions
-----------
* A polynomial over GF(p) is a list of ints ``c`` with ``c[i]`` the
  coefficient of X^i, every value in [0, p).
* ``k`` is the number of coefficients of an operand (degree < k), so a
  product has 2k-1 coefficients (reading of Thm. 1, where Alg. 1 states
  "degree less than k").
* A field GF(p^k) is given by p and the k low coefficients ``P_low`` of a
  monic defining polynomial P = X^k + sum_i P_low[i] X^i (Section 7).

Every function names the passage it follows.  Where the method reaches a
result that has a plain definition (a polynomial or matrix product over
GF(p) or GF(p^k)), the oracle is that definition; the paper's own steps
(Alg. 1, Alg. 2, Alg. 3, Alg. 4) are written out separately so that tests
can check the paper's printed intermediates and Thm. 2 / Thm. 3's
invariants.
"""

from __future__ import annotations

import itertools
from typing import Iterable, List, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# O1: polynomial product over GF(p) (Section 2, eq. (1); Alg. 1 ENSURE)
# ---------------------------------------------------------------------------


def poly_mul_z(a: Sequence[int], b: Sequence[int]) -> List[int]:
    """Product in Z[X]: coefficient j is sum_i a_i b_{j-i} (eq. (1))."""
    if not a or not b:
        return []
    out = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            out[i + j] += ai * bj
    return out


def poly_mul_mod_p(a: Sequence[int], b: Sequence[int], p: int) -> List[int]:
    """R = a*b in GF(p)[X], all len(a)+len(b)-1 coefficients kept (Alg. 1)."""
    return [c % p for c in poly_mul_z(a, b)]


# ---------------------------------------------------------------------------
# O3: arithmetic in GF(p^k) = GF(p)[X]/(P) (Section 7)
# ---------------------------------------------------------------------------


def monic(P_low: Sequence[int]) -> List[int]:
    """Full coefficient list of the monic P = X^k + sum P_low[i] X^i."""
    return list(P_low) + [1]


def poly_rem(c: Sequence[int], P_low: Sequence[int], p: int) -> List[int]:
    """Remainder of c modulo the monic P over GF(p), as k coefficients.

    Plain long division from the top coefficient down: X^k is replaced by
    -sum P_low[i] X^i.
    """
    k = len(P_low)
    r = [x % p for x in c]
    for top in range(len(r) - 1, k - 1, -1):
        lead = r[top]
        if lead:
            r[top] = 0
            for i in range(k):
                r[top - k + i] = (r[top - k + i] - lead * P_low[i]) % p
    r = r[:k] + [0] * max(0, k - len(r))
    return r


def field_add(a: Sequence[int], b: Sequence[int], p: int) -> List[int]:
    return [(x + y) % p for x, y in zip(a, b)]


def field_mul(a: Sequence[int], b: Sequence[int], p: int,
              P_low: Sequence[int]) -> List[int]:
    """Schoolbook product of two elements, then reduction modulo P."""
    return poly_rem(poly_mul_z(a, b), P_low, p)


def field_pow(a: Sequence[int], e: int, p: int, P_low: Sequence[int]) -> List[int]:
    k = len(P_low)
    result = [1] + [0] * (k - 1)
    base = list(a)
    while e:
        if e & 1:
            result = field_mul(result, base, p, P_low)
        base = field_mul(base, base, p, P_low)
        e >>= 1
    return result


def all_elements(p: int, k: int) -> Iterable[List[int]]:
    """Every element of GF(p^k) in coefficient form, base-p order."""
    for t in itertools.product(range(p), repeat=k):
        yield list(reversed(t))


def is_irreducible(P_low: Sequence[int], p: int) -> bool:
    """P monic of degree k is irreducible iff no monic divisor of degree
    1..k//2 exists (plain trial division over GF(p))."""
    k = len(P_low)
    P = monic(P_low)
    for d in range(1, k // 2 + 1):
        for low in itertools.product(range(p), repeat=d):
            D = list(low) + [1]
            if _poly_rem_general(P, D, p) == [0] * d:
                return False
    return True


def _poly_rem_general(c: Sequence[int], D: Sequence[int], p: int) -> List[int]:
    """Remainder of c by a monic D (used only for irreducibility)."""
    d = len(D) - 1
    r = [x % p for x in c]
    for top in range(len(r) - 1, d - 1, -1):
        lead = r[top]
        if lead:
            for i in range(d + 1):
                r[top - d + i] = (r[top - d + i] - lead * D[i]) % p
    return r[:d]


# ---------------------------------------------------------------------------
# O4: matrix product over GF(p^k) (Alg. 4 ENSURE, applied entrywise)
# ---------------------------------------------------------------------------


def gemm_gfpk_small(A, B, p: int, P_low: Sequence[int]):
    """C[i][j] = sum_l A[i][l] * B[l][j] in GF(p^k); one field product and
    one field addition at a time.  A is M x K x k, B is K x N x k (nested
    lists or arrays of ints in [0, p)); returns an M x N x k list."""
    k = len(P_low)
    M, K = len(A), len(A[0]) if len(A) else 0
    N = len(B[0]) if K else 0
    C = []
    for i in range(M):
        row = []
        for j in range(N):
            acc = [0] * k
            for l in range(K):
                acc = field_add(acc, field_mul(list(A[i][l]), list(B[l][j]), p, P_low), p)
            row.append(acc)
        C.append(row)
    return C


def gemm_gfpk_planes(A: np.ndarray, B: np.ndarray, p: int,
                     P_low: Sequence[int]) -> np.ndarray:
    """Same product, accumulated in Z[X] and reduced once.

    GF(p^k) is the image of Z[X] under reduction mod (p, P), a ring
    homomorphism, so summing the Z[X] products first and reducing at the
    end gives the same field element.  Plane t of the Z[X] sum is
    sum_{i+j=t} A_i @ B_j where A_i is the M x K integer matrix of the i-th
    coefficients; numpy's int64 matmul is the library step (exact: every
    entry is below K*k*(p-1)^2 < 2^63).  Then each of the 2k-1 planes is
    reduced mod p and X^t (t >= k) is replaced by its remainder mod P.
    """
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    k = len(P_low)
    M, K = A.shape[0], A.shape[1]
    N = B.shape[1]
    planes = [np.zeros((M, N), dtype=np.int64) for _ in range(2 * k - 1)]
    for i in range(k):
        Ai = np.ascontiguousarray(A[:, :, i])
        for j in range(k):
            planes[i + j] += Ai @ np.ascontiguousarray(B[:, :, j])
    planes = [pl % p for pl in planes]
    out = np.zeros((M, N, k), dtype=np.int64)
    for t in range(2 * k - 1):
        xt = poly_rem([0] * t + [1], P_low, p)  # X^t mod P
        for s in range(k):
            if xt[s]:
                out[:, :, s] += xt[s] * planes[t]
    return (out % p).astype(np.uint8)


def freivalds(A: np.ndarray, B: np.ndarray, C: np.ndarray, p: int, P_low: Sequence[int],
              rng: np.random.Generator, vectors: int = 20) -> bool:
    """Freivalds' test of Alg. 4's ENSURE (C = AB over GF(p^k)) on every
    entry at once: C x = A (B x) for x uniform in GF(p^k)^(N x vectors), the
    three products by gemm_gfpk_planes.  A true product always passes.  If
    C != AB, a nonzero row d of C - AB gives d x uniform over the field for
    each column of x, so a wrong C survives one column with probability at
    most 1/p^k."""
    x = rng.integers(0, p, size=(B.shape[1], vectors, len(P_low)), dtype=np.uint8)
    left = gemm_gfpk_planes(C, x, p, P_low)
    right = gemm_gfpk_planes(A, gemm_gfpk_planes(B, x, p, P_low), p, P_low)
    return bool(np.array_equal(left, right))


def gemm_entry(A_row: np.ndarray, B_col: np.ndarray, p: int,
               P_low: Sequence[int]) -> List[int]:
    """One entry C[i][j] = sum_l A[i][l] B[l][j] over GF(p^k), big ints.

    ``A_row`` is K x k, ``B_col`` is K x k.  Accumulate in Z[X] (exact) and
    reduce once (same homomorphism argument as ``gemm_gfpk_planes``)."""
    k = len(P_low)
    acc = [0] * (2 * k - 1)
    for a, b in zip(A_row.tolist(), B_col.tolist()):
        for i in range(k):
            ai = a[i]
            if ai:
                for j in range(k):
                    acc[i + j] += ai * b[j]
    return poly_rem(acc, P_low, p)


def polymul_batch(a: np.ndarray, b: np.ndarray, p: int) -> np.ndarray:
    """Row-wise O1 on n x k arrays: out[r] = a[r] * b[r] in GF(p)[X]."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    n, k = a.shape
    out = np.zeros((n, 2 * k - 1), dtype=np.int64)
    for i in range(k):
        for j in range(k):
            out[:, i + j] += a[:, i] * b[:, j]
    return (out % p).astype(np.uint8)


# ---------------------------------------------------------------------------
# DQT: evaluation at q (Section 2, eq. (1); Alg. 1 first step)
# ---------------------------------------------------------------------------


def dqt(coeffs: Sequence[int], q: int) -> int:
    """Evaluate sum c_i X^i at X = q with Horner's rule (Alg. 1, step 1)."""
    v = 0
    for c in reversed(list(coeffs)):
        v = v * q + c
    return v


def qadic_digits(r: int, q: int, n: int) -> List[int]:
    """The n base-q digits of r >= 0, least significant first (radix
    conversion of Alg. 1, step 3)."""
    out = []
    for _ in range(n):
        r, d = divmod(r, q)
        out.append(d)
    return out


def dqt_inverse(r: int, q: int, n: int, p: int) -> List[int]:
    """O2 as a definition: base-q digits of r, each taken mod p (Alg. 1,
    steps 3-4; also Alg. 2's ENSURE, mu_i = digit_i mod p)."""
    return [d % p for d in qadic_digits(r, q, n)]


def polymul_dqt(a: Sequence[int], b: Sequence[int], p: int, q: int) -> List[int]:
    """Alg. 1 step by step, in big integers: pack both operands at q,
    multiply once, convert back in radix q, reduce each digit mod p."""
    k = max(len(a), len(b))
    r = dqt(a, q) * dqt(b, q)
    return dqt_inverse(r, q, 2 * k - 1, p)


# ---------------------------------------------------------------------------
# eq. (2): the exactness conditions of Thm. 1
# ---------------------------------------------------------------------------


def eq2_holds(p: int, k: int, q: int, n_q: int, m: int = 53) -> bool:
    """q > n_q k (p-1)^2 and (2k-1) log2(q) < m, checked in integers:
    the second inequality is q^(2k-1) < 2^m."""
    return q > n_q * k * (p - 1) ** 2 and q ** (2 * k - 1) < 2 ** m


def max_pow2_q(p: int, k: int, m: int = 53) -> Tuple[int, int]:
    """Largest q = 2^b with q^(2k-1) < 2^m, and the largest n_q it allows
    under eq. (2)."""
    b = 1
    while (2 ** (b + 1)) ** (2 * k - 1) < 2 ** m:
        b += 1
    q = 2 ** b
    nq = (q - 1) // (k * (p - 1) ** 2) if p > 1 else 0
    return q, nq


# ---------------------------------------------------------------------------
# Alg. 2 (REDQ), as printed, in big integers
# ---------------------------------------------------------------------------


def redq_steps(r: int, p: int, q: int, d: int):
    """REDQ (Alg. 2) in big integers for r = sum_{i<=d} mu~_i q^i >= 0,
    built on Thm. 2 rather than on the listing's statements.

    Thm. 2: with rop = floor(r / p), every u_i = floor(r / q^i) -
    p floor(rop / q^i) lies in [0, p) and is congruent mod p to
    sum_{j>=i} mu~_j q^(j-i).  Those congruences form the triangular
    Toeplitz system of Section 5.1, so the digits mod p are Q_d u mod p
    (q_matrix below), and rho packs them back at q (the DQT).

    Returns (rop, u, mu, rho) with mu_i = mu~_i mod p.
    """
    rop = r // p
    u = [r // q ** i - p * (rop // q ** i) for i in range(d + 1)]
    mu = mat_vec_mod(q_matrix(d, q, p), u, p)
    return rop, u, mu, dqt(mu, q)


def q_matrix(d: int, q: int, p: int) -> List[List[int]]:
    """Q_d of Section 5.1 reduced mod p: 1 on the diagonal and -q on the
    superdiagonal, so that mu = Q_d u (mod p)."""
    Q = [[0] * (d + 1) for _ in range(d + 1)]
    for i in range(d + 1):
        Q[i][i] = 1
        if i < d:
            Q[i][i + 1] = (-q) % p
    return Q


def mat_vec_mod(Q: Sequence[Sequence[int]], v: Sequence[int], p: int) -> List[int]:
    return [sum(a * b for a, b in zip(row, v)) % p for row in Q]


def toeplitz_powers(d: int, q: int) -> List[List[int]]:
    """Upper-triangular Toeplitz matrix of powers of q (Section 5.1), whose
    inverse is Q_d."""
    return [[q ** (j - i) if j >= i else 0 for j in range(d + 1)]
            for i in range(d + 1)]


def q6_by_three_q2(u: Sequence[int], q: int, p: int) -> List[int]:
    """Alg. 3: Q_6 applied to u_0..u_6 with three overlapping Q_2 products,
    keeping the first two entries of the first two."""
    Q2 = q_matrix(2, q, p)
    a = mat_vec_mod(Q2, u[0:3], p)
    b = mat_vec_mod(Q2, u[2:5], p)
    c = mat_vec_mod(Q2, u[4:7], p)
    return [a[0], a[1], b[0], b[1], c[0], c[1], c[2]]


def q_by_windows(u: Sequence[int], q: int, p: int, w: int) -> List[int]:
    """Section 5.2 generalised: Q_d through overlapping Q_{w-1} windows of
    w residues each, advancing by w-1; ceil(d/(w-1)) windows."""
    d = len(u) - 1
    Qw = q_matrix(w - 1, q, p)
    mu = [0] * (d + 1)
    start = 0
    while True:
        win = list(u[start:start + w])
        win += [0] * (w - len(win))
        part = mat_vec_mod(Qw, win, p)
        last = start + w - 1 >= d
        keep = w if last else w - 1
        for j in range(keep):
            if start + j <= d:
                mu[start + j] = part[j]
        if last:
            return mu
        start += w - 1


# ---------------------------------------------------------------------------
# Thm. 3: the L and H tables of Alg. 4, and Alg. 4 itself
# ---------------------------------------------------------------------------


def table_L(uw: Sequence[int], q: int, p: int) -> List[int]:
    """L indexed by (u_0..u_{k-1}): sum_{i<=k-2} ((u_i - q u_{i+1}) mod p) X^i,
    as k coefficients (its degree is below k-1, so it is already reduced)."""
    k = len(uw)
    out = [0] * k
    for i in range(k - 1):
        out[i] = (uw[i] - q * uw[i + 1]) % p
    return out


def table_H(uw: Sequence[int], q: int, p: int, P_low: Sequence[int]) -> List[int]:
    """H indexed by (u_{k-1}..u_{2k-2}):
    u_{2k-2} X^{2k-2} + sum_{i=k-1}^{2k-3} ((u_i - q u_{i+1}) mod p) X^i,
    reduced modulo P."""
    k = len(uw)
    poly = [0] * (2 * k - 1)
    poly[2 * k - 2] = uw[k - 1] % p
    for t in range(k - 1):       # i = k-1+t runs over k-1 .. 2k-3
        poly[k - 1 + t] = (uw[t] - q * uw[t + 1]) % p
    return poly_rem(poly, P_low, p)


def fgdp(v1, v2, p: int, P_low: Sequence[int], q: int) -> List[int]:
    """Alg. 4 for one dot product v1^T v2 over GF(p^k), in big integers:
    the dot product of the packed operands is one exact integer r (Thm. 1,
    eq. (2)); its 2k-1 residues u of Thm. 2 index Thm. 3's two tables, L by
    (u_0..u_{k-1}) and H by (u_{k-1}..u_{2k-2}), whose sum mod p is the
    reduced field element."""
    k = len(P_low)
    r = sum(dqt(a, q) * dqt(b, q) for a, b in zip(v1, v2))
    u = redq_steps(r, p, q, 2 * k - 2)[1]
    return field_add(table_L(u[:k], q, p), table_H(u[k - 1:], q, p, P_low), p)


def binary_index(uw: Sequence[int], p: int) -> int:
    """Section 5.3 binary indexing: sum u_i 2^(c*i) with c = ceil(log2 p),
    u_0 least significant."""
    c = max(1, (p - 1).bit_length())
    return sum(int(x) << (c * i) for i, x in enumerate(uw))


# ---------------------------------------------------------------------------
# d-FQT: long polynomials in chunks of d+1 coefficients (Section 6)
# ---------------------------------------------------------------------------


def polymul_long(a: Sequence[int], b: Sequence[int], p: int) -> List[int]:
    """Definition of the product of two polynomials over GF(p) of any length:
    the convolution of the coefficient lists reduced mod p (numpy convolve
    on int64 as the library step; exact while len * (p-1)^2 < 2^63)."""
    if len(a) == 0 or len(b) == 0:
        return []
    c = np.convolve(np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64))
    return [int(x) % p for x in c]


def dfqt_degree(n_coeffs: int, d: int) -> int:
    """Section 6: a polynomial with n_coeffs = N + 1 coefficients becomes one
    of degree D_q = ceil((N+1)/(d+1)) - 1 in Y = X^(d+1)."""
    return -(-n_coeffs // (d + 1)) - 1


def dfqt_chunks(a: Sequence[int], d: int) -> List[List[int]]:
    """P = sum_i P_i Y^i with Y = X^(d+1): chunk i holds coefficients
    i(d+1) .. i(d+1)+d of P (the last chunk zero-padded)."""
    n = dfqt_degree(len(a), d) + 1
    padded = list(a) + [0] * (n * (d + 1) - len(a))
    return [padded[i * (d + 1):(i + 1) * (d + 1)] for i in range(n)]


def dfqt_polymul(a: Sequence[int], b: Sequence[int], p: int, d: int, q: int,
                 n_q: int) -> List[int]:
    """The d-FQT product of Section 6, step by step, in big integers.

    1. Split both operands into chunks of d+1 coefficients (degree <= d
       polynomials P_i, Q_j in X; the operands become polynomials in
       Y = X^(d+1)).
    2. Pack every chunk at q (DQT, eq. (1)).
    3. For every t, S_t = sum_i P_i(q) Q_{t-i}(q) is accumulated in blocks of
       at most n_q products; each block's integer sum is reduced by REDQ_{2d+1}
       (Alg. 2 on its 2d+1 q-adic digits, exact while eq. (2) holds with
       k = d+1, i.e. q > n_q (d+1)(p-1)^2 and q^(2d+1) below the mantissa
       bound) and the blocks' reduced digits are added mod p.
    4. Digit j of S_t is the coefficient of X^(t(d+1)+j); digits of
       consecutive t overlap (2d+1 > d+1) and are added mod p.
    """
    if len(a) == 0 or len(b) == 0:
        return []
    P = [dqt(ch, q) for ch in dfqt_chunks(a, d)]
    Q = [dqt(ch, q) for ch in dfqt_chunks(b, d)]
    nd = 2 * d + 1
    out = [0] * (len(a) + len(b) - 1)
    for t in range(len(P) + len(Q) - 1):
        terms = [P[i] * Q[t - i] for i in range(len(P)) if 0 <= t - i < len(Q)]
        mu_t = [0] * nd
        for s in range(0, len(terms), n_q):
            r = sum(terms[s:s + n_q])
            _, _, mu, _ = redq_steps(r, p, q, nd - 1)
            mu_t = [(x + y) % p for x, y in zip(mu_t, mu)]
        for j, m in enumerate(mu_t):
            n = t * (d + 1) + j
            if n < len(out):
                out[n] = (out[n] + m) % p
    return out


# ---------------------------------------------------------------------------
# Discrete-logarithm representation (Section 7, Alg. 4)
# ---------------------------------------------------------------------------
#
# Alg. 4 takes field elements as exponents of a generator g.  The paper leaves
# the generator and the code of zero open; the readings used here: g is the
# first element of multiplicative order p^k - 1 in base-p order (element
# index sum_i c_i p^i), and zero has the code m = p^k - 1, one past the
# largest exponent m - 1.


def elem_index(c: Sequence[int], p: int) -> int:
    """Base-p index sum_i c_i p^i of an element in coefficient form."""
    return sum(int(x) * p ** i for i, x in enumerate(c))


def elem_from_index(idx: int, p: int, k: int) -> List[int]:
    return [(idx // p ** i) % p for i in range(k)]


def mult_order(a: Sequence[int], p: int, P_low: Sequence[int]) -> int:
    """Smallest e >= 1 with a^e = 1, by repeated multiplication (a != 0)."""
    k = len(P_low)
    one = [1] + [0] * (k - 1)
    x, e = list(a), 1
    while x != one:
        x = field_mul(x, a, p, P_low)
        e += 1
        if e > p ** k:
            raise ValueError("element of infinite order: P is not irreducible")
    return e


def log_generator(p: int, P_low: Sequence[int]) -> int:
    """Index of the first element of order p^k - 1 in base-p order."""
    k = len(P_low)
    m = p ** k - 1
    for idx in range(1, p ** k):
        if mult_order(elem_from_index(idx, p, k), p, P_low) == m:
            return idx
    raise ValueError("no generator: P is not irreducible")


def log_tables(p: int, P_low: Sequence[int]):
    """(g, expo, logs): expo[e] is the index of g^e for e = 0..m-1, logs maps
    an element index to its exponent, and logs[0] = m codes zero."""
    k = len(P_low)
    m = p ** k - 1
    g = log_generator(p, P_low)
    ge = elem_from_index(g, p, k)
    expo, x = [], [1] + [0] * (k - 1)
    for _ in range(m):
        expo.append(elem_index(x, p))
        x = field_mul(x, ge, p, P_low)
    logs = {idx: e for e, idx in enumerate(expo)}
    logs[0] = m
    return g, expo, logs


def zech_table(p: int, P_low: Sequence[int]) -> List[int]:
    """Z[n] = log(1 + g^n) for n = 0..m-1 (the code m where 1 + g^n = 0):
    the field addition of the log representation rests on
    g^a + g^b = g^a (1 + g^(b-a))."""
    k = len(P_low)
    _, expo, logs = log_tables(p, P_low)
    one = [1] + [0] * (k - 1)
    return [logs[elem_index(field_add(one, elem_from_index(expo[n], p, k), p), p)]
            for n in range(len(expo))]


def to_log(c: Sequence[int], p: int, P_low: Sequence[int], tabs=None) -> int:
    _, _, logs = tabs or log_tables(p, P_low)
    return logs[elem_index(c, p)]


def from_log(code: int, p: int, P_low: Sequence[int], tabs=None) -> List[int]:
    k = len(P_low)
    _, expo, _ = tabs or log_tables(p, P_low)
    m = len(expo)
    if code == m:
        return [0] * k
    if not 0 <= code < m:
        raise ValueError(f"code {code} outside 0..{m}")
    return elem_from_index(expo[code], p, k)


def log_add(a: int, b: int, Z: Sequence[int]) -> int:
    """Field addition on codes: zero is the identity, otherwise
    a + Z[(b - a) mod m] mod m, and zero where 1 + g^(b-a) vanishes."""
    m = len(Z)
    if a == m:
        return b
    if b == m:
        return a
    z = Z[(b - a) % m]
    return m if z == m else (a + z) % m


def fgdp_log(v1: Sequence[int], v2: Sequence[int], p: int, P_low: Sequence[int], q: int,
             tabs=None, Z=None) -> int:
    """Alg. 4 on codes, step by step in big integers: every code becomes the
    evaluation at q of its element (the tabulated conversion), one integer
    dot product, rop and the residues u_0..u_{2k-2}, then L and H as codes
    (the two tables of Thm. 3 followed by the conversion to logarithms), and
    R = H + L by the field addition of codes."""
    k = len(P_low)
    tabs = tabs or log_tables(p, P_low)
    Z = Z if Z is not None else zech_table(p, P_low)
    pk = lambda code: dqt(from_log(code, p, P_low, tabs), q)
    r = sum(pk(a) * pk(b) for a, b in zip(v1, v2))
    rop = r // p
    u = [r // q ** i - p * (rop // q ** i) for i in range(2 * k - 1)]
    L = to_log(table_L(u[0:k], q, p), p, P_low, tabs)
    H = to_log(table_H(u[k - 1:2 * k - 1], q, p, P_low), p, P_low, tabs)
    return log_add(H, L, Z)


def gemm_log_alg4(A, B, p: int, P_low: Sequence[int], q: int, n_q: int):
    """C = A B on codes with Alg. 4 per entry, K cut into blocks of at most
    n_q products (each a dot product under eq. (2)), the block results added
    with the field addition of codes.  Small cases only (pure Python)."""
    tabs = log_tables(p, P_low)
    Z = zech_table(p, P_low)
    m = len(Z)
    M, K = len(A), len(A[0]) if len(A) else 0
    N = len(B[0]) if len(B) else 0
    C = [[m] * N for _ in range(M)]
    for i in range(M):
        for j in range(N):
            acc = m
            for s in range(0, K, n_q):
                part = fgdp_log(A[i][s:s + n_q], [B[l][j] for l in range(s, min(K, s + n_q))],
                                p, P_low, q, tabs, Z)
                acc = log_add(acc, part, Z)
            C[i][j] = acc
    return C


def gemm_log(A: np.ndarray, B: np.ndarray, p: int, P_low: Sequence[int]) -> np.ndarray:
    """Definition: the product over GF(p^k) of the elements the codes stand
    for, returned as codes (M x K and K x N arrays of codes; zero = p^k - 1)."""
    k = len(P_low)
    _, expo, logs = log_tables(p, P_low)
    m = len(expo)
    anti = np.array([elem_from_index(i, p, k) for i in expo] + [[0] * k], dtype=np.uint8)
    Cc = gemm_gfpk_planes(anti[np.asarray(A, dtype=np.int64)],
                          anti[np.asarray(B, dtype=np.int64)], p, P_low)
    lut = np.zeros(p ** k, dtype=np.uint16)
    for idx, e in logs.items():
        lut[idx] = e
    weights = np.array([p ** i for i in range(k)], dtype=np.int64)
    return lut[(Cc.astype(np.int64) * weights).sum(axis=-1)]


# ---------------------------------------------------------------------------
# Winograd's variant of Strassen's product over GF(p^k) (the setting of the
# paper's Fig. 3: finite-field Winograd matrix multiplication with the FQT as
# the base case)
# ---------------------------------------------------------------------------
#
# On a 2 x 2 block partition, seven block products and fifteen block
# additions (Winograd's schedule):
#   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2,
#   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21,
#   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4,
#   P5 = S1 T1, P6 = S2 T2, P7 = S3 T3,
#   C11 = P1 + P2, U2 = P1 + P6, U3 = U2 + P7, U4 = U2 + P5,
#   C12 = U4 + P3, C21 = U3 - P4, C22 = U3 + P5.
# Additions of field elements are coefficient-wise mod p.  Odd dimensions are
# peeled: the even part goes through the recursion, the last row, column or
# rank-one term through the definition.


def _fadd(X: np.ndarray, Y: np.ndarray, p: int) -> np.ndarray:
    return ((X.astype(np.int64) + Y) % p).astype(np.uint8)


def _fsub(X: np.ndarray, Y: np.ndarray, p: int) -> np.ndarray:
    return ((X.astype(np.int64) - Y) % p).astype(np.uint8)


def gemm_winograd(A: np.ndarray, B: np.ndarray, p: int, P_low: Sequence[int],
                  levels: int) -> np.ndarray:
    """C = A B over GF(p^k) (M x K x k and K x N x k coefficient arrays) with
    `levels` levels of Winograd's recursion over gemm_gfpk_planes."""
    M, K, k = A.shape
    N = B.shape[1]
    if levels <= 0 or M < 2 or N < 2 or K < 2:
        return gemm_gfpk_planes(A, B, p, P_low)
    m, n, kk = M // 2 * 2, N // 2 * 2, K // 2 * 2
    C = np.zeros((M, N, k), dtype=np.uint8)
    h, w, d = m // 2, n // 2, kk // 2
    A11, A12, A21, A22 = A[:h, :d], A[:h, d:kk], A[h:m, :d], A[h:m, d:kk]
    B11, B12, B21, B22 = B[:d, :w], B[:d, w:n], B[d:kk, :w], B[d:kk, w:n]
    S1 = _fadd(A21, A22, p)
    S2 = _fsub(S1, A11, p)
    S3 = _fsub(A11, A21, p)
    S4 = _fsub(A12, S2, p)
    T1 = _fsub(B12, B11, p)
    T2 = _fsub(B22, T1, p)
    T3 = _fsub(B22, B12, p)
    T4 = _fsub(T2, B21, p)
    rec = lambda X, Y: gemm_winograd(X, Y, p, P_low, levels - 1)
    P1, P2, P3 = rec(A11, B11), rec(A12, B21), rec(S4, B22)
    P4, P5, P6, P7 = rec(A22, T4), rec(S1, T1), rec(S2, T2), rec(S3, T3)
    U2 = _fadd(P1, P6, p)
    U3 = _fadd(U2, P7, p)
    U4 = _fadd(U2, P5, p)
    C[:h, :w] = _fadd(P1, P2, p)
    C[:h, w:n] = _fadd(U4, P3, p)
    C[h:m, :w] = _fsub(U3, P4, p)
    C[h:m, w:n] = _fadd(U3, P5, p)
    if kk < K:   # rank-one term of the last k
        C[:m, :n] = _fadd(C[:m, :n], gemm_gfpk_planes(A[:m, kk:], B[kk:, :n], p, P_low), p)
    if m < M:    # last row
        C[m:, :] = gemm_gfpk_planes(A[m:, :], B, p, P_low)
    if n < N:    # last column
        C[:m, n:] = gemm_gfpk_planes(A[:m, :], B[:, n:], p, P_low)
    return C


# ---------------------------------------------------------------------------
# Centred representation inside the FQT (a reading: Section 6 names the
# centred residues (1-p)/2 .. (p-1)/2 for delayed reduction; here they are
# packed instead of [0, p) coefficients)
# ---------------------------------------------------------------------------
#
# With every coefficient s in [-h, h], h = (p-1)/2, a product digit is at most
# k h^2 in magnitude and a block of n products at most n k h^2; while that
# stays below q/2, adding q/2 to every digit (the constant
# B = sum_{i<2k-1} (q/2) q^i) leaves non-negative digits below q, so the
# sum B + r has no borrows and REDQ applies unchanged.  The residues then
# carry the known shift of B, which L + H maps to one constant element.


def centred(c: Sequence[int], p: int) -> List[int]:
    h = (p - 1) // 2
    return [x - p if x > h else x for x in c]


def centred_nq_max(p: int, k: int, q: int) -> int:
    """Largest n with n k h^2 <= q/2 - 1 (p odd, q even)."""
    h = (p - 1) // 2
    return (q // 2 - 1) // (k * h * h)


def fgdp_centred(v1, v2, p: int, P_low: Sequence[int], q: int) -> List[int]:
    """Alg. 4 for one dot product with centred packing: evaluate the centred
    coefficients at q, add B, REDQ, L + H, then subtract L + H of B's own
    residues."""
    k = len(P_low)
    nd = 2 * k - 1
    B = sum((q // 2) * q ** i for i in range(nd))
    r = B + sum(dqt(centred(a, p), q) * dqt(centred(b, p), q) for a, b in zip(v1, v2))
    assert 0 <= r < q ** nd
    rop = r // p
    u = [r // q ** i - p * (rop // q ** i) for i in range(nd)]
    beta = [(B // q ** i) % p for i in range(nd)]
    R = field_add(table_L(u[0:k], q, p), table_H(u[k - 1:nd], q, p, P_low), p)
    C0 = field_add(table_L(beta[0:k], q, p), table_H(beta[k - 1:nd], q, p, P_low), p)
    return [(x - y) % p for x, y in zip(R, C0)]


def gemm_centred_alg4(A, B, p: int, P_low: Sequence[int], q: int, n_q: int):
    """C = A B with fgdp_centred on K-blocks of at most n_q products, block
    results added in the field.  Small cases only (pure Python)."""
    M, K = len(A), len(A[0]) if len(A) else 0
    N = len(B[0]) if len(B) else 0
    k = len(P_low)
    C = [[[0] * k for _ in range(N)] for _ in range(M)]
    for i in range(M):
        for j in range(N):
            acc = [0] * k
            for s in range(0, K, n_q):
                part = fgdp_centred(A[i][s:s + n_q], [B[l][j] for l in range(s, min(K, s + n_q))],
                                    p, P_low, q)
                acc = field_add(acc, part, p)
            C[i][j] = acc
    return C


def dfqt_polymul_centred(a: Sequence[int], b: Sequence[int], p: int, d: int, q: int,
                         n_q: int) -> List[int]:
    """The d-FQT product with centred chunks (the representation Section 6
    names for delayed reduction): coefficients above (p-1)/2 packed as c - p,
    every block of at most n_q chunk products shifted by B = sum (q/2) q^j
    (2d+1 digits) so its digits stay in [0, q) while n_q (d+1) ((p-1)/2)^2 <=
    q/2 - 1; the block's REDQ_{2d+1} digits then carry q/2 each, which comes
    off mod p."""
    if len(a) == 0 or len(b) == 0:
        return []
    nd = 2 * d + 1
    B = sum((q // 2) * q ** j for j in range(nd))
    P = [dqt(centred(ch, p), q) for ch in dfqt_chunks(a, d)]
    Q = [dqt(centred(ch, p), q) for ch in dfqt_chunks(b, d)]
    out = [0] * (len(a) + len(b) - 1)
    for t in range(len(P) + len(Q) - 1):
        terms = [P[i] * Q[t - i] for i in range(len(P)) if 0 <= t - i < len(Q)]
        mu_t = [0] * nd
        for s in range(0, len(terms), n_q):
            r = B + sum(terms[s:s + n_q])
            assert 0 <= r < q ** nd
            _, _, mu, _ = redq_steps(r, p, q, nd - 1)
            mu_t = [(x + y - q // 2) % p for x, y in zip(mu_t, mu)]
        for j, m in enumerate(mu_t):
            n = t * (d + 1) + j
            if n < len(out):
                out[n] = (out[n] + m) % p
    return out
