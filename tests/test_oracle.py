"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests re-types an oracle formula: each compares the oracle
with a value printed in the paper (tests/golden/), a closed form, a library
routine, an invariant, or brute force on tiny inputs.
"""
import itertools
import random

import numpy as np
import pytest

from oracle import gf
from golden_io import load

CONFIG_FIELDS = [(3, (1, 0)), (7, (1, 0)), (3, (2, 0, 0, 2)), (5, (3, 3, 0))]


# --- worked examples printed in the paper ---------------------------------

def test_example1_dqt():
    g = load("ex1_dqt.txt")
    p, q = g["p"], g["q"]
    assert gf.dqt(g["a"], q) == g["packed_a"]
    assert gf.dqt(g["b"], q) == g["packed_b"]
    assert gf.dqt(g["a"], q) * gf.dqt(g["b"], q) == g["product"]
    assert gf.qadic_digits(g["product"], q, 3) == g["digits"]
    assert gf.dqt_inverse(g["product"], q, 3, p) == g["result"]
    assert gf.polymul_dqt(g["a"], g["b"], p, q) == g["result"]
    assert gf.poly_mul_mod_p(g["a"], g["b"], p) == g["result"]


def test_example2_p_divides_q():
    g = load("ex2_redq_p_divides_q.txt")
    p, q = g["p"], g["q"]
    r = gf.dqt(g["a"], q) * gf.dqt(g["b"], q)
    assert r == g["product"]
    assert r - p * g["quotients"] == g["reduced"]
    rop, u, mu, rho = gf.redq_steps(r, p, q, 4)
    assert mu == g["result"]
    assert rho == g["reduced"]
    assert u == g["result"]                 # p | q: no correction needed
    assert gf.dqt_inverse(r, q, 5, p) == g["result"]
    assert gf.poly_mul_mod_p(g["a"], g["b"], p) == g["result"]
    # the quotient vector holds floor(digit / p) for every digit
    digits = gf.qadic_digits(r, q, 5)
    assert gf.dqt([d // p for d in digits], q) == g["quotients"]


def test_example3_full_redq():
    g = load("ex3_redq_full.txt")
    p, q = g["p"], g["q"]
    r = gf.dqt(g["R"], q)
    assert r == g["packed"]
    rop, u, mu, rho = gf.redq_steps(r, p, q, 3)
    assert rop == g["rop"]
    assert rop * p == g["rop_times_p"]
    assert u == g["u"]
    assert r // q == g["shifted"]
    assert (rop // q) * p == g["shifted_rop_times_p"]
    Q3 = gf.q_matrix(3, q, p)
    assert Q3[0][1] == Q3[1][2] == Q3[2][3] == g["correction"]
    assert gf.mat_vec_mod(Q3, u, p) == g["result"]
    assert mu == g["result"]
    assert [c % p for c in g["R"]] == g["result"]


# --- Thm. 2 and the REDQ algorithm against the definition -----------------

@pytest.mark.parametrize("p,q,d", [(3, 8, 4), (5, 8, 3), (7, 16, 2), (3, 4, 5),
                                   (5, 6, 3), (2, 4, 4), (3, 10, 3)])
def test_redq_bruteforce(p, q, d):
    for r in range(q ** (d + 1)):
        rop, u, mu, rho = gf.redq_steps(r, p, q, d)
        assert all(0 <= x < p for x in u), (r, u)            # Thm. 2, first part
        assert u == [(r // q ** i) % p for i in range(d + 1)]  # Thm. 2, second part
        assert mu == [x % p for x in gf.qadic_digits(r, q, d + 1)]
        assert mu == gf.dqt_inverse(r, q, d + 1, p)


def test_lemma2_nested_floors():
    rnd = random.Random(7)
    for _ in range(5000):
        r = rnd.randrange(0, 10 ** 12)
        a, b = rnd.randrange(1, 1000), rnd.randrange(1, 1000)
        assert (r // b) // a == r // (a * b) == (r // a) // b


@pytest.mark.parametrize("d,q,p", [(3, 10 ** 6, 23), (6, 128, 3), (4, 1024, 5), (2, 2 ** 17, 7)])
def test_qd_inverts_toeplitz(d, q, p):
    Q = gf.q_matrix(d, q, p)
    T = gf.toeplitz_powers(d, q)
    prod = [[sum(Q[i][l] * T[l][j] for l in range(d + 1)) % p for j in range(d + 1)]
            for i in range(d + 1)]
    assert prod == [[int(i == j) for j in range(d + 1)] for i in range(d + 1)]


@pytest.mark.parametrize("q", [128, 1024, 10 ** 6, 5])
def test_alg3_q6_from_three_q2_exhaustive(q):
    p = 3
    Q6 = gf.q_matrix(6, q, p)
    for u in itertools.product(range(p), repeat=7):
        assert gf.q6_by_three_q2(u, q, p) == gf.mat_vec_mod(Q6, u, p)


@pytest.mark.parametrize("p,d,w", [(3, 6, 3), (3, 6, 4), (5, 4, 3), (2, 8, 5)])
def test_time_memory_windows(p, d, w):
    q = 2 ** 7 + 3
    Qd = gf.q_matrix(d, q, p)
    for u in itertools.product(range(p), repeat=d + 1):
        assert gf.q_by_windows(u, q, p, w) == gf.mat_vec_mod(Qd, u, p)


# --- polynomial products ----------------------------------------------------

def test_poly_mul_matches_numpy_convolve():
    rnd = np.random.default_rng(11)
    for _ in range(200):
        la, lb = rnd.integers(1, 9, size=2)
        a = rnd.integers(0, 50, size=la).tolist()
        b = rnd.integers(0, 50, size=lb).tolist()
        assert gf.poly_mul_z(a, b) == np.convolve(a, b).tolist()


def test_poly_mul_k1_is_integer_product():
    for p in (2, 3, 5, 7, 11):
        for x in range(p):
            for y in range(p):
                assert gf.poly_mul_mod_p([x], [y], p) == [(x * y) % p]


def test_polymul_batch_rowwise_and_exhaustive_cfg1():
    p, k = 5, 3
    elems = [list(e) for e in gf.all_elements(p, k)]
    a = np.array([x for x in elems for _ in elems], dtype=np.uint8)
    b = np.array([y for _ in elems for y in elems], dtype=np.uint8)
    out = gf.polymul_batch(a, b, p)
    rnd = random.Random(3)
    for idx in rnd.sample(range(len(a)), 400):
        want = [int(c) for c in np.convolve(a[idx].astype(int), b[idx].astype(int)) % p]
        assert out[idx].tolist() == want


def test_dqt_alg1_agrees_when_eq2_holds_and_fails_past_bound():
    p, k = 5, 3
    # q = 64 is the smallest power of two above k (p-1)^2 = 48
    assert gf.eq2_holds(p, k, 64, 1)
    for a in itertools.product(range(p), repeat=k):
        b = [p - 1] * k
        assert gf.polymul_dqt(list(a), b, p, 64) == gf.poly_mul_mod_p(list(a), b, p)
    # at q = k (p-1)^2 exactly the middle digit of (p-1,...)^2 reaches q and carries
    q = k * (p - 1) ** 2
    assert not gf.eq2_holds(p, k, q, 1)
    a = [p - 1] * k
    assert gf.polymul_dqt(a, a, p, q) != gf.poly_mul_mod_p(a, a, p)


# --- the fields -------------------------------------------------------------

def test_irreducible_counts_match_gauss_formula():
    # number of monic irreducible polynomials of degree n over GF(p):
    # (1/n) sum_{d | n} mobius(d) p^(n/d)
    def mobius(n):
        res, m, f = 1, n, 2
        while f * f <= m:
            if m % f == 0:
                m //= f
                if m % f == 0:
                    return 0
                res = -res
            f += 1
        return -res if m > 1 else res

    for p, n in [(2, 2), (2, 3), (2, 4), (3, 2), (3, 3), (3, 4), (5, 2), (5, 3), (7, 2)]:
        want = sum(mobius(d) * p ** (n // d) for d in range(1, n + 1) if n % d == 0) // n
        got = sum(gf.is_irreducible(list(low), p)
                  for low in itertools.product(range(p), repeat=n))
        assert got == want, (p, n)


@pytest.mark.parametrize("p,P_low", CONFIG_FIELDS)
def test_config_polynomials_irreducible(p, P_low):
    assert gf.is_irreducible(P_low, p)


def test_reducible_rejected():
    assert not gf.is_irreducible([2, 0], 3)      # X^2 + 2 = (X+1)(X+2) over GF(3)
    assert not gf.is_irreducible([0, 0, 1], 5)   # X^3 + X^2 = X^2 (X+1)


def test_gf9_textbook():
    # GF(9) = GF(3)[X]/(X^2+1): X is a square root of -1
    assert gf.field_mul([0, 1], [0, 1], 3, (1, 0)) == [2, 0]
    assert gf.field_mul([1, 1], [1, 2], 3, (1, 0)) == [2, 0]   # (1+X)(1+2X) = 1+3X+2X^2 = -1


@pytest.mark.parametrize("p,P_low", CONFIG_FIELDS)
def test_field_axioms(p, P_low):
    k = len(P_low)
    elems = [tuple(e) for e in gf.all_elements(p, k)]
    one = tuple([1] + [0] * (k - 1))
    zero = tuple([0] * k)
    mul = {}
    for a in elems:
        for b in elems:
            mul[a, b] = tuple(gf.field_mul(a, b, p, P_low))
    order = p ** k
    for a in elems:
        assert mul[a, one] == a
        assert mul[a, zero] == zero
        # a^(p^k) = a for every element
        assert tuple(gf.field_pow(a, order, p, P_low)) == a
        if a != zero:
            # inverse exists, hence no zero divisors
            inv = tuple(gf.field_pow(a, order - 2, p, P_low))
            assert mul[a, inv] == one
        for b in elems:
            assert mul[a, b] == mul[b, a]
            if a != zero and b != zero:
                assert mul[a, b] != zero
    rnd = random.Random(5)
    for _ in range(3000):
        a, b, c = (rnd.choice(elems) for _ in range(3))
        assert mul[mul[a, b], c] == mul[a, mul[b, c]]
        bc = tuple(gf.field_add(b, c, p))
        assert mul[a, bc] == tuple(gf.field_add(mul[a, b], mul[a, c], p))
        # Frobenius: (a + b)^p = a^p + b^p
        lhs = gf.field_pow(gf.field_add(a, b, p), p, p, P_low)
        rhs = gf.field_add(gf.field_pow(a, p, p, P_low), gf.field_pow(b, p, p, P_low), p)
        assert lhs == rhs
    # the multiplicative group is cyclic of order p^k - 1
    def elem_order(a):
        e, x = 1, a
        while x != one:
            x, e = mul[x, a], e + 1
        return e
    assert max(elem_order(a) for a in elems if a != zero) == order - 1


# --- GEMM over GF(p^k) -----------------------------------------------------

@pytest.mark.parametrize("p,P_low", CONFIG_FIELDS)
def test_gemm_two_reduction_orders_agree(p, P_low):
    k = len(P_low)
    rng = np.random.default_rng(21)
    A = rng.integers(0, p, size=(5, 7, k))
    B = rng.integers(0, p, size=(7, 6, k))
    small = np.array(gf.gemm_gfpk_small(A.tolist(), B.tolist(), p, P_low), dtype=np.uint8)
    planes = gf.gemm_gfpk_planes(A, B, p, P_low)
    assert np.array_equal(small, planes)
    for i in range(5):
        for j in range(6):
            assert gf.gemm_entry(A[i], B[:, j], p, P_low) == planes[i, j].tolist()


def test_gemm_k1_is_numpy_matmul_mod_p():
    p = 11
    rng = np.random.default_rng(3)
    A = rng.integers(0, p, size=(17, 29, 1))
    B = rng.integers(0, p, size=(29, 13, 1))
    want = (A[:, :, 0] @ B[:, :, 0]) % p
    # k = 1: the "field" is GF(p) itself; P = X + 0 has degree 1
    got = gf.gemm_gfpk_planes(A, B, p, [0])
    assert np.array_equal(got[:, :, 0], want)


@pytest.mark.parametrize("p,P_low", CONFIG_FIELDS)
def test_gemm_identity_and_associativity(p, P_low):
    k = len(P_low)
    rng = np.random.default_rng(8)
    A = rng.integers(0, p, size=(6, 6, k))
    I = np.zeros((6, 6, k), dtype=np.int64)
    for i in range(6):
        I[i, i, 0] = 1
    assert np.array_equal(gf.gemm_gfpk_planes(A, I, p, P_low), A)
    assert np.array_equal(gf.gemm_gfpk_planes(I, A, p, P_low), A)
    B = rng.integers(0, p, size=(6, 4, k))
    C = rng.integers(0, p, size=(4, 5, k))
    left = gf.gemm_gfpk_planes(gf.gemm_gfpk_planes(A, B, p, P_low), C, p, P_low)
    right = gf.gemm_gfpk_planes(A, gf.gemm_gfpk_planes(B, C, p, P_low), p, P_low)
    assert np.array_equal(left, right)


@pytest.mark.parametrize("p,P_low", CONFIG_FIELDS)
def test_freivalds_accepts_the_product_and_catches_every_single_wrong_byte(p, P_low):
    # the check the full-size GPU outputs go through: the true product
    # passes, and C with any one coefficient changed (every position of a
    # small C, every nonzero offset) fails with 20 vectors
    k = len(P_low)
    rng = np.random.default_rng(31 + p)
    A = rng.integers(0, p, size=(4, 6, k), dtype=np.uint8)
    B = rng.integers(0, p, size=(6, 3, k), dtype=np.uint8)
    C = gf.gemm_gfpk_planes(A, B, p, P_low)
    assert gf.freivalds(A, B, C, p, P_low, rng)
    for i, j, s in itertools.product(range(4), range(3), range(k)):
        for off in range(1, p):
            bad = C.copy()
            bad[i, j, s] = (int(bad[i, j, s]) + off) % p
            assert not gf.freivalds(A, B, bad, p, P_low, rng), (i, j, s, off)
    # a transposed-operand mistake (C = B^T A^T read as AB) is caught too
    A2 = rng.integers(0, p, size=(5, 5, k), dtype=np.uint8)
    B2 = rng.integers(0, p, size=(5, 5, k), dtype=np.uint8)
    wrong = gf.gemm_gfpk_planes(B2, A2, p, P_low)
    if not np.array_equal(wrong, gf.gemm_gfpk_planes(A2, B2, p, P_low)):
        assert not gf.freivalds(A2, B2, wrong, p, P_low, rng)


# --- Thm. 3: the L/H tables and Alg. 4 -------------------------------------

@pytest.mark.parametrize("p,P_low", CONFIG_FIELDS)
def test_lh_tables_reduce_the_corrected_digits(p, P_low):
    k = len(P_low)
    q, _ = gf.max_pow2_q(p, k)
    d = 2 * k - 2
    Qd = gf.q_matrix(d, q, p)
    for u in itertools.product(range(p), repeat=2 * k - 1):
        mu = gf.mat_vec_mod(Qd, u, p)
        want = gf.poly_rem(mu, P_low, p)
        got = gf.field_add(gf.table_L(u[:k], q, p), gf.table_H(u[k - 1:], q, p, P_low), p)
        assert got == want


@pytest.mark.parametrize("p,P_low", CONFIG_FIELDS)
def test_fgdp_equals_dot_product(p, P_low):
    k = len(P_low)
    q, nq = gf.max_pow2_q(p, k)
    rng = np.random.default_rng(4)
    for n in (1, 2, min(nq, 40), nq if nq <= 64 else 64):
        v1 = rng.integers(0, p, size=(n, k))
        v2 = rng.integers(0, p, size=(n, k))
        assert gf.fgdp(v1.tolist(), v2.tolist(), p, P_low, q) == gf.gemm_entry(v1, v2, p, P_low)
    # adversarial: all coefficients p-1 at the largest admissible block
    n = min(nq, 64)
    v = [[p - 1] * k] * n
    assert gf.fgdp(v, v, p, P_low, q) == gf.gemm_entry(np.array(v), np.array(v), p, P_low)


@pytest.mark.parametrize("p,k", [(7, 2), (3, 4), (5, 3), (3, 2), (5, 3)])
def test_max_pow2_q_is_tight(p, k):
    q, nq = gf.max_pow2_q(p, k)
    assert gf.eq2_holds(p, k, q, nq)
    assert not gf.eq2_holds(p, k, q, nq + 1)
    assert not gf.eq2_holds(p, k, 2 * q, 1)


def test_block_bound_is_tight_for_dot_products():
    # GF(3^4) at q = 2^7: n_q = 7 passes, n_q = 8 overflows the middle digit
    p, P_low, q = 3, (2, 0, 0, 2), 128
    k = 4
    v = [[p - 1] * k] * 7
    assert gf.eq2_holds(p, k, q, 7) and not gf.eq2_holds(p, k, q, 8)
    assert gf.fgdp(v, v, p, P_low, q) == gf.gemm_entry(np.array(v), np.array(v), p, P_low)
    v8 = [[p - 1] * k] * 8
    assert gf.fgdp(v8, v8, p, P_low, q) != gf.gemm_entry(np.array(v8), np.array(v8), p, P_low)


def test_binary_index_layout():
    assert gf.binary_index([1, 2, 0, 1], 3) == 1 + (2 << 2) + (1 << 6)
    assert gf.binary_index([4, 4, 4], 5) == 4 + (4 << 3) + (4 << 6)


# --- d-FQT: long polynomials in chunks of d+1 coefficients (Section 6) ----

def _binomial_row_mod_p(n, p):
    """Coefficients of (1 + X)^n mod p from exact binomial coefficients."""
    from math import comb
    return [comb(n, i) % p for i in range(n + 1)]


@pytest.mark.parametrize("p", [2, 3, 5, 7])
def test_polymul_long_binomial_closed_form(p):
    # (1 + X)^m (1 + X)^n = (1 + X)^(m+n): a closed form for every coefficient
    for m, n in [(0, 0), (1, 4), (7, 9), (30, 41), (500, 500)]:
        a = _binomial_row_mod_p(m, p)
        b = _binomial_row_mod_p(n, p)
        assert gf.polymul_long(a, b, p) == _binomial_row_mod_p(m + n, p)


def test_polymul_long_frobenius():
    # over GF(p), (1 + X)^p = 1 + X^p (freshman's dream), squared via the product
    for p in (3, 5, 7, 11):
        f = _binomial_row_mod_p(p, p)
        assert f == [1] + [0] * (p - 1) + [1]
        sq = gf.polymul_long(f, f, p)
        assert sq == _binomial_row_mod_p(2 * p, p)
        want = [0] * (2 * p + 1)
        want[0] = 1
        want[p] = 2 % p
        want[2 * p] = 1
        assert sq == want


def test_polymul_long_agrees_with_schoolbook():
    rng = random.Random(3)
    for p in (2, 3, 13, 127):
        for la, lb in [(1, 1), (3, 8), (64, 65), (200, 17)]:
            a = [rng.randrange(p) for _ in range(la)]
            b = [rng.randrange(p) for _ in range(lb)]
            assert gf.polymul_long(a, b, p) == gf.poly_mul_mod_p(a, b, p)


def test_dfqt_degree_of_the_papers_example():
    # p = 3, N = 500, d = 4: D_q = ceil(501 / 5) - 1 = 100 chunks beyond the first
    assert gf.dfqt_degree(501, 4) == 100
    assert gf.dfqt_degree(1, 0) == 0 and gf.dfqt_degree(5, 4) == 0 and gf.dfqt_degree(6, 4) == 1
    # chunks: the last one zero-padded, concatenation restores the operand
    a = list(range(13))
    ch = gf.dfqt_chunks(a, 4)
    assert [len(c) for c in ch] == [5, 5, 5] and sum(ch, [])[:13] == a and ch[-1][3:] == [0, 0]


def _eq2_params(p, d):
    """(q, n_q max) at the largest q = 2^b with q^(2d+1) < 2^53."""
    return gf.max_pow2_q(p, d + 1)


@pytest.mark.parametrize("p,d", [(2, 1), (3, 0), (3, 1), (3, 2), (3, 4), (5, 3), (7, 2), (13, 1)])
def test_dfqt_equals_the_product_definition(p, d):
    q, nq = _eq2_params(p, d)
    rng = random.Random(p * 10 + d)
    for la, lb in [(1, 1), (d + 1, d + 1), (d + 2, 3 * d + 4), (37, 29), (101, 101)]:
        a = [rng.randrange(p) for _ in range(la)]
        b = [rng.randrange(p) for _ in range(lb)]
        want = gf.polymul_long(a, b, p)
        for n_q in sorted({1, max(1, nq // 2), nq}):
            assert gf.dfqt_polymul(a, b, p, d, q, n_q) == want, (la, lb, n_q)
        # all (p-1): every block's digits reach their largest value
        amax, bmax = [p - 1] * la, [p - 1] * lb
        assert gf.dfqt_polymul(amax, bmax, p, d, q, nq) == gf.polymul_long(amax, bmax, p)


def test_dfqt_general_q():
    # eq. (2) with a q that is not a power of two (Section 2 allows any q)
    p, d = 3, 4
    q = 59                      # q^9 < 2^53 and q > 2 * 5 * 2^2
    assert q ** 9 < 2 ** 53 and q > 2 * (d + 1) * (p - 1) ** 2
    rng = random.Random(9)
    a = [rng.randrange(p) for _ in range(501)]
    b = [rng.randrange(p) for _ in range(501)]
    assert gf.dfqt_polymul(a, b, p, d, q, 2) == gf.polymul_long(a, b, p)


def test_dfqt_exhaustive_tiny():
    # every pair of polynomials with 3 coefficients over GF(2) and GF(3), d = 1
    for p in (2, 3):
        q, nq = _eq2_params(p, 1)
        for a in itertools.product(range(p), repeat=3):
            for b in itertools.product(range(p), repeat=3):
                assert gf.dfqt_polymul(list(a), list(b), p, 1, q, nq) == \
                    gf.poly_mul_mod_p(list(a), list(b), p)


def test_dfqt_block_bound_is_tight():
    # q = 16, p = 3, d = 1: eq. (2) allows n_q = 1 (16 > 8) but not 2 (16 = 16);
    # with every coefficient 2 a block of two products has a middle digit of
    # 2 * 2 * 4 = 16 = q, which carries into the next digit and breaks the result
    p, d, q = 3, 1, 16
    a = [2] * 8
    b = [2] * 8
    want = gf.polymul_long(a, b, p)
    assert gf.dfqt_polymul(a, b, p, d, q, 1) == want
    assert gf.dfqt_polymul(a, b, p, d, q, 2) != want


# ---- discrete-log representation (Section 7, Alg. 4) ------------------------

@pytest.mark.parametrize("name", ["log_gf4.txt", "log_gf9.txt"])
def test_log_tables_hand_derived(name):
    g = load(name)
    P_low = tuple(g["P_low"])
    gen, expo, logs = gf.log_tables(g["p"], P_low)
    assert gen == g["generator"]
    assert expo == g["exp_index"]
    assert gf.zech_table(g["p"], P_low) == g["zech"]


LOG_FIELDS = [(2, (1, 1)), (3, (1, 0)), (7, (1, 0)), (3, (2, 0, 0, 2)), (5, (3, 3, 0)),
              (2, (1, 0, 1)), (13, (2,)), (2, (1,))]


@pytest.mark.parametrize("p,P_low", LOG_FIELDS)
def test_log_generator_is_first_of_full_order(p, P_low):
    k = len(P_low)
    m = p ** k - 1
    g = gf.log_generator(p, P_low)
    ge = gf.elem_from_index(g, p, k)
    # brute force: g^e != 1 for 0 < e < m, g^m = 1, and every element of
    # smaller index has a proper divisor of m as its order
    one = [1] + [0] * (k - 1)
    x = list(ge)
    for e in range(1, m):
        assert x != one, e
        x = gf.field_mul(x, ge, p, P_low)
    assert x == one
    for idx in range(1, g):
        o = gf.mult_order(gf.elem_from_index(idx, p, k), p, P_low)
        assert o < m and m % o == 0


def test_x_is_the_generator_of_gf81_and_gf125():
    # X has order 80 in GF(3)[X]/(X^4 + 2X^3 + 2) and 124 in
    # GF(5)[X]/(X^3 + 3X + 3); constants have order dividing p - 1, so X
    # (index p) is the first element of full order
    assert gf.log_generator(3, (2, 0, 0, 2)) == 3
    assert gf.log_generator(5, (3, 3, 0)) == 5


@pytest.mark.parametrize("p,P_low", LOG_FIELDS)
def test_log_tables_bijective_and_zech_identities(p, P_low):
    k = len(P_low)
    m = p ** k - 1
    tabs = gf.log_tables(p, P_low)
    gen, expo, logs = tabs
    assert sorted(expo) == list(range(1, p ** k))       # g^e runs over every nonzero element
    assert all(logs[expo[e]] == e for e in range(m))
    Z = gf.zech_table(p, P_low)
    for n in range(m):
        # g^Z[n] = 1 + g^n in coefficient form
        one_plus = gf.field_add([1] + [0] * (k - 1), gf.from_log(n, p, P_low, tabs), p)
        assert gf.from_log(Z[n], p, P_low, tabs) == one_plus
        # Z[-n] = Z[n] - n mod m (multiply 1 + g^n by g^-n)
        if Z[n] != m:
            assert Z[(-n) % m] == (Z[n] - n) % m
    # 1 + g^n = 0 exactly for g^n = -1: n = m/2 for odd p, n = 0 for p = 2
    assert Z.index(m) == (0 if p == 2 else m // 2)
    assert Z.count(m) == 1


@pytest.mark.parametrize("p,P_low", LOG_FIELDS[:6])
def test_log_add_is_field_add(p, P_low):
    k = len(P_low)
    m = p ** k - 1
    tabs = gf.log_tables(p, P_low)
    Z = gf.zech_table(p, P_low)
    codes = range(m + 1) if m < 130 else random.Random(3).sample(range(m + 1), 130)
    for a in codes:
        for b in codes:
            want = gf.field_add(gf.from_log(a, p, P_low, tabs), gf.from_log(b, p, P_low, tabs), p)
            assert gf.from_log(gf.log_add(a, b, Z), p, P_low, tabs) == want


@pytest.mark.parametrize("p,P_low", [(7, (1, 0)), (3, (2, 0, 0, 2)), (5, (3, 3, 0)),
                                     (2, (1, 0, 1))])
def test_alg4_on_logs_matches_the_definition(p, P_low):
    # Alg. 4 step by step (tabulated conversion, REDQ, L and H as codes, Zech
    # addition), in blocks of n_q, against the product of the antilogs
    k = len(P_low)
    m = p ** k - 1
    q, nq = gf.max_pow2_q(p, k)
    rng = np.random.default_rng(p + k)
    for (M, K, N) in [(3, 1, 2), (4, 9, 3), (2, 2 * nq + 3, 2)]:
        A = rng.integers(0, m + 1, size=(M, K))
        B = rng.integers(0, m + 1, size=(K, N))
        A[0, 0] = m                            # zeros are codes too
        want = gf.gemm_log(A, B, p, P_low)
        got = gf.gemm_log_alg4(A.tolist(), B.tolist(), p, P_low, q, nq)
        assert np.array_equal(np.array(got), want), (M, K, N)
    # every element p-1 coefficient-wise: the packed sums reach eq. (2)'s bound
    full = gf.to_log([p - 1] * k, p, P_low)
    A = np.full((2, nq), full)
    B = np.full((nq, 2), full)
    assert np.array_equal(np.array(gf.gemm_log_alg4(A.tolist(), B.tolist(), p, P_low, q, nq)),
                          gf.gemm_log(A, B, p, P_low))


def test_gemm_log_definition_on_small_cases():
    # the log-form definition against the one-product-at-a-time field
    # arithmetic on codes: a sum of g^(a+b) terms built with log_add
    p, P_low = 5, (3, 3, 0)
    m = p ** 3 - 1
    Z = gf.zech_table(p, P_low)
    rng = np.random.default_rng(11)
    A = rng.integers(0, m + 1, size=(3, 7))
    B = rng.integers(0, m + 1, size=(7, 4))
    C = gf.gemm_log(A, B, p, P_low)
    for i in range(3):
        for j in range(4):
            acc = m
            for l in range(7):
                a, b = int(A[i, l]), int(B[l, j])
                prod = m if m in (a, b) else (a + b) % m      # g^a g^b = g^(a+b)
                acc = gf.log_add(acc, prod, Z)
            assert C[i, j] == acc


# ---- Winograd's product over GF(p^k) -----------------------------------------

@pytest.mark.parametrize("p,P_low", [(7, (1, 0)), (3, (2, 0, 0, 2)), (5, (3, 3, 0)), (2, (1, 0, 1)),
                                     (13, (2,))])
def test_winograd_matches_the_definition(p, P_low):
    k = len(P_low)
    rng = np.random.default_rng(p * 10 + k)
    for (M, N, K) in [(2, 2, 2), (4, 6, 8), (7, 5, 9), (16, 16, 16), (33, 18, 21), (3, 2, 1),
                      (1, 5, 4)]:
        A = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        B = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
        want = gf.gemm_gfpk_planes(A, B, p, P_low)
        for levels in (1, 2, 3):
            assert np.array_equal(gf.gemm_winograd(A, B, p, P_low, levels), want), (M, N, K, levels)


def test_winograd_one_level_by_hand_gf2():
    # GF(2), 2 x 2 blocks of 1 x 1: the seven products and fifteen additions
    # against the 2 x 2 product written out
    A = np.array([[1, 1], [0, 1]], dtype=np.uint8).reshape(2, 2, 1)
    B = np.array([[1, 0], [1, 1]], dtype=np.uint8).reshape(2, 2, 1)
    # [[1+1, 0+1], [0+1, 0+1]] mod 2
    want = np.array([[0, 1], [1, 1]], dtype=np.uint8).reshape(2, 2, 1)
    assert np.array_equal(gf.gemm_winograd(A, B, 2, (1,), 1), want)


def test_winograd_identity_and_zero():
    p, P_low = 5, (3, 3, 0)
    k = 3
    rng = np.random.default_rng(4)
    A = rng.integers(0, p, size=(12, 12, k), dtype=np.uint8)
    I = np.zeros((12, 12, k), dtype=np.uint8)
    for i in range(12):
        I[i, i, 0] = 1
    assert np.array_equal(gf.gemm_winograd(A, I, p, P_low, 2), A)
    assert np.array_equal(gf.gemm_winograd(I, A, p, P_low, 2), A)
    assert not gf.gemm_winograd(A, np.zeros_like(A), p, P_low, 2).any()


# ---- centred packing -----------------------------------------------------------

@pytest.mark.parametrize("p,P_low", [(3, (2, 0, 0, 2)), (5, (3, 3, 0)), (7, (1, 0)), (3, (1, 0)),
                                     (13, (2,))])
def test_centred_alg4_matches_the_definition(p, P_low):
    k = len(P_low)
    q, _ = gf.max_pow2_q(p, k)
    nq = min(gf.centred_nq_max(p, k, q), 64)
    rng = np.random.default_rng(p * k)
    for (M, K, N) in [(3, 1, 2), (4, 9, 3), (2, 2 * nq + 3, 2)]:
        A = rng.integers(0, p, size=(M, K, k))
        B = rng.integers(0, p, size=(K, N, k))
        got = gf.gemm_centred_alg4(A.tolist(), B.tolist(), p, P_low, q, nq)
        want = gf.gemm_gfpk_planes(A.astype(np.uint8), B.astype(np.uint8), p, P_low)
        assert np.array_equal(np.array(got, dtype=np.uint8).reshape(want.shape), want), (M, K, N)


@pytest.mark.parametrize("p,P_low", [(3, (2, 0, 0, 2)), (5, (3, 3, 0)), (7, (1, 0))])
def test_centred_bound_is_tight(p, P_low):
    # the extreme digit sums: every centred coefficient h against every h
    # (all products +h^2) and against -h (all -h^2).  At n_q = centred_nq_max
    # both are exact; one product more pushes the positive extreme to q/2,
    # whose shifted digit q carries into the next one and breaks the result
    # (the negative side may reach -q/2 exactly: shifted digit 0)
    k = len(P_low)
    h = (p - 1) // 2
    q, _ = gf.max_pow2_q(p, k)
    if q > 2 ** 10:
        q = 2 ** 10                    # a small q keeps the case short
    nq = gf.centred_nq_max(p, k, q)
    pos, neg = [h] * k, [p - h] * k    # centred values h and -h

    def run(b, n):
        A = [[pos] * n]
        B = [[b] for _ in range(n)]
        got = gf.gemm_centred_alg4(A, B, p, P_low, q, n)
        want = gf.gemm_gfpk_planes(np.array(A, dtype=np.uint8), np.array(B, dtype=np.uint8),
                                   p, P_low)
        return np.array_equal(np.array(got, dtype=np.uint8).reshape(want.shape), want)

    assert run(pos, nq) and run(neg, nq)
    assert not run(pos, nq + 1)


def test_centred_doubles_n_q():
    # GF(3^4) at q = 2^7: 7 products per block in [0, p), 15 centred;
    # GF(5^3) at q = 2^10: 21 and 42; GF(7^2) at q = 2^17: 1820 and 3640
    assert gf.centred_nq_max(3, 4, 2 ** 7) == 15 and gf.max_pow2_q(3, 4)[1] == 7
    assert gf.centred_nq_max(5, 3, 2 ** 10) == 42 and gf.max_pow2_q(5, 3)[1] == 21
    assert gf.centred_nq_max(7, 2, 2 ** 17) == 3640 and gf.max_pow2_q(7, 2)[1] == 1820


@pytest.mark.parametrize("p,d", [(3, 4), (3, 3), (5, 2), (7, 1), (3, 0), (13, 1)])
def test_dfqt_centred_matches_the_definition(p, d):
    b = 52 // (2 * d + 1)
    q = 2 ** b
    h = (p - 1) // 2
    nq = (q // 2 - 1) // ((d + 1) * h * h)
    assert nq >= 1
    rng = random.Random(p * 10 + d)
    for (la, lb) in [(1, 1), (5, 3), (40, 17), (501, 501)]:
        a = [rng.randrange(p) for _ in range(la)]
        b_ = [rng.randrange(p) for _ in range(lb)]
        want = gf.polymul_long(a, b_, p)
        for n_q in sorted({1, max(1, nq // 2), nq}):
            assert gf.dfqt_polymul_centred(a, b_, p, d, q, n_q) == want, (la, lb, n_q)
    # the extremes: all h (every chunk product digit +h^2 per term) and h
    # against -h, in blocks at the centred bound
    for bv in (h, p - h):
        a = [h] * 200
        b_ = [bv] * 200
        assert gf.dfqt_polymul_centred(a, b_, p, d, q, nq) == gf.polymul_long(a, b_, p)


def test_dfqt_centred_n_q_for_the_workload():
    # p = 3, d = 4: q = 2^5 holds one [0, p) chunk product per block (5 * 4 < 32)
    # and three centred ones (3 * 5 * 1 <= 15)
    q = 2 ** 5
    assert (q - 1) // (5 * 4) == 1
    assert (q // 2 - 1) // (5 * 1) == 3
