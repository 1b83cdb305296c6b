"""Pins the CPU oracle to facts fixed outside itself (no GPU needed).

Each test checks the oracle against something it does not compute the same
way: the numbers the paper prints for its worked example, closed forms,
invariants of cyclic codes, textbook special cases, and brute force over tiny
GF(2^4) codes.  A plausible slip in the oracle (a dropped term, a wrong sign
or index, a transposed operand, a wrong root offset, a wrong field
polynomial) fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import oracle
import workloads

F8 = None


def f8():
    global F8
    if F8 is None:
        F8 = oracle.Field(8, 0x11D)
    return F8


def poly_eval_columns(mul, coeffs, x):
    """Evaluates sum_d coeffs[d] * x^d per column; coeffs (deg+1, B).
    Horner's rule with the product table (independent of the oracle's
    encode and decode routines)."""
    acc = np.zeros(coeffs.shape[1], dtype=np.uint8)
    for d in range(coeffs.shape[0] - 1, -1, -1):
        acc = mul[acc, x] ^ coeffs[d]
    return acc


def codeword_coeffs(k, m, data, parity):
    """Stack into coefficient order: degrees 0..m-1 parity, m..m+k-1 data."""
    return np.concatenate([parity, data], axis=0)


# ------------------------------------------------------------- field ----

def test_powers_printed_in_vandermonde_example(golden_example):
    # Sec. 3.3, step 2: the matrix is printed both as alpha^e and as bytes.
    F = f8()
    exps = golden_example["vandermonde_exponents"]
    vals = golden_example["vandermonde"]
    assert [F.alpha_pow(e) for e in exps] == vals


def test_powers_of_two_pin_0x11d():
    # alpha^8 = 29 and alpha^10 = 116 (Sec. 3.3 example) reduce x^8 by 0x11D:
    # 2^8 = 256 -> 256 ^ 0x11D = 29.  Any other polynomial gives another byte.
    F = f8()
    assert F.alpha_pow(8) == 0x11D ^ 0x100
    assert [F.alpha_pow(e) for e in range(8)] == [1 << e for e in range(8)]


@pytest.mark.parametrize("w,count", [(4, 2), (8, 16)])
def test_number_of_primitive_polynomials(w, count):
    # Closed form: there are phi(2^w - 1) / w primitive polynomials of degree w
    # (phi(15)/4 = 2, phi(255)/8 = 16).  The oracle's primitivity check must
    # accept exactly that many.
    ok = []
    for poly in range(1 << w, 1 << (w + 1)):
        try:
            oracle.Field(w, poly)
            ok.append(poly)
        except ValueError:
            pass
    assert len(ok) == count
    assert (0x13 in ok) if w == 4 else (0x11D in ok)


@pytest.mark.parametrize("w,poly", [(8, 0x11D), (4, 0x13), (4, 0x19)])
def test_product_table_matches_log_exp(w, poly):
    # Two independent constructions of the product: shift-and-add table versus
    # alpha^(log a + log b).
    F = oracle.Field(w, poly)
    mul = F.mul_table()
    exp = F.exp_table()
    log = F.log_table()
    a = np.arange(1, F.q)
    lhs = mul[1:, 1:]
    rhs = exp[(log[a][:, None] + log[a][None, :]) % F.order]
    assert np.array_equal(lhs, rhs)
    assert not mul[0].any() and not mul[:, 0].any()
    # exp is a permutation of the nonzero elements
    assert sorted(exp.tolist()) == list(range(1, F.q))


def test_field_axioms():
    F = f8()
    mul = F.mul_table()
    rng = np.random.default_rng(1)
    a, b, c = rng.integers(0, 256, (3, 20000))
    assert np.array_equal(mul[a, b], mul[b, a])
    assert np.array_equal(mul[mul[a, b], c], mul[a, mul[b, c]])
    assert np.array_equal(mul[a, b ^ c], mul[a, b] ^ mul[a, c])
    # every nonzero element has an inverse, and 1 is the identity
    assert all((mul[x] == 1).sum() == 1 for x in range(1, 256))
    assert np.array_equal(mul[1], np.arange(256))


# -------------------------------------------------------------- g(x) ----

def test_genpoly_worked_example(golden_example):
    # Sec. 3.1: (x+2^0)(x+2^1)(x+2^2) = x^3 + 7x^2 + 14x + 8
    assert oracle.genpoly(f8(), 3).tolist() == golden_example["genpoly_m3"]


@pytest.mark.parametrize("m", range(1, 17))
def test_genpoly_roots_are_first_m_powers(m):
    # Sec. 3.1: the roots of g are alpha^0 .. alpha^(m-1); g is monic of
    # degree m and alpha^m is not a root (so the roots start at alpha^0).
    F = f8()
    g = oracle.genpoly(F, m)
    mul = F.mul_table()
    assert g[m] == 1
    for i in range(m + 2):
        val = poly_eval_columns(mul, g[:, None], F.alpha_pow(i))[0]
        assert (val == 0) == (i < m), (m, i)


def test_genpoly_m1_is_x_plus_1():
    assert oracle.genpoly(f8(), 1).tolist() == [1, 1]


# ------------------------------------------------------------ encode ----

def test_encode_worked_example(golden_example):
    # Sec. 3.2, example after eq. (2)
    F = f8()
    data = np.array(golden_example["data"], dtype=np.uint8)[:, None]
    par = oracle.encode(F, 4, 3, data)
    assert par[:, 0].tolist() == golden_example["parity"]


def test_only_0x11d_reproduces_the_example(golden_example):
    # The paper names the primitive root (2) but not the field polynomial;
    # among the 16 primitive polynomials only 0x11D yields the printed parity.
    data = np.array(golden_example["data"], dtype=np.uint8)[:, None]
    hits = []
    for poly in range(0x100, 0x200):
        try:
            F = oracle.Field(8, poly)
        except ValueError:
            continue
        if oracle.encode(F, 4, 3, data)[:, 0].tolist() == golden_example["parity"]:
            hits.append(poly)
    assert hits == [0x11D]


def test_reversed_data_order_is_excluded(golden_example):
    # Eq. (2) could be read with d_0 on the highest degree; that reading gives
    # a different parity than the one printed, so it is not the paper's.
    F = f8()
    data = np.array(golden_example["data"][::-1], dtype=np.uint8)[:, None]
    assert oracle.encode(F, 4, 3, data)[:, 0].tolist() != golden_example["parity"]


@pytest.mark.parametrize("k,m", [(1, 1), (4, 3), (6, 3), (10, 4), (12, 4), (32, 8),
                                 (5, 16), (200, 55), (3, 7)])
def test_codewords_vanish_at_the_roots(k, m):
    # p(x) + x^m d(x) = 0 mod g (Sec. 3.3), so the codeword evaluates to 0 at
    # every root alpha^i, i < m, and (being of degree < n <= order) not at
    # alpha^m for random data.
    F = f8()
    data = workloads.random_bytes(k * 100 + m, (k, 129))
    par = oracle.encode(F, k, m, data)
    c = codeword_coeffs(k, m, data, par)
    mul = F.mul_table()
    for i in range(m):
        assert not poly_eval_columns(mul, c, F.alpha_pow(i)).any(), i
    assert poly_eval_columns(mul, c, F.alpha_pow(m)).any()


@pytest.mark.parametrize("k", [1, 2, 7, 32])
def test_m1_parity_is_xor_of_data(k):
    # g = x + 1 and x^e mod (x+1) = 1, so single parity is the XOR of the data.
    F = f8()
    data = workloads.random_bytes(k, (k, 1000))
    par = oracle.encode(F, k, 1, data)
    assert np.array_equal(par[0], np.bitwise_xor.reduce(data, axis=0))


def test_encode_linearity():
    # Update property (Sec. 3.2): encoding the data difference gives the
    # parity difference.
    F = f8()
    a = workloads.random_bytes(11, (10, 4096))
    b = workloads.random_bytes(12, (10, 4096))
    pa, pb = oracle.encode(F, 10, 4, a), oracle.encode(F, 10, 4, b)
    assert np.array_equal(oracle.encode(F, 10, 4, a ^ b), pa ^ pb)


def x_power_mod_g(mul, g, m, e):
    """Coefficients of x^e mod g(x), by e multiplications by x (an LFSR
    shift), not by long division of a full polynomial."""
    r = np.zeros(m, dtype=np.uint8)
    r[0] = 1
    for _ in range(e):
        lead = r[m - 1]
        r = np.concatenate([[0], r[:-1]]).astype(np.uint8)
        r ^= mul[lead, g[:m]]
    return r


@pytest.mark.parametrize("k,m", [(4, 3), (10, 4), (6, 3), (32, 8), (3, 1)])
def test_encode_equals_generator_matrix_closed_form(k, m):
    # Sec. 6: the polynomial code is the matrix code with
    # P[i][j] = coefficient i of x^(m+j) mod g(x).
    F = f8()
    mul = F.mul_table()
    g = oracle.genpoly(F, m)
    P = np.stack([x_power_mod_g(mul, g, m, m + j) for j in range(k)], axis=1)
    data = workloads.random_bytes(k + 7 * m, (k, 777))
    expect = np.zeros((m, data.shape[1]), dtype=np.uint8)
    for i in range(m):
        for j in range(k):
            expect[i] ^= mul[P[i, j], data[j]]
    assert np.array_equal(oracle.encode(F, k, m, data), expect)


# ------------------------------------------------------------ decode ----

def test_decode_worked_example(golden_example):
    # Sec. 3.3: erase d0..d2, syndromes (70, 91, 171), Vandermonde matrix as
    # printed, solution (48, 6, 112).
    F = f8()
    er = golden_example["erasures"]
    word = np.array(golden_example["data"] + golden_example["parity"], dtype=np.uint8)
    word_erased = word.copy()
    word_erased[er] = 0
    assert oracle.syndromes(F, 4, 3, word_erased, er).tolist() == golden_example["syndromes"]
    assert oracle.vandermonde(F, 4, 3, er).ravel().tolist() == golden_example["vandermonde"]
    blocks = word_erased[:, None].copy()
    oracle.decode(F, 4, 3, blocks, er)
    assert blocks[er, 0].tolist() == golden_example["recovered"]


def test_positions_follow_eq2():
    # data d_j on degree m+j, parity p_i on degree i
    assert [oracle.position(4, 3, b) for b in range(7)] == [3, 4, 5, 6, 0, 1, 2]


def test_decode_every_pattern_rs63():
    # Any k of the n blocks recover the data (Sec. 1); all 130 patterns of
    # RS(6,3) including the empty one, erased rows filled with garbage.
    F = f8()
    k, m, B = 6, 3, 517
    data = workloads.random_bytes(7, (k, B))
    full = np.concatenate([data, oracle.encode(F, k, m, data)])
    pats = workloads.all_patterns(k + m, m)
    assert len(pats) == 130
    rng = np.random.default_rng(3)
    for er in pats:
        blocks = full.copy()
        for b in er:
            blocks[b] = rng.integers(0, 256, B, dtype=np.uint8)
        rng.shuffle(er)  # order of the list does not matter
        oracle.decode(F, k, m, blocks, er)
        assert np.array_equal(blocks, full), er


def test_decode_all_parity_erased_equals_encode():
    # Sec. 3.3: the procedure is symmetric; with all m parity erased, decoding
    # computes what encoding does.
    F = f8()
    k, m = 10, 4
    data = workloads.random_bytes(9, (k, 3000))
    blocks = np.concatenate([data, np.zeros((m, 3000), dtype=np.uint8)])
    oracle.decode(F, k, m, blocks, list(range(k, k + m)))
    assert np.array_equal(blocks[k:], oracle.encode(F, k, m, data))


@pytest.mark.parametrize("k,m", [(2, 2), (3, 2), (2, 3), (4, 3)])
def test_bruteforce_gf16_every_vector_every_pattern(k, m):
    # Brute force: all 16^k data vectors (one per column) and every erasure
    # pattern of size <= m on GF(2^4).
    F = oracle.Field(4, 0x13)
    cols = np.array(list(itertools.product(range(16), repeat=k)), dtype=np.uint8).T
    data = np.ascontiguousarray(cols)
    full = np.concatenate([data, oracle.encode(F, k, m, data)])
    for er in workloads.all_patterns(k + m, m):
        blocks = full.copy()
        blocks[er] = 0x0F
        oracle.decode(F, k, m, blocks, er)
        assert np.array_equal(blocks, full), er


@pytest.mark.parametrize("k,m", [(2, 2), (3, 2)])
def test_bruteforce_gf16_mds_distance(k, m):
    # The code is MDS: distinct codewords differ in at least m+1 symbols, and
    # the bound is met.  Checked over all pairs of codewords.
    F = oracle.Field(4, 0x19)
    data = np.ascontiguousarray(
        np.array(list(itertools.product(range(16), repeat=k)), dtype=np.uint8).T)
    cw = np.concatenate([data, oracle.encode(F, k, m, data)]).T.astype(np.int16)
    dmin = k + m
    for i in range(cw.shape[0]):
        d = (cw[i + 1:] != cw[i]).sum(axis=1)
        if d.size:
            dmin = min(dmin, int(d.min()))
    assert dmin == m + 1


def test_bruteforce_gf256_rs21_all_vectors():
    F = f8()
    data = np.ascontiguousarray(
        np.array(list(itertools.product(range(256), repeat=2)), dtype=np.uint8).T)
    full = np.concatenate([data, oracle.encode(F, 2, 1, data)])
    for er in workloads.all_patterns(3, 1):
        blocks = full.copy()
        blocks[er] = 0xA5
        oracle.decode(F, 2, 1, blocks, er)
        assert np.array_equal(blocks, full)


def test_invert_round_trip():
    F = f8()
    mul = F.mul_table()
    rng = np.random.default_rng(5)
    for t in range(1, 9):
        for _ in range(20):
            A = rng.integers(0, 256, (t, t), dtype=np.uint8)
            try:
                Ai = oracle.invert(F, A)
            except ValueError:
                continue
            prod = np.zeros((t, t), dtype=np.uint8)
            for i in range(t):
                for j in range(t):
                    acc = 0
                    for x in range(t):
                        acc ^= int(mul[A[i, x], Ai[x, j]])
                    prod[i, j] = acc
            assert np.array_equal(prod, np.eye(t, dtype=np.uint8))


def test_oracle_rejects_bad_arguments():
    F = f8()
    blocks = np.zeros((7, 4), dtype=np.uint8)
    for er in ([0, 1, 2, 3], [0, 0], [7], [-1]):
        with pytest.raises(ValueError):
            oracle.decode(F, 4, 3, blocks, er)
    with pytest.raises(ValueError):
        oracle.encode(F, 250, 6, np.zeros((250, 1), dtype=np.uint8))
    with pytest.raises(ValueError):
        oracle.Field(8, 0x11B)  # irreducible (AES) but x is not primitive
