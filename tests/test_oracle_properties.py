"""Property checks of the CPU oracle over randomly drawn codes (hypothesis):
any field polynomial of the library's two field sizes, any k and m that fit,
any data.  Every encoded codeword vanishes at the roots of g(x) (evaluated by
Horner's rule with the product table, independently of the oracle's encode),
encoding is linear (the update property of Sec. 3.2), and decoding any
erasure pattern of at most m blocks gives the erased blocks back
(Sec. 3.3)."""
import numpy as np
import pytest

import oracle

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

# primitive polynomials of GF(2^4) and GF(2^8) (x = alpha generates the field)
POLYS = {4: (0x13, 0x19), 8: (0x11D, 0x12B, 0x12D, 0x14D, 0x15F, 0x163, 0x165, 0x169,
                          0x171, 0x187, 0x18D, 0x1A9, 0x1C3, 0x1CF, 0x1E7, 0x1F5)}
FIELDS = {}


def field(w, poly):
    if (w, poly) not in FIELDS:
        FIELDS[(w, poly)] = oracle.Field(w, poly)
    return FIELDS[(w, poly)]


@st.composite
def codes(draw):
    w = draw(st.sampled_from((4, 8)))
    poly = draw(st.sampled_from(POLYS[w]))
    n_max = (1 << w) - 1
    m = draw(st.integers(1, min(8, n_max - 1)))
    k = draw(st.integers(1, min(24, n_max - m)))
    cols = draw(st.integers(1, 24))
    seed = draw(st.integers(0, 2 ** 32 - 1))
    rng = np.random.default_rng(seed)
    data = rng.integers(0, 1 << w, size=(k, cols), dtype=np.uint8)
    return w, poly, k, m, data, rng


def horner(mul, coeffs, x):
    acc = np.zeros(coeffs.shape[1], dtype=np.uint8)
    for d in range(coeffs.shape[0] - 1, -1, -1):
        acc = mul[acc, x] ^ coeffs[d]
    return acc


@settings(max_examples=60, deadline=None)
@given(codes())
def test_codewords_vanish_at_the_roots(c):
    w, poly, k, m, data, _ = c
    F = field(w, poly)
    par = oracle.encode(F, k, m, data)
    mul = F.mul_table()
    word = np.concatenate([par, data], axis=0)   # degrees 0..m-1 parity, then data
    for i in range(m):
        assert not horner(mul, word, F.alpha_pow(i)).any()


@settings(max_examples=60, deadline=None)
@given(codes())
def test_encode_is_linear(c):
    w, poly, k, m, data, rng = c
    F = field(w, poly)
    other = rng.integers(0, 1 << w, size=data.shape, dtype=np.uint8)
    assert np.array_equal(oracle.encode(F, k, m, data ^ other),
                          oracle.encode(F, k, m, data) ^ oracle.encode(F, k, m, other))


@settings(max_examples=60, deadline=None)
@given(codes(), st.data())
def test_decode_restores_any_pattern(c, d):
    w, poly, k, m, data, rng = c
    F = field(w, poly)
    full = np.concatenate([data, oracle.encode(F, k, m, data)])
    t = d.draw(st.integers(1, m))
    er = sorted(rng.choice(k + m, size=t, replace=False).tolist())
    recv = full.copy()
    recv[er] = 0
    oracle.decode(F, k, m, recv, er)
    assert np.array_equal(recv, full)
