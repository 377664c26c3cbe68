"""Pins of the low-precision conversion oracle (oracle/lowprec.py), CPU only.

The BF16 rounding is checked against a brute-force search over BF16 bit patterns
(the two neighbours of each value and the rounding rule written out), against
exactly constructed ties, and against the error bounds of an 8-bit significand.
"""
import numpy as np
import pytest

from oracle import lowprec as lp


def _brute_bf16(a: float) -> float:
    """Nearest BF16 number to a by enumeration of candidate bit patterns; ties go to
    the pattern with an even last bit."""
    if a == 0.0:
        return 0.0
    f = np.float32(a)                      # within one FP32 ulp of a
    base = int(np.array([f], dtype=np.float32).view(np.uint32)[0]) >> 16
    best = None
    for bits in range(max(base - 2, 0), min(base + 3, 0xFFFF) + 1):
        v = float(lp.bf16_value(np.array([bits]))[0])
        if not np.isfinite(v):
            continue
        d = abs(v - a)
        key = (d, bits & 1)               # nearer first, then the even pattern
        if best is None or key < best[0]:
            best = (key, v)
    return best[1]


def test_bf16_matches_brute_force_search():
    rng = np.random.default_rng(7)
    vals = np.concatenate([
        rng.standard_normal(400) * np.exp(rng.uniform(-30, 30, 400)),
        rng.uniform(-1, 1, 200),
        np.array([1.0, -1.0, 3.0, 1e-3, 123456.789, 2.0 ** -120, -(2.0 ** 100)]),
    ])
    got = lp.bf16_rne(vals)
    want = np.array([_brute_bf16(float(v)) for v in vals])
    assert np.array_equal(got, want)


def test_bf16_ties_go_to_even():
    # 1 + k/128 are BF16 numbers (7 stored bits); the midpoints 1 + (k + 1/2)/128
    # must round to the neighbour with an even k.
    for k in range(0, 127):
        mid = 1.0 + (k + 0.5) / 128.0
        r = float(lp.bf16_rne(np.array([mid]))[0])
        even = k if k % 2 == 0 else k + 1
        assert r == 1.0 + even / 128.0, (k, r)
    # one unit past a midpoint (in FP64) rounds away from it
    assert float(lp.bf16_rne(np.array([1.0 + 0.5 / 128 + 2.0 ** -40]))[0]) == 1.0 + 1 / 128
    # a value just below a midpoint that FP32 rounding would carry onto the midpoint
    # (double rounding) must still round down
    x = 1.0 + 1.5 / 128.0 - 2.0 ** -30
    assert float(lp.bf16_rne(np.array([x]))[0]) == 1.0 + 1 / 128


def test_bf16_values_and_bounds():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(5000) * np.exp(rng.uniform(-20, 20, 5000))
    hi = lp.bf16_rne(a)
    m, e = np.frexp(a)
    # 8 significant bits
    q = np.ldexp(hi, 8 - e)
    assert np.array_equal(q, np.round(q))
    # within half a unit of the 8th bit
    assert np.all(np.abs(a - hi) <= np.ldexp(0.5, e - 8))
    # bit patterns round-trip
    assert np.array_equal(lp.bf16_value(lp.bf16_bits(hi)), hi)


def test_bf16x2_carries_sixteen_bits():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((64, 64)) * 10.0
    hi, lo = lp.to_bf16x2(A)
    err = np.abs(A - (hi + lo))
    # |A - hi| <= 2^-8 |A| and lo rounds that remainder to 8 bits: <= 2^-16 |A|
    assert np.all(err <= np.abs(A) * 2.0 ** -16)
    assert np.all(np.abs(lo) <= np.abs(A) * 2.0 ** -8)
    # the pair is much better than hi alone
    assert err.max() < np.abs(A - hi).max() / 50


def test_f32_is_nearest_even():
    # 1 + 2^-24 is the midpoint of 1 and 1 + 2^-23: ties to even gives 1
    assert lp.to_f32(np.array([1.0 + 2.0 ** -24]))[0] == np.float32(1.0)
    assert lp.to_f32(np.array([1.0 + 3 * 2.0 ** -24]))[0] == np.float32(1.0 + 2.0 ** -22)
    rng = np.random.default_rng(11)
    a = rng.standard_normal(1000)
    f = lp.to_f32(a).astype(np.float64)
    m, e = np.frexp(a)
    assert np.all(np.abs(a - f) <= np.ldexp(0.5, e - 24))


@pytest.mark.parametrize("bad", ["half_up", "truncate"])
def test_planted_rounding_mistakes_are_caught(bad, monkeypatch):
    """A half-up or truncating rounding in place of ties-to-even fails the pins."""
    def wrong(a):
        a = np.asarray(a, dtype=np.float64)
        m, e = np.frexp(a)
        s = m * 256.0
        q = np.floor(s + 0.5) if bad == "half_up" else np.trunc(s)
        return np.ldexp(q, e - 8)
    monkeypatch.setattr(lp, "bf16_rne", wrong)
    with pytest.raises(AssertionError):
        test_bf16_ties_go_to_even()
