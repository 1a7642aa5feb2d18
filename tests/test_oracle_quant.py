"""Pins of the core-quantization oracle (oracle/quant.py) against what the
paper and the arithmetic fix, independently of the oracle's own formulas:

* Table 2 of Section 3.3: the leading / trailing / sign classification, the
  run lengths and the significant set of the printed 2 x 2 x 2 example at its
  printed breakpoint (fixture tests/golden/table2_bitplanes.json, derived by
  hand from the table);
* the scale exponent of Section 3.3 on closed forms;
* the dequantization correction of Section 4.3: over all integers a whose
  bits above plane p are fixed, the squared errors sum to
  m (m^2 + 2) / 12 with m = 2^p (the discrete form of the paper's 2^(2p)/12),
  against m (m - 1) (2m - 1) / 6 without the correction;
* the breakpoint of Sections 3.3 / 4.2 by brute force: every position of the
  walk decoded from its own stream and its error summed directly;
* round trips: decoding recovers every encoded bit exactly, and with every bit
  encoded the core up to the rounding to integers.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import quant

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _table2():
    with open(os.path.join(GOLDEN, "table2_bitplanes.json")) as f:
        g = json.load(f)
    top = g["top_plane"]
    q = [sum(b << (top - i) for i, b in enumerate(row)) for row in g["bits"]]
    neg = [bool(s) for s in g["sign"]]
    return g, q, neg


def test_table2_fields_at_printed_breakpoint():
    g, q, neg = _table2()
    P, c = g["breakpoint_plane"], g["breakpoint_position"]
    runs, signs, trail = quant.encode_block_fields(q, neg, P, c)
    assert runs == g["runs"]
    assert signs == g["signs"]
    assert trail == g["trailing"]


def test_table2_significance_and_bit_categories():
    g, q, neg = _table2()
    P, c = g["breakpoint_plane"], g["breakpoint_position"]
    low = quant.lowest_planes(len(q), P, c)
    assert [64 - p for p in low] == g["encoded_bits_per_coefficient"]
    sig = [g["names"][i] for i in range(len(q)) if (q[i] >> low[i]) != 0]
    assert sig == g["significant"]
    # leading bits: the encoded planes down to and including the first one-bit
    for i in range(len(q)):
        known = 64 - low[i]
        first_one = next((t for t in range(known) if (q[i] >> (63 - t)) & 1), None)
        lead = known if first_one is None else first_one + 1
        assert lead == g["leading_bits_per_coefficient"][i], g["names"][i]
        assert known - lead == g["trailing_bits_per_coefficient"][i], g["names"][i]


def test_table2_stream_round_trip():
    g, q, neg = _table2()
    P, c = g["breakpoint_plane"], g["breakpoint_position"]
    words = quant.encode_block(q, neg, P, c)
    mag, negd = quant.decode_block(words, len(q), P, c)
    low = quant.lowest_planes(len(q), P, c)
    assert mag == [(qi >> p) << p for qi, p in zip(q, low)]
    # signs come back for significant coefficients only
    assert negd == [neg[i] and mag[i] != 0 for i in range(len(q))]


@pytest.mark.parametrize("m,k", [(1.0, 63), (0.75, 64), (0.5, 64), (0.125, 66), (3.0, 62),
                                 (2.0 ** -70, 133), (1.5 * 2.0 ** 100, -37)])
def test_scale_exponent_closed_form(m, k):
    v = np.array([0.0, -m, m / 3.0])
    assert quant.scale_exponent(v) == k
    assert 2 ** 63 <= math.ldexp(m, k) < 2 ** 64


def test_scale_of_zero_core():
    assert quant.scale_exponent(np.zeros(5)) is None
    k, q, neg = quant.quantize(np.zeros(5))
    assert k is None and q == [0] * 5


@pytest.mark.parametrize("p", [1, 2, 3, 5, 9])
def test_dequantization_correction_closed_form(p):
    m = 1 << p
    for hi in (1, 5, 1 << 20):
        base = hi << p
        total = sum(quant.err(base + x, p) for x in range(m))
        assert total == m * (m * m + 2) // 12
        uncorrected = sum(x * x for x in range(m))
        assert uncorrected == m * (m - 1) * (2 * m - 1) // 6
        if p >= 2:  # (for m = 2 both happen to give 1)
            assert uncorrected != total
    # every bit known: exact; nothing known: zero
    assert quant.err(12345, 0) == 0
    assert quant.decoded(12345, 64) == 0
    # no one-bit known yet: decodes to zero, not to the middle of [0, 2^p)
    assert quant.decoded(7, 3) == 0 and quant.err(7, 3) == 49


def _walk_error(values, k, q, neg, P, c):
    """Error of the walk stopped at (P, c), summed directly from the values
    decoded out of the stream of that breakpoint (float64, scaled units)."""
    words = quant.encode_block(q, neg, P, c)
    mag, negd = quant.decode_block(words, len(q), P, c)
    low = quant.lowest_planes(len(q), P, c)
    tot = 0.0
    for i in range(len(q)):
        d = 0.0
        if mag[i]:
            d = float(mag[i]) + (2.0 ** (low[i] - 1) if low[i] >= 1 else 0.0)
        tot += (float(q[i]) - d) ** 2
    return tot


@pytest.mark.parametrize("seed", range(6))
def test_breakpoint_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 9))
    values = rng.standard_normal(n) * np.logspace(0, -3, n)
    k, q, neg = quant.quantize(values)
    # every stop of the walk in order, down to plane 44 (errors by brute force)
    stops = [(64, 0, _walk_error(values, k, q, neg, 64, 0))]
    for p in range(63, 43, -1):
        for c in range(1, n + 1):
            stops.append((p, c, _walk_error(values, k, q, neg, p, c)))
    init = stops[0][2]
    for frac in (0.5, 1e-2, 1e-4, 1e-6, 3e-8, 1e-9):
        t_units = init * frac
        # keep clear of ties between the target and a stop's error
        if any(abs(e - t_units) <= 1e-9 * t_units for _, _, e in stops):
            continue
        exp = None
        for P in range(63, 43, -1):
            plane = [s for s in stops if s[0] == P]
            if plane[-1][2] <= t_units:
                exp = next((s[0], s[1]) for s in plane if s[2] <= t_units)
                break
        assert exp is not None
        got = quant.breakpoint(q, math.ldexp(t_units, -2 * k), k)
        assert got == exp, (seed, frac, got, exp)


def test_breakpoint_degenerate_targets():
    rng = np.random.default_rng(3)
    v = rng.standard_normal(17)
    k, q, neg = quant.quantize(v)
    init = float(sum(qi * qi for qi in q))
    assert quant.breakpoint(q, math.ldexp(init * 1.01, -2 * k), k) == (64, 0)
    assert quant.breakpoint(q, -1.0, k) == (0, 17)
    words = quant.encode(v, -1.0, 8)
    out = quant.dequantize(words)
    # every bit encoded: the core up to the rounding to integers (half a unit of 2^-k)
    assert np.max(np.abs(out - v)) <= math.ldexp(0.5, -k)
    words = quant.encode(v, 10.0 * float(np.sum(v * v)), 8)
    assert np.all(quant.dequantize(words) == 0.0)


def test_zero_core_stream():
    words = quant.encode(np.zeros((3, 4)), 1e-3, 5)
    h, mag, neg = quant.decode(words)
    assert h["k"] is None and h["P"] == 64 and mag == [0] * 12
    assert np.all(quant.dequantize(words) == 0.0)


@pytest.mark.parametrize("block_len", [1, 3, 7, 64])
def test_blocks_round_trip_and_error(block_len):
    rng = np.random.default_rng(11)
    v = rng.standard_normal((5, 4, 3)) * np.logspace(0, -4, 60).reshape(5, 4, 3)
    target = 1e-6 * float(np.sum(v * v))
    words = quant.encode(v, target, block_len)
    h, mag, neg = quant.decode(words)
    k, q, negq = quant.quantize(v)
    assert h["k"] == k and h["n"] == 60 and h["nblocks"] == -(-60 // block_len)
    assert (h["P"], h["count"]) == quant.breakpoint(q, target, k)
    low = quant.lowest_planes(60, h["P"], h["count"])
    assert mag == [(qi >> p) << p for qi, p in zip(q, low)]
    out = quant.dequantize(words)
    err = float(np.sum((out - v.ravel()) ** 2))
    # the tracked error reaches the target, measured on the decoded values
    assert err <= target * (1 + 1e-9)
    assert abs(err - quant.core_sse(v, words)) <= 1e-9 * target
    # the stream does not depend on how the core is cut into blocks
    assert quant.decode(quant.encode(v, target, 60))[1] == mag
