"""Plain CPU oracle of the core quantization and encoding (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  It
shares no code with the GPU path.  Everything here is exact: the quantized
magnitudes and every squared error are Python integers.

Paper passages followed (arXiv 2107.01384):
  * Section 3.3 (TTHRESH bit-plane truncation, Table 2): the core B is scaled by
    2^k with 2^63 <= 2^k |B|_max < 2^64 and rounded to integers.  The
    magnitudes of the lexicographically vectorised core form a bit matrix, one
    row per coefficient, whose columns (bit planes) are walked from the most
    significant one, bit by bit; the error of encoding every bit so far is
    tracked, and the walk ends at the breakpoint where the target is reached.
    A coefficient with an encoded one-bit is significant.  Its zeros before
    and including its first one are leading bits, run-length coded per plane;
    its later bits (trailing bits) and the signs of significant coefficients
    are stored raw.  Insignificant coefficients decode to zero, without sign.
  * Section 4.2 (parallel quantization and encoding): the vectorised core is
    cut into blocks of equal length; each plane is processed in full and the
    error checked at the end of the plane; only the plane in which the target
    is reached is walked again with error checks, and each block keeps its own
    breakpoint.  Blocks are encoded independently and stored with their sizes.
  * Section 4.3 (dequantization correction): a magnitude known down to plane
    p decodes to its known bits plus 2^(p-1), the middle of the interval the
    unknown bits leave, and the error tracking uses these decoded values.
  * Supplement S.5 (precise error control): the rounding of a floating-point
    running error, which the supplement guards against, does not arise here:
    the tracked error is an exact integer.

Readings where the paper is silent (listed in the design doc):
  * rounding to integers is to nearest, ties to even;
  * with every bit known (p = 0) the decoded value is the integer itself;
  * the breakpoint: plane P is the first plane (from the top) at whose end the
    tracked error is at or below the target; inside P, the first position at
    which the running error is at or below the target.  Per-block breakpoints
    follow from that position (blocks before it encode plane P in full, the
    block holding it up to it, later blocks not at all): the paper's threads
    racing on plane P, in the limit of instant synchronisation;
  * the error is tracked in units of the scaled core (SSE * 2^(2k)) and
    compared exactly with the target;
  * an all-zero core has no scale (k is stored as KZERO) and encodes nothing;
    a target at or above the error of encoding nothing encodes nothing
    (P = 64); a negative target encodes every bit;
  * the stream layout is this library's own (the paper's format is not given):
    runs as LEB128 varints, sign and trailing bits packed least significant bit
    first into 32-bit words; no entropy coder (supplement S.6) is applied.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import List, Optional, Sequence, Tuple

import numpy as np

PLANES = 64
KZERO = -(2 ** 31)          # scale exponent stored for an all-zero core
MAGIC = 0x51435441          # 'ATCQ'
HEADER_WORDS = 10           # magic, k, P, block_len, n (2), count (2), nblocks (2)


# ---------------------------------------------------------------- scale, round
def scale_exponent(values) -> Optional[int]:
    """k with 2^63 <= 2^k max|b| < 2^64 (Section 3.3), None for an all-zero core."""
    m = float(np.max(np.abs(np.asarray(values, dtype=np.float64)))) if np.size(values) else 0.0
    if m == 0.0:
        return None
    _, e = math.frexp(m)     # m = f 2^e, 1/2 <= f < 1
    return 64 - e


def quantize(values) -> Tuple[Optional[int], List[int], List[bool]]:
    """(k, magnitudes, negative flags) of the lexicographically vectorised core:
    q_i = round(2^k |b_i|), ties to even (Section 3.3)."""
    v = np.asarray(values, dtype=np.float64).ravel()
    if not np.all(np.isfinite(v)):
        raise ValueError("core holds non-finite values")
    k = scale_exponent(v)
    if k is None:
        return None, [0] * v.size, [False] * v.size
    q = [int(round(math.ldexp(abs(float(b)), k))) for b in v]
    neg = [bool(b < 0.0) for b in v]
    return k, q, neg


# ---------------------------------------------------------------- decoding
def decoded(q: int, p: int) -> int:
    """Magnitude decoded from the bits of planes >= p (Section 4.3): zero while
    no one-bit is known, else the known bits plus 2^(p-1) (nothing added once
    every bit is known)."""
    if p >= PLANES:
        return 0
    hi = (q >> p) << p
    if hi == 0:
        return 0
    return hi + ((1 << (p - 1)) if p >= 1 else 0)


def err(q: int, p: int) -> int:
    """Squared error of one magnitude known down to plane p."""
    e = q - decoded(q, p)
    return e * e


def lowest_planes(n: int, P: int, count: int) -> List[int]:
    """Lowest encoded plane of every coefficient for the breakpoint (P, count):
    the first `count` coefficients down to P, the others down to P + 1."""
    return [P if i < count else P + 1 for i in range(n)]


def sse(q: Sequence[int], P: int, count: int) -> int:
    """Exact quantization error (scaled units) at the breakpoint (P, count)."""
    return sum(err(qi, p) for qi, p in zip(q, lowest_planes(len(q), P, count)))


def target_units(target_sse: float, k: Optional[int]) -> Fraction:
    """The target in the scaled units, exactly: target * 2^(2k)."""
    t = Fraction(target_sse)
    if k is None:
        return t
    return t * (Fraction(2) ** (2 * k))


# ---------------------------------------------------------------- breakpoint
def breakpoint(q: Sequence[int], target_sse: float, k: Optional[int]) -> Tuple[int, int]:
    """Breakpoint (P, count) of the bit-plane walk (Sections 3.3, 4.2, 4.3):
    planes 63 .. P+1 are encoded for every coefficient, plane P for the first
    `count` coefficients.  (64, 0) encodes nothing."""
    n = len(q)
    T = target_units(target_sse, k)
    s_prev = sum(qi * qi for qi in q)          # nothing encoded
    if s_prev <= T:
        return PLANES, 0
    for p in range(PLANES - 1, -1, -1):
        s_end = sum(err(qi, p) for qi in q)    # plane p processed in full
        if s_end <= T:
            run = s_prev                       # walk plane p again, bit by bit
            for j, qi in enumerate(q):
                run += err(qi, p) - err(qi, p + 1)
                if run <= T:
                    return p, j + 1
            raise AssertionError("plane end reached the target, its walk did not")
        s_prev = s_end
    return 0, n                                # target below zero: every bit


def block_counts(n: int, block_len: int, count: int) -> List[int]:
    """Coefficients of each block encoded on the breakpoint plane (Section 4.2)."""
    nb = (n + block_len - 1) // block_len
    out = []
    for b in range(nb):
        lo, hi = b * block_len, min(n, (b + 1) * block_len)
        out.append(min(max(count - lo, 0), hi - lo))
    return out


# ---------------------------------------------------------------- encoding
def _varint(v: int) -> List[int]:
    out = []
    while True:
        byte = v & 0x7F
        v >>= 7
        if v:
            out.append(byte | 0x80)
        else:
            out.append(byte)
            return out


def encode_block_fields(q: Sequence[int], neg: Sequence[bool], P: int, count: int):
    """Runs, sign bits and trailing bits of one block (Section 3.3): for each
    plane from 63 down to P (plane P only for the first `count` coefficients
    of the block), the leading bits of the coefficients not yet significant
    as zero-run lengths (the zeros before each one-bit, then the zeros after
    the last one; nothing for a plane without leading bits), the sign of each
    coefficient whose first one-bit this is, and the bits of the coefficients
    already significant."""
    runs: List[int] = []
    signs: List[int] = []
    trail: List[int] = []
    m = len(q)
    sig = [False] * m
    for p in range(PLANES - 1, P - 1, -1):
        upto = count if p == P else m
        zeros = 0
        any_leading = False
        for i in range(upto):
            bit = (q[i] >> p) & 1
            if sig[i]:
                trail.append(bit)
                continue
            any_leading = True
            if bit:
                runs.append(zeros)
                zeros = 0
                sig[i] = True
                signs.append(1 if neg[i] else 0)
            else:
                zeros += 1
        if any_leading:
            runs.append(zeros)
    return runs, signs, trail


def _pack_bits(bits: Sequence[int]) -> List[int]:
    words = [0] * ((len(bits) + 31) // 32)
    for i, b in enumerate(bits):
        if b:
            words[i >> 5] |= 1 << (i & 31)
    return words


def _pack_bytes(data: Sequence[int]) -> List[int]:
    words = [0] * ((len(data) + 3) // 4)
    for i, b in enumerate(data):
        words[i >> 2] |= b << (8 * (i & 3))
    return words


def encode_block(q, neg, P, count) -> List[int]:
    """One block as 32-bit words: [run bytes, sign bits, trailing bits], then
    the run bytes, the sign words and the trailing-bit words."""
    runs, signs, trail = encode_block_fields(q, neg, P, count)
    rb = [b for r in runs for b in _varint(r)]
    return [len(rb), len(signs), len(trail)] + _pack_bytes(rb) + _pack_bits(signs) + _pack_bits(trail)


def encode(values, target_sse: float, block_len: int) -> np.ndarray:
    """Quantize and encode a core (any shape, vectorised in C order) to the
    stream of Section 4.2: header, block sizes in words, blocks."""
    k, q, neg = quantize(values)
    n = len(q)
    if k is None:
        P, count = PLANES, 0
    else:
        P, count = breakpoint(q, target_sse, k)
    nb = (n + block_len - 1) // block_len
    counts = block_counts(n, block_len, count)
    blocks = []
    for b in range(nb):
        lo, hi = b * block_len, min(n, (b + 1) * block_len)
        blocks.append(encode_block(q[lo:hi], neg[lo:hi], P, counts[b]))
    head = [MAGIC, (k if k is not None else KZERO) & 0xFFFFFFFF, P, block_len,
            n & 0xFFFFFFFF, n >> 32, count & 0xFFFFFFFF, count >> 32, nb & 0xFFFFFFFF, nb >> 32]
    sizes = []
    for blk in blocks:
        sizes += [len(blk) & 0xFFFFFFFF, len(blk) >> 32]
    words = head + sizes + [w for blk in blocks for w in blk]
    return np.array(words, dtype=np.uint32)


# ---------------------------------------------------------------- decoding
def _header(words):
    w = [int(x) for x in words[:HEADER_WORDS]]
    if w[0] != MAGIC:
        raise ValueError("not an encoded core")
    k = w[1] - (1 << 32) if w[1] >= (1 << 31) else w[1]
    return {"k": None if k == KZERO else k, "P": w[2], "block_len": w[3], "n": w[4] | (w[5] << 32),
            "count": w[6] | (w[7] << 32), "nblocks": w[8] | (w[9] << 32)}


def decode_block(words: Sequence[int], m: int, P: int, count: int):
    """Known magnitude bits (bits of planes >= each coefficient's lowest
    encoded plane) and negative flags of one block."""
    nrb, nsb, ntb = int(words[0]), int(words[1]), int(words[2])
    pos = 3
    rb = []
    for i in range(nrb):
        rb.append((int(words[pos + (i >> 2)]) >> (8 * (i & 3))) & 0xFF)
    pos += (nrb + 3) // 4
    sign_bits = [(int(words[pos + (i >> 5)]) >> (i & 31)) & 1 for i in range(nsb)]
    pos += (nsb + 31) // 32
    trail_bits = [(int(words[pos + (i >> 5)]) >> (i & 31)) & 1 for i in range(ntb)]
    runs = []
    i = 0
    while i < len(rb):
        v, sh = 0, 0
        while True:
            b = rb[i]
            i += 1
            v |= (b & 0x7F) << sh
            sh += 7
            if not b & 0x80:
                break
        runs.append(v)
    mag = [0] * m
    neg = [False] * m
    sig = [False] * m
    ri = si = ti = 0
    for p in range(PLANES - 1, P - 1, -1):
        upto = count if p == P else m
        lead = [i for i in range(upto) if not sig[i]]
        for i in range(upto):
            if sig[i]:
                mag[i] |= trail_bits[ti] << p
                ti += 1
        if lead:
            at = 0
            while True:
                at += runs[ri]
                ri += 1
                if at == len(lead):
                    break
                c = lead[at]
                mag[c] |= 1 << p
                sig[c] = True
                neg[c] = bool(sign_bits[si])
                si += 1
                at += 1
    if ri != len(runs) or si != nsb or ti != ntb:
        raise ValueError("block holds more fields than its planes use")
    return mag, neg


def decode(words) -> Tuple[dict, List[int], List[bool]]:
    """Header, known magnitude bits and negative flags of every coefficient."""
    h = _header(words)
    n, L, nb = h["n"], h["block_len"], h["nblocks"]
    sizes = [int(words[HEADER_WORDS + 2 * b]) | (int(words[HEADER_WORDS + 2 * b + 1]) << 32) for b in range(nb)]
    pos = HEADER_WORDS + 2 * nb
    counts = block_counts(n, L, h["count"])
    mag, neg = [], []
    for b in range(nb):
        m = min(n, (b + 1) * L) - b * L
        mb, nbits = decode_block(words[pos: pos + sizes[b]], m, h["P"], counts[b])
        mag += mb
        neg += nbits
        pos += sizes[b]
    return h, mag, neg


def dequantize(words) -> np.ndarray:
    """Decoded core values (FP64, vectorised): sign * (known bits + 2^(p-1))
    * 2^-k with p each coefficient's lowest encoded plane (Section 4.3)."""
    h, mag, neg = decode(words)
    n = h["n"]
    out = np.zeros(n, dtype=np.float64)
    if h["k"] is None:
        return out
    planes = lowest_planes(n, h["P"], h["count"])
    for i in range(n):
        d = decoded(mag[i], planes[i])
        if d:
            v = math.ldexp(float(d), -h["k"])   # int -> double rounds to nearest even
            out[i] = -v if neg[i] else v
    return out


def core_sse(values, words) -> float:
    """Quantization error |B - B~|^2 in the core's units from the stream's
    breakpoint, exact up to the final rounding."""
    k, q, _ = quantize(values)
    h = _header(words)
    if k is None:
        return 0.0
    return float(Fraction(sse(q, h["P"], h["count"])) / (Fraction(2) ** (2 * k)))
