"""The lookup algorithm of section 6, step by step, in numpy -- TEST INFRASTRUCTURE ONLY.

This is a second, independent reference: where ``oracle.first_error`` is the
plain definition (a branchy walk), this module follows the paper's own method
so that its intermediate values can be pinned to the worked example of Table 9
and compared with the GPU validator's classification.

Steps (section 6):

* The input is consumed as a stream; the bytes before the start are taken as
  zero (ASCII NUL).
* Section 6.1: each byte is paired with its predecessor ``prev1``.  Three
  16-entry tables are indexed by the high nibble of ``prev1``, the low nibble
  of ``prev1`` and the high nibble of the byte, and the three results are ANDed.
  Bits 0-6 of the result mark an error; bit 7 marks two continuation bytes in a
  row.
* Section 6.2: a second continuation byte is required where the byte two
  before is a three- or four-byte lead (>= 0xE0) or the byte three before is a
  four-byte lead (>= 0xF0).  Any difference between that requirement and bit 7
  is an error.
* Section 6.3: at the end, the last byte must be < 0xC0, the second-to-last
  < 0xE0 and the third-to-last < 0xF0 (missing bytes count as zero).
* Section 6.4: a 64-byte block made only of ASCII skips the classification and
  only checks that the previous block did not end inside a character.

Table contents.  The paper prints the error patterns (Table 8) but not the
table bytes.  Each error bit is a product of one condition on each of the three
nibbles; a table entry is the OR of the bits whose condition holds for that
nibble.  Bits are labelled in the order implied by the values Table 9 prints
(which differs from the numbering in Table 8's first column):

  bit 0 too short   lead (C..F high nibble) followed by ASCII or another lead
  bit 1 too long    ASCII followed by a continuation
  bit 2 overlong 3  E0 followed by 80..9F
  bit 3 too large   F4..FF followed by 90..BF
  bit 4 surrogate   ED followed by A0..BF
  bit 5 overlong 2  C0 or C1 followed by a continuation
  bit 6 overlong 4  F0 (and F5..FF) followed by 80..8F
  bit 7 two continuations in a row (not an error by itself)

The "5+ byte" leads F8..FF and the too-large leads F5..F7 are caught by bits
3/6 when followed by a continuation and by bit 0 or the end check otherwise.
"""
from __future__ import annotations

import numpy as np

TOO_SHORT, TOO_LONG, OVERLONG_3, TOO_LARGE, SURROGATE, OVERLONG_2, OVERLONG_4, TWO_CONTS = (
    1 << k for k in range(8))

_ANY = set(range(16))
_ASCII = set(range(0, 8))
_CONT = set(range(8, 12))
_LEAD = set(range(12, 16))

# (bit, high nibble of prev1, low nibble of prev1, high nibble of the byte) -- Table 8.
PATTERNS = [
    (TOO_LONG, _ASCII, _ANY, _CONT),                    # 0xxxxxxx 10xxxxxx
    (TOO_SHORT, _LEAD, _ANY, _ASCII | _LEAD),           # 11xxxxxx followed by 0xxxxxxx or 11xxxxxx
    (OVERLONG_2, {0xC}, {0, 1}, _CONT),                 # 1100000x 10xxxxxx
    (SURROGATE, {0xE}, {0xD}, {0xA, 0xB}),              # 11101101 101xxxxx
    (OVERLONG_3, {0xE}, {0}, {0x8, 0x9}),               # 11100000 100xxxxx
    (OVERLONG_4, {0xF}, {0} | set(range(5, 16)), {0x8}),  # 11110000 or 11110101..11111111, then 1000xxxx
    (TOO_LARGE, {0xF}, set(range(4, 16)), {0x9, 0xA, 0xB}),  # 11110100..11111111, then 1001xxxx..1011xxxx
    (TWO_CONTS, _CONT, _ANY, _CONT),                    # 10xxxxxx 10xxxxxx
]


def derive_tables():
    """The three 16-entry tables (byte_1_high, byte_1_low, byte_2_high) from the patterns."""
    t1 = np.zeros(16, np.uint8)
    t2 = np.zeros(16, np.uint8)
    t3 = np.zeros(16, np.uint8)
    for bit, c1, c2, c3 in PATTERNS:
        for k in range(16):
            if k in c1:
                t1[k] |= bit
            if k in c2:
                t2[k] |= bit
            if k in c3:
                t3[k] |= bit
    return t1, t2, t3


BYTE_1_HIGH, BYTE_1_LOW, BYTE_2_HIGH = derive_tables()


def _shift(b: np.ndarray, k: int) -> np.ndarray:
    """b shifted right by k positions along the last axis, zeros shifted in (the zero start state)."""
    out = np.zeros_like(b)
    if k < b.shape[-1]:
        out[..., k:] = b[..., :-k] if k else b
    return out


def classify(b: np.ndarray):
    """Section 6.1 for every position; returns (prev1, byte_1_high, byte_1_low, byte_2_high, AND)."""
    b = np.asarray(b, dtype=np.uint8)
    prev1 = _shift(b, 1)
    r1 = BYTE_1_HIGH[prev1 >> 4]
    r2 = BYTE_1_LOW[prev1 & 0x0F]
    r3 = BYTE_2_HIGH[b >> 4]
    return prev1, r1, r2, r3, (r1 & r2 & r3)


def must_be_2_3_continuation(b: np.ndarray) -> np.ndarray:
    """Section 6.2: 0x80 where a second continuation is required, else 0."""
    b = np.asarray(b, dtype=np.uint8)
    req = (_shift(b, 2) >= 0xE0) | (_shift(b, 3) >= 0xF0)
    return np.where(req, 0x80, 0).astype(np.uint8)


def position_errors(b: np.ndarray) -> np.ndarray:
    """Per-position error bytes (sections 6.1-6.2), with one extra virtual position at the end.

    The last entry is the section 6.3 end check, written as the same test on a
    virtual zero byte after the input.
    """
    b = np.asarray(b, dtype=np.uint8)
    padded = np.concatenate([b, np.zeros(b.shape[:-1] + (1,), np.uint8)], axis=-1)
    sc = classify(padded)[4]
    return sc ^ must_be_2_3_continuation(padded)


def is_incomplete(last3: np.ndarray) -> np.ndarray:
    """Section 6.3 on the last three bytes [b[n-3], b[n-2], b[n-1]] (zero where missing)."""
    last3 = np.asarray(last3, dtype=np.uint8)
    return (last3[..., 2] >= 0xC0) | (last3[..., 1] >= 0xE0) | (last3[..., 0] >= 0xF0)


def validate(b) -> bool:
    """The lookup validator over one buffer, 64-byte blocks with the ASCII path of section 6.4."""
    b = np.frombuffer(bytes(b), np.uint8) if isinstance(b, (bytes, bytearray)) else np.asarray(b, np.uint8)
    error = 0
    prev_incomplete = False
    prev_block = np.zeros(64, np.uint8)
    n = b.size
    for start in range(0, n, 64):
        block = np.zeros(64, np.uint8)             # a short last block is padded with ASCII zeros
        block[: min(64, n - start)] = b[start:start + 64]
        if not np.any(block >= 0x80):
            error |= int(prev_incomplete)
        else:
            both = np.concatenate([prev_block, block])
            sc = classify(both)[4][64:]
            err = sc ^ must_be_2_3_continuation(both)[64:]
            error |= int(np.bitwise_or.reduce(err))
        last3 = block[61:64]
        prev_incomplete = bool(is_incomplete(last3))
        prev_block = block
    # Section 6.3.  When the last block was padded with zeros, the padding was
    # classified like input and prev_incomplete is False here; when it was
    # full, its last three bytes are the end of the stream.
    error |= int(prev_incomplete)
    return error == 0
