"""Pins for the branchy oracle against facts fixed by the paper and by mathematics.

None of these re-derive the oracle's own code: they use the closed-form counts
implied by Table 1, the paper's labelled examples, CPython's strict UTF-8
decoder, a decode/re-encode invariant, and sweeps of every code point.
"""
import os

import numpy as np
import pytest

import oracle
from conftest import read_labelled_vectors

# Table 1 (section 2): number of code points encoded with 1, 2, 3, 4 bytes.
# Three-byte: U+0800..D7FF and U+E000..FFFF; four-byte: U+10000..10FFFF.
C = {1: 0x80, 2: 0x800 - 0x80, 3: (0xD800 - 0x800) + (0x10000 - 0xE000), 4: 0x110000 - 0x10000}


def valid_count(n):
    """a(n) = number of valid strings of n bytes = sum_L C_L a(n-L)."""
    a = [1]
    for m in range(1, n + 1):
        a.append(sum(C[L] * a[m - L] for L in range(1, 5) if m - L >= 0))
    return a[n]


def bad_start_count(m):
    """z(m) = number of m-byte strings that do not begin with a whole valid character."""
    return 256 ** m - sum(C[L] * 256 ** (m - L) for L in range(1, 5) if L <= m)


def test_closed_form_constants():
    assert sum(C.values()) == 1_112_064           # Unicode scalar values
    assert [valid_count(n) for n in range(5)] == [1, 128, 18_304, 2_650_112, 383_270_912]


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_exhaustive_first_error_histogram(n):
    """Brute force over all 256**n strings: #first_err == k is a(k) z(n-k); #valid is a(n)."""
    hist = oracle.exhaustive_hist(n)
    expected = [valid_count(k) * bad_start_count(n - k) for k in range(n)] + [valid_count(n)]
    assert hist.tolist() == expected
    assert int(hist.sum()) == 256 ** n


def test_labelled_vectors():
    for b, exp, label, src in read_labelled_vectors():
        assert oracle.first_error(b) == exp, (b.hex(), label, src)


def _cpython_first_error(b: bytes) -> int:
    try:
        b.decode("utf-8", "strict")
        return -1
    except UnicodeDecodeError as e:
        return e.start


def test_cpython_agreement_all_short_strings():
    """CPython's strict decoder (a library routine) on every string of length <= 2."""
    bad = []
    for n in (1, 2):
        for v in range(256 ** n):
            b = v.to_bytes(n, "little")
            if oracle.first_error(b) != _cpython_first_error(b):
                bad.append(b)
    assert not bad, bad[:10]


BOUNDARY_ALPHABET = bytes([0x00, 0x41, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF, 0xE0,
                           0xE1, 0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xF7, 0xF8, 0xFF])


def _alphabet_strings(n):
    idx = np.indices((len(BOUNDARY_ALPHABET),) * n).reshape(n, -1).T
    alpha = np.frombuffer(BOUNDARY_ALPHABET, np.uint8)
    return alpha[idx]


@pytest.mark.parametrize("n", [3, 4])
def test_cpython_agreement_boundary_alphabet(n):
    """Every string of length n over the range endpoints of Table 1 and their neighbours."""
    strs = _alphabet_strings(n)
    offsets = np.arange(strs.shape[0] + 1, dtype=np.int64) * n
    flags, ferr = oracle.first_error_batch(strs.reshape(-1), offsets)
    expected = np.array([_cpython_first_error(bytes(s)) for s in strs], dtype=np.int64)
    assert np.array_equal(ferr, expected)
    assert np.array_equal(flags, (expected < 0).astype(np.uint8))


def test_result_ignores_bytes_past_the_end():
    """Only the n given bytes count: memory after them holds continuation bytes here."""
    strs = _alphabet_strings(3)
    for s in strs:
        b = bytes(s)
        padded = np.frombuffer(b + b"\x80\xbf\x80", np.uint8)
        assert oracle.first_error(padded[:3]) == _cpython_first_error(b)
        for n in (1, 2):
            assert oracle.first_error(padded[:n]) == _cpython_first_error(b[:n])


def test_cpython_agreement_random_mixtures():
    """Random byte strings biased toward UTF-8 structure, lengths 0..40."""
    rng = np.random.default_rng(1234)
    pool = np.frombuffer(BOUNDARY_ALPHABET + bytes(range(0x80, 0xC0)) + "aé中😀".encode(), np.uint8)
    for _ in range(20000):
        n = int(rng.integers(0, 41))
        b = bytes(pool[rng.integers(0, pool.size, n)]) if rng.random() < 0.7 else rng.bytes(n)
        assert oracle.first_error(b) == _cpython_first_error(b), b.hex()


def test_every_scalar_value_is_valid():
    """All 1,112,064 scalar values, each encoded alone (by CPython) and all concatenated."""
    cps = [c for c in range(0x110000) if not 0xD800 <= c <= 0xDFFF]
    enc = [chr(c).encode("utf-8") for c in cps]
    lens = np.array([len(e) for e in enc], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(lens)])
    data = np.frombuffer(b"".join(enc), np.uint8)
    flags, ferr = oracle.first_error_batch(data, offsets)
    assert flags.all() and (ferr == -1).all()
    assert oracle.first_error(data) == -1
    assert np.bincount(lens)[1:].tolist() == [C[1], C[2], C[3], C[4]]


def _encode_forced(cp, length):
    """Encode cp with a fixed byte length (overlong when the length exceeds the shortest)."""
    if length == 2:
        return bytes([0xC0 | (cp >> 6), 0x80 | (cp & 0x3F)])
    if length == 3:
        return bytes([0xE0 | (cp >> 12), 0x80 | ((cp >> 6) & 0x3F), 0x80 | (cp & 0x3F)])
    return bytes([0xF0 | (cp >> 18), 0x80 | ((cp >> 12) & 0x3F), 0x80 | ((cp >> 6) & 0x3F), 0x80 | (cp & 0x3F)])


def _first_errors(seqs):
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(lens)])
    data = np.frombuffer(b"".join(seqs), np.uint8)
    return oracle.first_error_batch(data, offsets)[1]


def test_invalid_forms_rejected_at_offset_zero():
    """Surrogates (rule f), every overlong form (rule d), and U+110000..1FFFFF (rule e)."""
    surrogates = [_encode_forced(c, 3) for c in range(0xD800, 0xE000)]
    over2 = [_encode_forced(c, 2) for c in range(0x80)]
    over3 = [_encode_forced(c, 3) for c in range(0x800)]
    over4 = [_encode_forced(c, 4) for c in range(0x10000)]
    large = [_encode_forced(c, 4) for c in range(0x110000, 0x200000)]
    for name, seqs, count in [("surrogate", surrogates, 2048), ("overlong2", over2, 128),
                              ("overlong3", over3, 2048), ("overlong4", over4, 65536),
                              ("too_large", large, 0x200000 - 0x110000)]:
        assert len(seqs) == count
        ferr = _first_errors(seqs)
        assert (ferr == 0).all(), name
    # the same forms after a valid prefix: the offset moves with the prefix
    pre = "aé中".encode()
    ferr = _first_errors([pre + s for s in surrogates[:64] + over4[:64] + large[:64]])
    assert (ferr == len(pre)).all()


def _decode_permissive(b):
    """Decode any 1..4-byte bit pattern (no range checks); None if the structure is broken."""
    out, i, n = [], 0, len(b)
    while i < n:
        c = b[i]
        if c < 0x80:
            L, v = 1, c
        elif 0xC0 <= c < 0xE0:
            L, v = 2, c & 0x1F
        elif 0xE0 <= c < 0xF0:
            L, v = 3, c & 0x0F
        elif 0xF0 <= c < 0xF8:
            L, v = 4, c & 0x07
        else:
            return None
        if i + L > n:
            return None
        for k in range(1, L):
            if b[i + k] & 0xC0 != 0x80:
                return None
            v = (v << 6) | (b[i + k] & 0x3F)
        out.append(v)
        i += L
    return out


def _encode_shortest(cps):
    out = bytearray()
    for v in cps:
        if v < 0x80:
            out.append(v)
        elif v < 0x800:
            out += _encode_forced(v, 2)
        elif v < 0x10000:
            out += _encode_forced(v, 3)
        else:
            out += _encode_forced(v, 4)
    return bytes(out)


def _invariant_valid(b):
    """Valid iff the structural decoding gives non-surrogate scalars <= U+10FFFF that re-encode to b."""
    cps = _decode_permissive(b)
    if cps is None:
        return False
    if any(v > 0x10FFFF or 0xD800 <= v <= 0xDFFF for v in cps):
        return False
    return _encode_shortest(cps) == b


def test_decode_reencode_invariant():
    rng = np.random.default_rng(99)
    cases = [v.to_bytes(2, "little") for v in range(65536)]
    alpha = _alphabet_strings(3)
    cases += [bytes(s) for s in alpha]
    for _ in range(5000):
        n = int(rng.integers(1, 24))
        cases.append(rng.bytes(n))
    for b in cases:
        assert (oracle.first_error(b) < 0) == _invariant_valid(b), b.hex()


def test_first_error_is_longest_valid_prefix():
    """first_err = k means b[:k] is valid and no longer prefix ending on a character is."""
    rng = np.random.default_rng(5)
    for _ in range(3000):
        b = rng.bytes(int(rng.integers(1, 16))) if rng.random() < 0.5 else \
            ("aé中😀"[rng.integers(0, 4)] * 3).encode()[: int(rng.integers(1, 13))] + rng.bytes(2)
        k = oracle.first_error(b)
        if k < 0:
            assert _invariant_valid(b)
            continue
        assert oracle.first_error(b[:k]) == -1
        assert all(not _invariant_valid(b[:m]) for m in range(k + 1, len(b) + 1))


def test_batch_matches_single_and_relative_offsets():
    rng = np.random.default_rng(7)
    strs = [rng.bytes(int(rng.integers(0, 12))) for _ in range(500)] + [b"", "é".encode(), b"\x80"]
    lens = np.array([len(s) for s in strs], dtype=np.int64)
    base = 5
    offsets = base + np.concatenate([[0], np.cumsum(lens)])
    data = np.frombuffer(b"\xff" * base + b"".join(strs), np.uint8)
    flags, ferr = oracle.first_error_batch(data, offsets, nthreads=3)
    for k, s in enumerate(strs):
        assert ferr[k] == oracle.first_error(s)
        assert flags[k] == (ferr[k] < 0)


# ---- error classes (section 3 rules a..f) ------------------------------------------------


def _golden_classes():
    rows = []
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "error_classes.txt")
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        hx, off, cls, label, src = [x.strip() for x in line.split("|")]
        rows.append((bytes.fromhex(hx), int(off), int(cls), label))
    return rows


def test_error_class_of_the_papers_examples():
    for b, off, cls, label in _golden_classes():
        assert oracle.first_error(b) == off, label
        assert oracle.error_class(b) == cls, label


def _encode(cp: int, nbytes: int) -> bytes:
    """cp in nbytes UTF-8 form, whatever its value (overlong, surrogate or too large allowed)."""
    if nbytes == 1:
        return bytes([cp])
    lead = (0xFF << (8 - nbytes)) & 0xFF
    out = [0x80 | ((cp >> (6 * k)) & 0x3F) for k in range(nbytes - 1)][::-1]
    return bytes([lead | (cp >> (6 * (nbytes - 1)))] + out)


def test_error_class_by_code_point():
    """Every surrogate, overlong and too-large form, built by an encoder, gets its rule."""
    for cp in range(0xD800, 0xE000):
        assert oracle.error_class(_encode(cp, 3)) == 6
    for cp in range(0, 0x80):
        assert oracle.error_class(_encode(cp, 2)) == 4
    for cp in range(0, 0x800, 7):
        assert oracle.error_class(_encode(cp, 3)) == 4
    for cp in range(0, 0x10000, 97):
        assert oracle.error_class(_encode(cp, 4)) == 4
    for cp in range(0x110000, 0x200000, 1009):
        assert oracle.error_class(_encode(cp, 4)) == 5
    for cp in (0x80, 0x7FF, 0x800, 0xFFFF, 0x10000, 0x10FFFF, 0xE000, 0xD7FF):
        n = 1 if cp < 0x80 else 2 if cp < 0x800 else 3 if cp < 0x10000 else 4
        b = _encode(cp, n)
        assert oracle.error_class(b) == 0
        for cut in range(1, n):                   # truncated: too short
            assert oracle.error_class(b[:cut]) == 2
        assert oracle.error_class(b[:1] + b"A" + b[2:]) == 2 if n > 1 else True
    for lead in range(0x80, 0xC0):                # stray continuation: too long
        assert oracle.error_class(bytes([lead, 0x41])) == 3
    for lead in range(0xF8, 0x100):               # five or more header bits
        assert oracle.error_class(bytes([lead]) + b"\x80" * 5) == 1


def test_error_class_agrees_with_cpython_reasons():
    """CPython's decoder reason narrows the class: start byte, continuation byte or end of data.

    CPython rejects C0, C1 and F5..F7 as start bytes outright; by the section 3
    rules they are too short when their continuations are missing, else overlong
    (C0, C1) or too large (F5..F7).
    """
    cont = {2, 4, 5, 6}            # a bad second/third/fourth byte
    alpha = [0x00, 0x41, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF, 0xE0, 0xE1, 0xEC,
             0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xF7, 0xF8, 0xFF]
    import itertools
    for n in (1, 2, 3, 4):
        for t in itertools.product(alpha, repeat=n):
            b = bytes(t)
            s = oracle.first_error(b)
            cls = oracle.error_class(b, s)
            try:
                b.decode("utf-8")
                assert s == -1 and cls == 0
                continue
            except UnicodeDecodeError as e:
                assert e.start == s and cls != 0
                if e.reason == "invalid start byte":
                    lead = b[s]
                    want = {3} if 0x80 <= lead <= 0xBF else {1} if lead >= 0xF8 else \
                        {2, 4} if lead in (0xC0, 0xC1) else {2, 5}
                    assert cls in want, (b.hex(), cls)
                elif e.reason == "invalid continuation byte":
                    assert cls in cont, (b.hex(), cls)
                else:
                    assert e.reason == "unexpected end of data" and cls == 2, (b.hex(), cls)


def _golden_class_batch():
    """A CSR batch of the golden rows, with known offsets and classes.

    offsets[0] is not 0 (padding bytes FF, themselves a class-1 error, come first),
    empty and valid strings sit between the rows, and each truncated row is followed by
    a string that starts with continuation bytes, so reading past a string's end would
    complete the truncated character and change its class.
    """
    # the golden rows, and characters cut by the string end (section 3 rule b: too short)
    rows = _golden_classes() + [(b"\xf0\x9f\x98", 0, 2, "cut"), (b"A\xe9\x8f", 1, 2, "cut"), (b"\xc3", 0, 2, "cut")]
    strs, ferr, cls = [], [], []
    for i, (b, off, c, _) in enumerate(rows):
        strs += [b, b"", "é".encode()] if i % 2 else [b]
        ferr += [off, -1, -1] if i % 2 else [off]
        cls += [c, 0, 0] if i % 2 else [c]
        if c == 2:
            strs.append(b"\x80\xbf\x80\x41")
            ferr.append(0)
            cls.append(3)
    pad = b"\xff" * 7
    data = np.frombuffer(pad + b"".join(strs), np.uint8)
    lens = np.array([len(s) for s in strs], np.int64)
    offsets = len(pad) + np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return data, offsets, np.array(ferr, np.int64), np.array(cls, np.uint8)


def test_error_class_batch_golden():
    """The batch form slices each string itself: classes of the golden rows at their offsets."""
    data, offsets, ferr, cls = _golden_class_batch()
    assert sorted(set(cls.tolist())) == [0, 1, 2, 3, 4, 5, 6]
    assert offsets[0] != 0 and (np.diff(offsets) == 0).any()
    got = oracle.error_class_batch(data, offsets, ferr)
    assert got.tolist() == cls.tolist()
    # the offsets the classes are computed from are the first-error offsets the oracle reports
    flags, fe = oracle.first_error_batch(data, offsets)
    assert fe.tolist() == ferr.tolist() and flags.tolist() == (ferr < 0).astype(np.uint8).tolist()
    # a batch of nothing but empty strings is all valid
    e = oracle.error_class_batch(data, np.full(5, 3, np.int64), np.full(4, -1, np.int64))
    assert e.tolist() == [0, 0, 0, 0]
