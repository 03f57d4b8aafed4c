"""GPU parity: the HIP validator against the oracle, element by element (needs an MI355X).

Bit-exact comparison of flags and first-error offsets (integer results, no
tolerance).  Inputs are seeded and synthetic (paper_2010_03090_amd.synth).
"""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import lookup_model as lm
from conftest import read_golden_rows, read_labelled_vectors
from paper_2010_03090_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(params=[4, 8], ids=["tile4k", "tile8k"])
def batch_tile(u8, request):
    """Run a batch test with 4 KiB and with 8 KiB wave tiles (the batch kernel's tile setting)."""
    old = u8.get_config()
    u8.set_config(batch_unroll=request.param)
    say(f"batch tile {request.param} KiB")
    yield request.param
    u8.set_config(**old)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))  # the repository root

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def u8():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_03090_amd as u8
    u8.load()
    return u8


def dev(a):
    a = np.ascontiguousarray(a)
    if not a.flags.writeable:
        a = a.copy()
    return torch.from_numpy(a).cuda()


def test_table9_on_gpu(u8):
    say("case: table9")
    rows = read_golden_rows("table9_classification.txt")
    b = np.array(rows["input"], np.uint8)
    sc, err = u8.classify(dev(b))
    sc = sc.cpu().numpy()
    assert sc[: b.size].tolist() == rows["and"]
    assert not err.cpu().numpy().any()


def test_classification_matches_lookup_model(u8):
    """Per-position classification and error bytes equal the section 6 model on varied buffers."""
    bufs = []
    pairs = np.stack(np.meshgrid(np.arange(256), np.arange(256), indexing="ij"), -1).reshape(-1).astype(np.uint8)
    bufs.append(pairs)                                           # every (prev, byte) pair
    alpha = np.array([0x00, 0x41, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF, 0xE0,
                      0xE1, 0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xF7, 0xF8, 0xFF], np.uint8)
    bufs.append(alpha[np.indices((27,) * 4).reshape(4, -1).T].reshape(-1))   # all 4-sequences of the alphabet
    rng = np.random.default_rng(11)
    bufs.append(rng.integers(0, 256, 100_003, dtype=np.uint8))
    for v in ("mixed", "cjk", "emoji"):
        b = synth.text(50_001, v, 3)
        synth.inject_random(b, 5)
        bufs.append(b)
    for i, b in enumerate(bufs):
        say(f"case: classify buffer {i} len {b.size}")
        sc, err = u8.classify(dev(b))
        padded = np.concatenate([b, [0]]).astype(np.uint8)
        exp_sc = lm.classify(padded)[4]
        exp_err = exp_sc ^ lm.must_be_2_3_continuation(padded)
        assert np.array_equal(sc.cpu().numpy(), exp_sc), i
        assert np.array_equal(err.cpu().numpy(), exp_err), i


def test_labelled_vectors_single(u8):
    for b, exp, label, src in read_labelled_vectors():
        say(f"case: labelled {b.hex()} {label}")
        assert u8.first_error(dev(np.frombuffer(b, np.uint8))) == exp, (label, src)


def test_empty_and_tiny(u8):
    say("case: empty")
    assert u8.first_error(torch.empty(0, dtype=torch.uint8, device="cuda")) == -1
    for v in range(256):
        b = np.array([v], np.uint8)
        assert u8.first_error(dev(b)) == oracle.first_error(b)


def test_single_error_at_every_offset_and_alignment(u8):
    """One injected error at each offset around chunk, lane, slab and tile boundaries, unaligned bases."""
    rng = np.random.default_rng(21)
    base_len = 9000
    big = dev(np.zeros(base_len + 64, np.uint8))
    positions = sorted(set(list(range(0, 80)) + [k + d for k in (1024, 2048, 3072, 4096, 8192 - 16)
                                                 for d in range(-6, 7)] + list(rng.integers(0, base_len, 200))))
    checked = 0
    for variant in ("mixed", "latin", "ascii", "emoji", "cjk"):
        clean = synth.text(base_len, variant, 7)
        for pos in positions:
            for cls in range(7):
                if (pos + cls) % 3:
                    continue
                buf = clean.copy()
                if cls == 6:
                    cut = int(pos) % 40 + 1
                    buf = buf[: max(1, base_len - cut)].copy()
                    s = synth.inject(buf, 0, 6, pos)
                else:
                    s = synth.inject(buf, int(pos), cls, int(pos) * 7 + cls)
                if s < 0:
                    continue
                shift = int(pos) % 16
                big[shift: shift + buf.size].copy_(torch.from_numpy(buf))
                view = big[shift: shift + buf.size]
                got = u8.first_error(view)
                exp = oracle.first_error(buf)
                assert exp == s
                assert got == exp, (variant, int(pos), cls, shift, got, exp)
                checked += 1
    say(f"checked {checked} single-error buffers")


def test_two_byte_text_with_longer_characters_at_chunk_edges(u8):
    """Text of 1- and 2-byte characters takes a short form of the checks per tile; a byte
    >= 0xE0 in a chunk or in the three bytes before it must send the tile to the full
    checks.  A 3- or 4-byte character (valid, or cut short) is placed across each chunk,
    slab and tile edge of 2-byte text, at every split."""
    n = 40 * 1024
    base = np.full(n, 0x61, np.uint8)
    base[5::37], base[6::37] = 0xC3, 0xA9          # U+00E9 every 37 bytes
    edges = [16 * k for k in range(1, 6)] + [1024, 2048, 3072, 4096, 8192, 12288, 20480 + 16]
    chars = [np.array(c, np.uint8) for c in ((0xE2, 0x82, 0xAC), (0xF0, 0x9F, 0x98, 0x80), (0xE2, 0x82),
                                             (0xF0, 0x9F, 0x98), (0xED, 0xA0, 0x80))]
    big = dev(np.zeros(n + 16, np.uint8))
    valid = 0
    for e in edges:
        for ch in chars:
            for k in range(1, ch.size + 1):
                buf = base.copy()
                buf[e - k: e - k + ch.size] = ch
                for shift in (0, 5):
                    big[shift: shift + n].copy_(torch.from_numpy(buf))
                    got = u8.first_error(big[shift: shift + n])
                    exp = oracle.first_error(buf)
                    assert got == exp, (e, ch.tolist(), k, shift, got, exp)
                valid += exp == -1
    assert valid > 20
    say(f"checked {len(edges) * sum(c.size for c in chars) * 2} buffers, {valid} valid")


def test_three_byte_text_with_other_characters_at_chunk_edges(u8):
    """Text of characters of at most three bytes first takes a comparison form of the
    checks per tile; a byte >= 0xF0 in a chunk or in the three bytes before it, or an
    error, must send the tile to the table form.  4-byte characters (valid, cut short, too
    large, overlong), bytes F5..FF and the 3-byte special cases are placed across each
    chunk, slab and tile edge of CJK-like text, at every split, at two alignments and
    with the section 6.4 test on and off."""
    n = 40 * 1024
    base = np.tile(np.array([0xE4, 0xB8, 0xAD, 0xE6, 0x96, 0x87, 0x41], np.uint8), n // 7 + 1)[:n]
    base[-(n % 7 or 7):] = 0x41
    edges = [16 * k for k in range(1, 6)] + [1024, 2048, 3072, 4096, 8192, 12288, 20480 + 16]
    chars = [np.array(c, np.uint8) for c in ((0xF0, 0x9F, 0x98, 0x80), (0xF4, 0x8F, 0xBF, 0xBF), (0xF0, 0x9F, 0x98),
                                             (0xF4, 0x90, 0x80, 0x80), (0xF0, 0x80, 0x80, 0x80), (0xF5, 0x80, 0x80),
                                             (0xFF,), (0xED, 0xA0, 0x80), (0xE0, 0x80, 0x80), (0xE0, 0xA0, 0x80),
                                             (0xED, 0x9F, 0xBF), (0xC0, 0x80), (0x80,), (0xE4, 0xB8))]
    big = dev(np.zeros(n + 16, np.uint8))
    old = u8.get_config()
    valid = checked = 0
    try:
        for ascii_ in (0, 1):
            u8.set_config(ascii=ascii_)
            for e in edges:
                for ch in chars:
                    for k in range(1, ch.size + 1):
                        buf = base.copy()
                        buf[e - k: e - k + ch.size] = ch
                        exp = oracle.first_error(buf)
                        for shift in (0, 5):
                            big[shift: shift + n].copy_(torch.from_numpy(buf))
                            got = u8.first_error(big[shift: shift + n])
                            assert got == exp, (ascii_, e, ch.tolist(), k, shift, got, exp)
                            checked += 1
                        valid += exp == -1
    finally:
        u8.set_config(**old)
    assert valid > 20
    say(f"checked {checked} buffers, {valid // 2} valid")


def test_sizes_and_alignments_valid_and_random(u8):
    big = dev(np.zeros(70_000, np.uint8))
    sizes = list(range(0, 70)) + [1023, 1024, 1025, 4095, 4096, 4097, 16384 + 5, 65536 - 1, 65536 + 3]
    for n in sizes:
        for shift in (0, 1, 7, 15):
            for variant in ("mixed", "random"):
                b = synth.text(n, variant, n * 31 + shift)
                big[shift: shift + n].copy_(torch.from_numpy(b))
                got = u8.first_error(big[shift: shift + n])
                assert got == oracle.first_error(b), (n, shift, variant)


def test_config0_mixed_1mib_and_64_corrupted_copies(u8):
    say("case: config0")
    clean, copies = synth.single_buffer_with_errors(1 << 20, "mixed", 0, 64)
    assert u8.first_error(dev(clean)) == -1 == oracle.first_error(clean)
    for buf, s, cls in copies:
        assert u8.first_error(dev(buf)) == s == oracle.first_error(buf), cls


@pytest.mark.parametrize("variant", ["ascii", "latin", "cjk", "emoji", "random"])
def test_config1_full_size_1gib(u8, variant):
    """1 GiB buffers, plus the copy with an error in the last 4 bytes, at the launch shape the
    benchmark times (unroll 4, 20 waves per CU) with the ASCII skip off and on, and at the
    library's default configuration."""
    n = 1 << 30
    seed = {"ascii": 1, "latin": 2, "cjk": 3, "emoji": 4, "random": 5}[variant]
    b = synth.text(n, variant, seed)
    t = dev(b)
    exp = oracle.first_error(b)
    if variant != "random":
        assert exp == -1
        tail, s, cls = synth.tail_error_copy(b[-64:], seed)
        t_err = t.clone()
        t_err[-64:].copy_(torch.from_numpy(tail))
    old = u8.get_config()
    try:
        for cfg in (dict(unroll=4, waves_per_cu=20, ascii=0), dict(unroll=4, waves_per_cu=20, ascii=1), old):
            say(f"case: config1 {variant} {cfg}")
            u8.set_config(**cfg)
            assert u8.first_error(t) == exp
            if variant != "random":
                assert u8.first_error(t_err) == s + n - 64
    finally:
        u8.set_config(**old)
    del t
    torch.cuda.empty_cache()


def test_batch_exhaustive_short_strings(u8, batch_tile):
    """Every string of length 0..3 in one CSR batch (each at many alignments)."""
    say("case: batch exhaustive <= 3")
    parts, lens = [], []
    for n in range(0, 4):
        if n == 0:
            parts.append(np.zeros(0, np.uint8)); lens += [0] * 3
            continue
        v = np.arange(256 ** n, dtype=np.uint32)
        strs = np.stack([(v >> (8 * k)) & 0xFF for k in range(n)], 1).astype(np.uint8)
        parts.append(strs.reshape(-1))
        lens += [n] * strs.shape[0]
    data = np.concatenate(parts)
    lens = np.array(lens, np.int64)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    flags, ferr = u8.validate_batch(dev(data), dev(offsets))
    torch.cuda.synchronize()
    assert np.array_equal(ferr.cpu().numpy(), e_o)
    assert np.array_equal(flags.cpu().numpy(), f_o)


def test_batch_semantics(u8, batch_tile):
    """offsets[0] != 0, empty strings, strings across tiles, and each string alone == in the batch."""
    rng = np.random.default_rng(5)
    lens = np.concatenate([rng.integers(0, 9, 400), rng.integers(0, 5000, 40), [0, 0, 1, 0, 70000, 0]])
    rng.shuffle(lens)
    for base in (0, 3, 4096 + 13):
        say(f"case: batch semantics base {base}")
        data, offsets, expected = synth.batch_from_lengths(lens, "mixed", 9 + base, err_frac=0.3, base=base)
        f_o, e_o = oracle.first_error_batch(data, offsets)
        assert np.array_equal(e_o[expected >= 0], expected[expected >= 0])
        td = dev(data)
        flags, ferr = u8.validate_batch(td, dev(offsets))
        torch.cuda.synchronize()
        ferr = ferr.cpu().numpy()
        assert np.array_equal(ferr, e_o)
        assert np.array_equal(flags.cpu().numpy(), f_o)
        for k in rng.choice(lens.size, 50, replace=False):
            s, e = int(offsets[k]), int(offsets[k + 1])
            alone = u8.first_error(td[s:e]) if e > s else -1
            assert alone == ferr[k]


def test_batch_random_bytes_and_tiny_strings(u8, batch_tile):
    rng = np.random.default_rng(8)
    lens = rng.integers(0, 6, 200_000)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    data = rng.integers(0, 256, int(offsets[-1]), dtype=np.uint8)
    say("case: batch random tiny")
    f_o, e_o = oracle.first_error_batch(data, offsets)
    flags, ferr = u8.validate_batch(dev(data), dev(offsets))
    torch.cuda.synchronize()
    assert np.array_equal(ferr.cpu().numpy(), e_o)
    assert np.array_equal(flags.cpu().numpy(), f_o)


def test_batch_config2_full_size(u8, batch_tile):
    """1,000,000 log-normal strings (median 64 B, sigma 1.2), 1% with an injected error."""
    say("case: config2")
    data, offsets, expected = synth.lognormal_batch(1_000_000, 2)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    assert np.array_equal(e_o[expected >= 0], expected[expected >= 0])
    flags, ferr = u8.validate_batch(dev(data), dev(offsets))
    torch.cuda.synchronize()
    assert np.array_equal(ferr.cpu().numpy(), e_o)
    assert np.array_equal(flags.cpu().numpy(), f_o)
    assert int((f_o == 0).sum()) >= 10_000


def test_batch_config3_heavy_tail(u8, batch_tile):
    """20,000 Pareto strings (alpha 1.1, 1 KiB .. 64 MiB), per-string variants, 0.5% errors."""
    say("case: config3a")
    data, offsets, expected = synth.pareto_batch(20_000, 3)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    flags, ferr = u8.validate_batch(dev(data), dev(offsets))
    torch.cuda.synchronize()
    assert np.array_equal(ferr.cpu().numpy(), e_o)
    assert np.array_equal(flags.cpu().numpy(), f_o)
    assert np.array_equal(e_o[expected >= 0], expected[expected >= 0])


def test_batch_config3_heavy_tail_4gib(u8, batch_tile):
    """The heavy tail at x_m 34 KiB: 20,000 Pareto strings, about 4.3 GB, strings up to 64 MiB."""
    say("case: config3b generate")
    data, offsets, expected = synth.pareto_batch(20_000, 3, xm=34 * 1024)
    assert data.size > 4_000_000_000 and int(np.diff(offsets).max()) > 32 << 20
    f_o, e_o = oracle.first_error_batch(data, offsets)
    assert np.array_equal(e_o[expected >= 0], expected[expected >= 0])
    say(f"case: config3b validate {data.size} bytes")
    td, to = dev(data), dev(offsets)
    flags, ferr = u8.validate_batch(td, to)
    torch.cuda.synchronize()
    assert np.array_equal(ferr.cpu().numpy(), e_o)
    assert np.array_equal(flags.cpu().numpy(), f_o)
    assert 50 <= int((f_o == 0).sum()) <= 150
    del td, to, flags, ferr
    torch.cuda.empty_cache()


def test_batch_strings_across_tiles_and_waves(u8, batch_tile):
    """Strings that span several 4 KiB tiles and several waves, errors near every kind of edge."""
    rng = np.random.default_rng(17)
    lens = np.concatenate([[4095, 4096, 4097, 8191, 8192, 8193, 12289, 0, 1, 2, 3, 0, 0],
                           rng.integers(0, 20, 300), rng.integers(4000, 70000, 60), [1_500_000, 2_000_003, 0, 5]])
    rng.shuffle(lens)
    variants = rng.choice(["mixed", "cjk", "emoji", "latin", "ascii"], lens.size).tolist()
    old = u8.get_config()
    try:
        for seed, err in ((31, 0.5), (32, 0.05), (33, 1.0)):
            data, offsets, expected = synth.batch_from_lengths(lens, variants, seed, err_frac=err, base=seed)
            f_o, e_o = oracle.first_error_batch(data, offsets)
            assert np.array_equal(e_o[expected >= 0], expected[expected >= 0])
            td, to = dev(data), dev(offsets)
            for waves in (1, 2, 5, 16, 64):
                say(f"case: across waves seed {seed} batch_waves_per_cu {waves}")
                u8.set_config(batch_waves_per_cu=waves)
                flags, ferr = u8.validate_batch(td, to)
                torch.cuda.synchronize()
                assert np.array_equal(ferr.cpu().numpy(), e_o), (seed, waves)
                assert np.array_equal(flags.cpu().numpy(), f_o), (seed, waves)
    finally:
        u8.set_config(**old)


def test_batch_pieces_at_tile_edges_inside_long_strings(u8, batch_tile):
    """Strings of CJK-like text spanning several 4 KiB tiles (a tile inside one string skips
    the boundary work), each with one piece placed so that a chosen byte of it falls within
    three bytes of a tile edge: lone continuations, leads cut short, overlong, surrogate and
    too-large sequences, bytes F5..FF, and valid 2-, 3- and 4-byte characters cut by the
    edge; some strings end inside a character, short strings sit between them.  Several
    grid sizes move the edges of the waves' runs of tiles."""
    rng = np.random.default_rng(91)
    T = 4096
    cjk = bytes.fromhex("e4b880")
    pieces = [b"\x80", b"\xc3", b"\xc0\x80", b"\xe0\x80\x80", b"\xed\xa0\x80", b"\xf4\x90\x80\x80", b"\xf5",
              b"\xe3\x82", b"\xf0\x9f\x98", b"\xe4\xb8\x80", b"\xf0\x9f\x98\x80", b"\xc3\xa9", b"\xef\xbf\xbf"]
    parts, lens, placed = [], [], []
    pos = 0
    for i in range(3 * len(pieces) * 7):
        if i % 5 == 4:  # a short string between the long ones
            sh = b"a" * int(rng.integers(0, 6))
            parts.append(sh); lens.append(len(sh)); pos += len(sh)
            continue
        piece = pieces[i % len(pieces)]
        j = int(rng.integers(0, len(piece)))
        target = (pos // T + 1 + int(rng.integers(0, 3))) * T + int(rng.integers(-3, 4))
        gap = target - j - pos
        ncjk = (gap - 1) // 3
        body = cjk * ncjk + b"a" * (gap - 3 * ncjk) + piece + b"a" + cjk * int(rng.integers(700, 3000))
        if rng.random() < 0.2:
            body += b"\xe4\xb8"  # the string ends inside a character
        placed.append((pos + gap + j, piece[j]))
        parts.append(body); lens.append(len(body)); pos += len(body)
    data = np.frombuffer(b"".join(parts), np.uint8).copy()
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    assert all(int(data[p]) == b and abs(p - round(p / T) * T) <= 3 for p, b in placed)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    assert (f_o == 0).sum() > 30 and (f_o == 1).sum() > 30
    td, to = dev(data), dev(offsets)
    old = u8.get_config()
    try:
        for waves in (1, 3, 16, 64):
            say(f"case: pieces at tile edges, batch_waves_per_cu {waves}")
            u8.set_config(batch_waves_per_cu=waves)
            flags, ferr = u8.validate_batch(td, to)
            torch.cuda.synchronize()
            assert np.array_equal(ferr.cpu().numpy(), e_o), waves
            assert np.array_equal(flags.cpu().numpy(), f_o), waves
    finally:
        u8.set_config(**old)


def test_batch_long_strings_across_thousands_of_waves(u8, batch_tile):
    """Strings of 32-64 MiB spanning hundreds to thousands of waves (whose arrivals are
    gathered in groups), valid or with one error near their start, middle or end, or cut
    short at the end; short strings around them; several grid sizes."""
    rng = np.random.default_rng(57)
    lens = np.array([5, 64 << 20, 3, (32 << 20) + 17, 0, 1000, (48 << 20) + 5, 2], np.int64)
    data, offsets, _ = synth.batch_from_lengths(lens, ["cjk", "emoji", "ascii", "latin", "ascii", "mixed", "cjk",
                                                       "ascii"], 58)
    f0, e0 = oracle.first_error_batch(data, offsets)
    assert (f0 == 1).all()
    cases = [("valid", data)]
    for name in ("start", "middle", "end"):
        d = data.copy()
        for k in (1, 3, 6):
            s0, s1 = int(offsets[k]), int(offsets[k + 1])
            lo = {"start": 4096, "middle": (s1 - s0) // 2, "end": s1 - s0 - 64}[name]
            synth.inject_random(d[s0:s1], int(rng.integers(0, 2**62)), lo=lo, hi=lo + 64)
        cases.append((name, d))
    d = data.copy()
    d[int(offsets[2]) - 1] = 0xE4  # string 1 ends inside a character
    cases.append(("cut", d))
    old = u8.get_config()
    try:
        for name, d in cases:
            f_o, e_o = oracle.first_error_batch(d, offsets)
            td, to = dev(d), dev(offsets)
            for waves in (4, 16, 64):
                say(f"case: long strings {name}, batch_waves_per_cu {waves}")
                u8.set_config(batch_waves_per_cu=waves)
                flags, ferr = u8.validate_batch(td, to)
                torch.cuda.synchronize()
                assert np.array_equal(ferr.cpu().numpy(), e_o), (name, waves)
                assert np.array_equal(flags.cpu().numpy(), f_o), (name, waves)
            del td
    finally:
        u8.set_config(**old)


def test_batch_graph_replays(u8, batch_tile):
    """The captured-graph entry point: every replay, with eager work between them, equals the oracle."""
    cases = []
    for seed, n in ((21, 50_000), (22, 7), (23, 3_000), (24, 1)):
        data, offsets, _ = synth.lognormal_batch(n, seed)
        f_o, e_o = oracle.first_error_batch(data, offsets)
        cases.append((dev(data), dev(offsets), f_o, e_o))
    side = synth.text(300_001, "mixed", 25)
    synth.inject(side, 222_222, "overlong", 1)
    side_exp = oracle.first_error(side)
    tside = dev(side)
    old = u8.get_config()
    try:
        for rep in range(3):
            for i, (td, to, f_o, e_o) in enumerate(cases):
                say(f"case: graph replay {rep} batch {i} n {e_o.size}")
                n = e_o.size
                flags = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
                ferr = torch.full((n,), -9, dtype=torch.int64, device="cuda")
                u8.validate_batch_graph(td, to, flags, ferr)
                # eager work on the same stream between replays
                assert u8.first_error(tside) == side_exp
                f2, e2 = u8.validate_batch(td, to)
                torch.cuda.synchronize()
                assert np.array_equal(ferr.cpu().numpy(), e_o), (rep, i)
                assert np.array_equal(flags.cpu().numpy(), f_o), (rep, i)
                assert np.array_equal(e2.cpu().numpy(), e_o)
            # a changed launch configuration re-captures the graph
            u8.set_config(batch_waves_per_cu=(3, 16, 5)[rep])
        # many calls in flight on one stream (more than the staging slots), then one check each
        td, to, f_o, e_o = cases[2]
        outs = [torch.full((e_o.size,), -9, dtype=torch.int64, device="cuda") for _ in range(70)]
        flags = torch.empty(e_o.size, dtype=torch.uint8, device="cuda")
        for o in outs:
            u8.validate_batch_graph(td, to, flags, o)
        torch.cuda.synchronize()
        for o in outs:
            assert np.array_equal(o.cpu().numpy(), e_o)
        # another stream gets its own graph
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            td, to, f_o, e_o = cases[0]
            ferr = torch.empty(e_o.size, dtype=torch.int64, device="cuda")
            u8.validate_batch_graph(td, to, flags.new_empty(e_o.size), ferr)
        s.synchronize()
        assert np.array_equal(ferr.cpu().numpy(), e_o)
    finally:
        u8.set_config(**old)


def test_batch_graph_as_the_first_call_of_a_process(u8, tmp_path):
    """A process whose first batch call is the captured-graph entry point (the launch
    configuration's one-time queries then run before the capture): results equal the
    oracle's.  Run in a child process, since this one has made batch calls already."""
    import subprocess
    data, offsets, _ = synth.lognormal_batch(5000, 31)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    np.save(tmp_path / "data.npy", data)
    np.save(tmp_path / "offsets.npy", offsets)
    np.save(tmp_path / "expected.npy", e_o)
    code = (
        "import sys, numpy as np, torch\n"
        f"sys.path.insert(0, {str(ROOT)!r})\n"
        "import paper_2010_03090_amd as u8\n"
        "u8.load()\n"
        f"d = np.load({str(tmp_path / 'data.npy')!r}); o = np.load({str(tmp_path / 'offsets.npy')!r})\n"
        f"e = np.load({str(tmp_path / 'expected.npy')!r})\n"
        "td, to = torch.from_numpy(d).cuda(), torch.from_numpy(o).cuda()\n"
        "flags = torch.empty(e.size, dtype=torch.uint8, device='cuda')\n"
        "ferr = torch.full((e.size,), -9, dtype=torch.int64, device='cuda')\n"
        "u8.validate_batch_graph(td, to, flags, ferr)\n"
        "torch.cuda.synchronize()\n"
        "assert np.array_equal(ferr.cpu().numpy(), e)\n"
        "print('graph first call ok', flush=True)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=100)
    assert r.returncode == 0 and "graph first call ok" in r.stdout, r.stderr[-2000:]


def test_tuning_invariance(u8):
    """Every launch configuration gives identical results."""
    old = u8.get_config()
    bufs = [synth.text(300_001, "mixed", 1), synth.text(70_000, "ascii", 2), synth.text(5000, "random", 3)]
    b = synth.text(200_000, "latin", 4)
    synth.inject(b, 150_000, 2, 4)
    bufs.append(b)
    expected = [oracle.first_error(x) for x in bufs]
    data, offsets, _ = synth.lognormal_batch(20_000, 6)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    td, to = dev(data), dev(offsets)
    tb = [dev(x) for x in bufs]
    try:
        for unroll in (1, 2, 4, 8):
            for ascii_ in (0, 1):
                for waves in (1, 3, 16, 4096):
                    # batch grids of 24 and 64 waves per CU exceed the resident waves (no priority levels)
                    bwaves = {1: 1, 3: 24, 16: 7, 4096: 64}[waves]
                    # the batch tile: 8 KiB with unroll 2 and 8, 4 KiB with 1 and 4 (both with every grid)
                    u8.set_config(unroll=unroll, ascii=ascii_, waves_per_cu=waves,
                                  batch_waves_per_cu=bwaves, batch_ascii=ascii_,
                                  batch_unroll=8 if unroll in (2, 8) else 4)
                    for t, e in zip(tb, expected):
                        assert u8.first_error(t) == e, (unroll, ascii_, waves)
                    flags, ferr = u8.validate_batch(td, to)
                    torch.cuda.synchronize()
                    assert np.array_equal(ferr.cpu().numpy(), e_o), (unroll, ascii_, waves)
    finally:
        u8.set_config(**old)


def test_autotune_keeps_results_exact(u8, tmp_path):
    """The autotuner picks and applies a configuration; results stay bit-exact; the cache applies it."""
    from paper_2010_03090_amd import tune
    old = u8.get_config()
    b = synth.text(3_000_001, "mixed", 19)
    synth.inject(b, 2_500_000, "too_large", 2)
    exp = oracle.first_error(b)
    data, offsets, _ = synth.lognormal_batch(30_000, 20)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    path = str(tmp_path / "tune.json")
    try:
        say("case: autotune")
        cfg = tune.autotune(sample_mib=16, batch_strings=20_000, rounds=2, path=path)
        assert u8.get_config() == cfg
        assert u8.first_error(dev(b)) == exp
        flags, ferr = u8.validate_batch(dev(data), dev(offsets))
        torch.cuda.synchronize()
        assert np.array_equal(ferr.cpu().numpy(), e_o) and np.array_equal(flags.cpu().numpy(), f_o)
        u8.set_config(**old)
        assert tune.apply_cached(path) == cfg and u8.get_config() == cfg
    finally:
        u8.set_config(**old)


def test_async_and_streams(u8):
    b = synth.text(1 << 20, "cjk", 9)
    synth.inject(b, 777_777, 4, 1)
    t = dev(b)
    out = torch.empty(4, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        u8.validate_async(t, out[1:2])
    s.synchronize()
    assert int(out[1]) == oracle.first_error(b)
    assert u8.first_error(t, stream=s) == oracle.first_error(b)


def test_pageable_host_pointer_rejected(u8):
    import ctypes
    buf = ctypes.create_string_buffer(b"abc")
    lib = u8.load()
    assert lib.utf8v_validate_ex(ctypes.addressof(buf), 3, None, None) == -2


def test_stream_any_split_equals_whole(u8):
    """Chunked validation: every split (inside characters, empty and 1-byte chunks) equals the whole."""
    rng = np.random.default_rng(23)
    wholes = []
    for v in ("mixed", "emoji", "cjk", "latin"):   # latin: the short form, with leads carried across splits
        b = synth.text(200_003, v, 30)
        wholes.append(b.copy())
        for cls in range(7):
            c = b.copy()
            synth.inject(c, int(rng.integers(0, c.size)), cls, cls + 1)
            wholes.append(c)
    wholes.append(rng.integers(0, 256, 50_000, dtype=np.uint8))
    t = synth.text(9_999, "emoji", 31)
    wholes.append(t[:-1].copy())                      # cut inside the last character
    for n in range(0, 8):
        wholes.append(synth.text(n, "mixed", 40 + n))
    wholes.append(np.array([0xE2, 0x82], np.uint8))   # incomplete, then more later
    for i, whole in enumerate(wholes):
        exp = oracle.first_error(whole)
        td = dev(whole) if whole.size else torch.empty(0, dtype=torch.uint8, device="cuda")
        for trial in range(4):
            say(f"case: stream whole {i} ({whole.size} B) split {trial}")
            k = int(rng.integers(1, 12))
            cuts = np.sort(rng.integers(0, whole.size + 1, k)) if whole.size else np.zeros(k, np.int64)
            if trial == 3 and whole.size:
                cuts = np.unique(np.concatenate([cuts, np.arange(0, min(whole.size, 9))]))  # 1-byte chunks
            bounds = [0] + cuts.tolist() + [whole.size]
            with u8.Stream() as s:
                for a, b in zip(bounds[:-1], bounds[1:]):
                    s.update(td[a:b])
                assert s.position == whole.size
                assert s.finish() == exp, (i, trial, bounds[:6])


def test_stream_finish_then_continue(u8):
    """A finish reports the prefix; feeding more and finishing again reports the longer stream."""
    ok = "x€y😀".encode()
    part = np.frombuffer(ok[:3], np.uint8)     # "x" and two of the euro sign's three bytes
    rest = np.frombuffer(ok[3:], np.uint8)
    with u8.Stream() as s:
        s.update(dev(part))
        assert s.finish() == oracle.first_error(part) == 1
        s.update(dev(rest))
        assert s.finish() == -1 == oracle.first_error(np.frombuffer(ok, np.uint8))
        s.reset()
        s.update(dev(np.frombuffer(b"\xff", np.uint8)))
        assert s.finish() == 0


def _golden_class_rows():
    import os
    rows = []
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "error_classes.txt")
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            hx, off, cls, label, _ = [x.strip() for x in line.split("|")]
            rows.append((np.frombuffer(bytes.fromhex(hx), np.uint8), int(off), int(cls), label))
    return rows


def test_error_class_paper_examples(u8):
    for b, off, cls, label in _golden_class_rows():
        say(f"case: error class {label}")
        assert u8.first_error(dev(b)) == off, label
        assert u8.error_class(dev(b)) == cls, label


def test_error_classes_batch_exhaustive_and_mixed(u8):
    """Classes of every string of length <= 3, of a labelled mix, and of the 1M-string batch."""
    parts, lens = [], []
    for n in range(1, 4):
        v = np.arange(256 ** n, dtype=np.uint32)
        strs = np.stack([(v >> (8 * k)) & 0xFF for k in range(n)], 1).astype(np.uint8)
        parts.append(strs.reshape(-1))
        lens += [n] * strs.shape[0]
    cases = [(np.concatenate(parts), np.concatenate([[0], np.cumsum(lens)]).astype(np.int64))]
    data, offsets, _ = synth.lognormal_batch(1_000_000, 2)
    cases.append((data, offsets))
    rng = np.random.default_rng(3)
    lens = rng.integers(0, 9, 100_000)
    cases.append((rng.integers(0, 256, int(lens.sum()), dtype=np.uint8),
                  np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)))
    for i, (data, offsets) in enumerate(cases):
        say(f"case: error classes batch {i} ({offsets.size - 1} strings)")
        f_o, e_o = oracle.first_error_batch(data, offsets)
        c_o = oracle.error_class_batch(data, offsets, e_o)
        td, to = dev(data), dev(offsets)
        flags, ferr = u8.validate_batch(td, to)
        cls = u8.error_classes(td, to, ferr)
        torch.cuda.synchronize()
        assert np.array_equal(ferr.cpu().numpy(), e_o)
        got = cls.cpu().numpy()
        assert np.array_equal(got, c_o), np.nonzero(got != c_o)[0][:10]
        if i == 0:   # no string of three bytes holds a complete four-byte sequence: no class 5
            assert set(np.unique(c_o).tolist()) == {0, 1, 2, 3, 4, 6}
        if i == 1:   # the injected error kinds reach every class but 5+ byte leads alone
            assert {2, 3, 4, 5, 6} <= set(np.unique(c_o).tolist())


def test_copy_validate(u8):
    """One pass copies and validates: dst equals src, offsets equal the oracle's (device and pinned host src)."""
    rng = np.random.default_rng(29)
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    sizes = [0, 1, 3, 15, 16, 17, 63, 4095, 4097, 65_537, 1_000_003]
    for i, n in enumerate(sizes):
        b = synth.text(n, ["mixed", "cjk", "emoji", "random"][i % 4], 50 + i)
        if n > 8 and i % 2:
            synth.inject(b, int(rng.integers(0, n)), i % 7, i)
        exp = oracle.first_error(b)
        for host_src in (False, True):
            for off in (0, 5, 15):
                say(f"case: copy_validate n {n} host {host_src} offset {off}")
                base = torch.from_numpy(np.concatenate([np.zeros(off, np.uint8), b, np.zeros(7, np.uint8)]))
                src = (base.pin_memory() if host_src else base.cuda())[off:off + n]
                dbuf = torch.full((n + 64,), 0xAB, dtype=torch.uint8, device="cuda")
                dst = dbuf[off + 16:off + 16 + n]
                u8.copy_validate(src, dst, out)
                torch.cuda.synchronize()
                assert int(out[0]) == exp, (n, host_src, off)
                d = dbuf.cpu().numpy()
                assert np.array_equal(d[off + 16:off + 16 + n], b)
                assert (d[:off + 16] == 0xAB).all() and (d[off + 16 + n:] == 0xAB).all()   # nothing outside dst


def test_copy_kernel(u8):
    """The copy kernel used as the copy ceiling moves every byte (whole tiles and the tail)."""
    rng = np.random.default_rng(81)
    for n in (16, 4096, 3 * 4096 + 16, 1 << 20, (5 << 20) + 4096 + 48):
        say(f"case: copy {n}")
        src = dev(np.frombuffer(rng.bytes(n), np.uint8))
        dst = torch.full((n + 64,), 0xAB, dtype=torch.uint8, device="cuda")
        u8.copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(dst[:n], src) and bool((dst[n:] == 0xAB).all())


def test_copy_validate_rejects_misaligned_or_overlapping(u8):
    lib = u8.load()
    t = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    assert lib.utf8v_copy_validate(t.data_ptr() + 1, t.data_ptr() + 2048, 100, out.data_ptr(), None) == -1
    assert lib.utf8v_copy_validate(t.data_ptr() + 16, t.data_ptr(), 100, out.data_ptr(), None) == -1


def test_async_calls_captured_in_a_torch_graph(u8):
    """validate_async / validate_batch_async captured in a HIP graph (torch.cuda.CUDAGraph), replayed
    several times with eager work and synchronizations between, each replay checked."""
    b = synth.text(3_000_017, "mixed", 60)
    synth.inject(b, 2_000_000, "surrogate", 1)
    exp = oracle.first_error(b)
    data, offsets, _ = synth.lognormal_batch(50_000, 61)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    tb, td, to = dev(b), dev(data), dev(offsets)
    out = torch.full((1,), -9, dtype=torch.int64, device="cuda")
    flags = torch.empty(e_o.size, dtype=torch.uint8, device="cuda")
    ferr = torch.empty(e_o.size, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):   # first calls on this stream create its workspace outside the capture
        u8.validate_async(tb, out)
        u8.validate_batch_async(td, to, flags, ferr)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        u8.validate_async(tb, out)
        u8.validate_batch_async(td, to, flags, ferr)
        # the graph entry point refuses to be recorded (a replay would keep this call's arguments)
        with pytest.raises(u8.Utf8vError) as ei:
            u8.validate_batch_graph(td, to, flags, ferr)
        assert ei.value.status == -1
    for rep in range(4):
        say(f"case: torch graph replay {rep}")
        out.fill_(-9)
        ferr.fill_(-9)
        flags.fill_(9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(out[0]) == exp
        assert np.array_equal(ferr.cpu().numpy(), e_o) and np.array_equal(flags.cpu().numpy(), f_o)
        assert u8.first_error(tb) == exp          # eager work between replays


def test_batch_many_empty_strings(u8, batch_tile):
    """Runs of empty strings (many boundaries at one position) between non-empty ones."""
    rng = np.random.default_rng(62)
    lens = np.zeros(200_000, np.int64)
    idx = rng.choice(lens.size, 3000, replace=False)
    lens[idx] = rng.integers(1, 3000, idx.size)
    for err in (0.0, 0.3):
        say(f"case: many empty strings, err {err}")
        data, offsets, expected = synth.batch_from_lengths(lens, "mixed", 63, err_frac=err)
        f_o, e_o = oracle.first_error_batch(data, offsets)
        flags, ferr = u8.validate_batch(dev(data), dev(offsets))
        torch.cuda.synchronize()
        assert np.array_equal(ferr.cpu().numpy(), e_o)
        assert np.array_equal(flags.cpu().numpy(), f_o)
    lens = np.zeros(1000, np.int64)                # only empty strings
    data, offsets, _ = synth.batch_from_lengths(lens, "mixed", 64, base=5)
    flags, ferr = u8.validate_batch(dev(np.zeros(8, np.uint8)), dev(offsets))
    torch.cuda.synchronize()
    assert (ferr.cpu().numpy() == -1).all() and (flags.cpu().numpy() == 1).all()


def test_sync_calls_from_many_threads_on_one_stream(u8):
    """Synchronous validations issued concurrently from host threads on the same stream each get their own result."""
    import threading
    bufs = []
    for i in range(8):
        b = synth.text(400_000 + 4099 * i, "mixed", 70 + i)
        if i % 2:
            synth.inject(b, 100_000 * (i % 4) + 77, i % 7, i)
        bufs.append((dev(b), oracle.first_error(b)))
    errors = []

    def worker(k):
        try:
            for rep in range(25):
                t, exp = bufs[(k + rep) % len(bufs)]
                got = u8.first_error(t, stream=torch.cuda.default_stream())
                if got != exp:
                    errors.append((k, rep, got, exp))
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))
    say("case: 6 host threads, one stream")
    th = [threading.Thread(target=worker, args=(k,)) for k in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors[:5]


def _exhaustive_short_batch():
    parts, lens = [], []
    for n in range(1, 4):
        v = np.arange(256 ** n, dtype=np.uint32)
        strs = np.stack([(v >> (8 * k)) & 0xFF for k in range(n)], 1).astype(np.uint8)
        parts.append(strs.reshape(-1))
        lens += [n] * strs.shape[0]
    return np.concatenate(parts), np.array(lens, np.int64)


def test_batch_exhaustive_short_strings_at_shifted_alignments(u8, batch_tile):
    """Every string of 1..3 bytes, with the whole batch shifted against 16-byte chunks, 1 KiB slabs
    and 4 KiB tiles (a prefix of k bytes before offsets[0])."""
    data, lens = _exhaustive_short_batch()
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    for k in (1, 2, 3, 13, 15, 16, 17, 1021, 1023, 1025, 4093, 4095, 4097, 4099):
        say(f"case: exhaustive <= 3 shifted by {k}")
        shifted = np.concatenate([np.full(k, 0xE2, np.uint8), data])   # a lead byte run before the batch
        flags, ferr = u8.validate_batch(dev(shifted), dev(offsets + k))
        torch.cuda.synchronize()
        assert np.array_equal(ferr.cpu().numpy(), e_o), k
        assert np.array_equal(flags.cpu().numpy(), f_o), k


def test_batch_subrange_with_invalid_bytes_around(u8, batch_tile):
    """A batch over [lo, hi) of a larger buffer whose bytes outside the range would change the
    results if read: lead bytes before lo, continuation bytes after hi that complete a truncated
    last string.  Errors at the first and last bytes of the range, both edges at many offsets
    against 16-byte chunks and 4 KiB tiles."""
    rng = np.random.default_rng(31)
    alphabet = np.array([0x41, 0x80, 0xA0, 0xBF, 0xC2, 0xE0, 0xE2, 0xED, 0xF0, 0xF4, 0xFF], np.uint8)
    cases = 0
    for pre in (1, 2, 3, 15, 16, 17, 1023, 4093, 4097):
        for body_len in (1, 2, 3, 14, 17, 300, 4096 + 5):
            say(f"case: sub-range pre {pre} body {body_len}")
            body = alphabet[rng.integers(0, alphabet.size, body_len)]
            # the last string ends in a truncated 3-byte sequence; bytes after hi complete it
            tail = np.array([0xE2, 0x82], np.uint8)
            body = np.concatenate([body, tail])
            cuts = np.sort(rng.choice(np.arange(1, body.size), min(body.size - 1, 12), replace=False))
            rel = np.unique(np.concatenate([[0], cuts, [body.size - 2], [body.size]]))
            data = np.concatenate([np.full(pre, 0xF0, np.uint8), body, np.array([0xAC, 0x80, 0x80], np.uint8)])
            offsets = (rel + pre).astype(np.int64)
            f_o, e_o = oracle.first_error_batch(data, offsets)
            assert f_o[-1] == 0   # the truncated last string is invalid on its own
            flags, ferr = u8.validate_batch(dev(data), dev(offsets))
            torch.cuda.synchronize()
            assert np.array_equal(ferr.cpu().numpy(), e_o), (pre, body_len)
            assert np.array_equal(flags.cpu().numpy(), f_o), (pre, body_len)
            cases += 1
    assert cases == 63


def test_batch_two_byte_text_with_longer_characters_and_errors(u8, batch_tile):
    """Batches of 1- and 2-byte text take a short form of the plain checks per tile; a byte
    >= 0xE0 in a tile or in the three bytes before a chunk must send the tile to the full
    checks.  Pieces are placed across chunk, slab and tile edges: 3- and 4-byte characters
    (valid or cut short) in some trials, only 2-byte errors (a lone continuation, a lead
    before ASCII, C0 or C1 leads, a lead at a string's end) in others; string boundaries
    fall at, near and away from those edges."""
    rng = np.random.default_rng(41)
    n = 48 * 1024
    base = np.full(n, 0x61, np.uint8)
    base[5::37], base[6::37] = 0xC3, 0xA9          # U+00E9 every 37 bytes
    edges = [16, 32, 1024, 2048, 4096, 8192, 12288, 16384 + 16, 20480 + 1024, 40960 + 48]
    longer = [(0xE2, 0x82, 0xAC), (0xF0, 0x9F, 0x98, 0x80), (0xE2, 0x82), (0xF0, 0x9F, 0x98), (0xED, 0xA0, 0x80)]
    short = [(0x80,), (0xC3, 0x41), (0xC0, 0x80), (0xC1, 0xBF), (0xC3,), (0xC3, 0xA9), (0xDF, 0xBF, 0xBF)]
    for trial in range(8):
        say(f"case: batch 2-byte text trial {trial}")
        pieces = short if trial % 2 else short + longer
        buf = base.copy()
        for e in edges:
            pc = np.array(pieces[rng.integers(len(pieces))], np.uint8)
            k = int(rng.integers(1, pc.size + 1))
            buf[e - k: e - k + pc.size] = pc
        cuts = set(rng.integers(1, n, 60).tolist()) | {e + int(rng.integers(-3, 4)) for e in edges}
        offsets = np.array(sorted({0, n} | {c for c in cuts if 0 < c < n}), np.int64)
        f_o, e_o = oracle.first_error_batch(buf, offsets)
        assert (f_o == 0).any() and (f_o == 1).any()
        flags, ferr = u8.validate_batch(dev(buf), dev(offsets))
        torch.cuda.synchronize()
        assert np.array_equal(ferr.cpu().numpy(), e_o), trial
        assert np.array_equal(flags.cpu().numpy(), f_o), trial


def test_batch_boundary_alphabet_length_4_and_5(u8, batch_tile):
    """All strings of length 4 and 5 over the 27 boundary bytes of the byte-range table."""
    alpha = np.array([0x00, 0x41, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF, 0xE0,
                      0xE1, 0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xF7, 0xF8, 0xFF], np.uint8)
    for n in (4, 5):
        say(f"case: boundary alphabet length {n}")
        idx = np.indices((alpha.size,) * n, dtype=np.int32).reshape(n, -1).T
        data = alpha[idx].reshape(-1)
        offsets = np.arange(0, data.size + 1, n, dtype=np.int64)
        f_o, e_o = oracle.first_error_batch(data, offsets)
        flags, ferr = u8.validate_batch(dev(data), dev(offsets))
        torch.cuda.synchronize()
        assert np.array_equal(ferr.cpu().numpy(), e_o), n
        assert np.array_equal(flags.cpu().numpy(), f_o), n


@pytest.mark.gpu
def test_batch_length_mix_far_from_stationary(u8, batch_tile):
    """Length mixes where string index and byte position are far from proportional, so the
    interpolated first round of each wave's boundary search misses and the search falls
    back to 64-ary rounds; every launch shape gives the oracle's results."""
    rng = np.random.default_rng(71)
    mixes = {
        # 400k one-byte strings, then 200 strings of 200 KiB
        "tiny_then_huge": np.concatenate([np.ones(400_000, np.int64), np.full(200, 200_000, np.int64)]),
        # the reverse
        "huge_then_tiny": np.concatenate([np.full(200, 200_000, np.int64), np.ones(400_000, np.int64)]),
        # alternating blocks of 50k short strings and 40 long ones
        "blocks": np.concatenate([np.concatenate([rng.integers(0, 8, 50_000), rng.integers(50_000, 150_000, 40)])
                                  for _ in range(6)]).astype(np.int64),
    }
    old = u8.get_config()
    try:
        for name, lens in mixes.items():
            for err in (0.0, 0.02):
                say(f"case: length mix {name}, err {err}")
                data, offsets, _ = synth.batch_from_lengths(lens, "mixed", 72, err_frac=err)
                f_o, e_o = oracle.first_error_batch(data, offsets)
                d_data, d_off = dev(data), dev(offsets)
                for waves in (4, 16, 48):
                    u8.set_config(batch_waves_per_cu=waves)
                    flags, ferr = u8.validate_batch(d_data, d_off)
                    torch.cuda.synchronize()
                    assert np.array_equal(ferr.cpu().numpy(), e_o), (name, err, waves)
                    assert np.array_equal(flags.cpu().numpy(), f_o), (name, err, waves)
    finally:
        u8.set_config(**old)


@pytest.mark.gpu
def test_batch_paper_randomized_inputs(u8, batch_tile):
    """The paper's randomized inputs (section 7.3: code-point byte length uniform over {1},
    {1,2}, {1,2,3}, {1,2,3,4}) as 16 KiB strings, some with an injected error, equal the oracle."""
    for i, variant in enumerate(("unif1", "unif2", "unif3", "unif4")):
        say(f"case: paper-shaped {variant}")
        data, offsets, expected = synth.batch_from_lengths(np.full(512, 16384, np.int64), variant, 80 + i,
                                                           err_frac=0.05)
        f_o, e_o = oracle.first_error_batch(data, offsets)
        assert np.array_equal(e_o[expected >= 0], expected[expected >= 0])
        flags, ferr = u8.validate_batch(dev(data), dev(offsets))
        torch.cuda.synchronize()
        assert np.array_equal(ferr.cpu().numpy(), e_o), variant
        assert np.array_equal(flags.cpu().numpy(), f_o), variant


def test_randomized_shapes_against_the_oracle(u8, batch_tile):
    """Seeded random single buffers (1- and 2-byte text most often, with random errors and a
    stray 3- or 4-byte character), batches (mixed per-string variants, log-normal or Pareto
    lengths, 0-50% errors, a prefix before offsets[0]) and chunked streams of 2-byte text."""
    variants = ["latin", "ascii", "mixed", "cjk", "emoji", "latin", "latin"]
    big = dev(np.zeros(2 * 2**20 + 64, np.uint8))
    for it in range(60):
        rng = np.random.default_rng(7000 + it)
        kind = it % 3
        say(f"case: randomized shape {it} kind {kind}")
        if kind == 0:
            n = int(rng.integers(1, 2 * 2**20))
            b = synth.text(n, variants[int(rng.integers(len(variants)))], it)
            for _ in range(int(rng.integers(0, 4))):
                synth.inject_random(b, int(rng.integers(2**40)))
            if rng.random() < 0.3 and n > 8:
                ch = [(0xE2, 0x82, 0xAC), (0xF0, 0x9F, 0x98, 0x80), (0xED, 0x9F, 0xBF)][int(rng.integers(3))]
                p = int(rng.integers(0, n - 4))
                b[p:p + len(ch)] = ch
            sh = int(rng.integers(0, 16))
            big[sh: sh + n].copy_(torch.from_numpy(b))
            assert u8.first_error(big[sh: sh + n]) == oracle.first_error(b), (it, n, sh)
        elif kind == 1:
            m = int(rng.integers(1, 20000))
            dist = ["lognormal", "pareto"][int(rng.integers(2))]
            lens = synth.lengths(m, dist, float(rng.choice([8, 64, 512])), 1.2 if dist == "lognormal" else 1.1,
                                 0, 100000, it)
            per = ([variants[int(i)] for i in rng.integers(0, len(variants), m)] if rng.random() < 0.5
                   else variants[int(rng.integers(len(variants)))])
            data, offsets, _ = synth.batch_from_lengths(lens, per, it, err_frac=float(rng.choice([0.0, 0.01, 0.1, 0.5])),
                                                        base=int(rng.integers(0, 40)))
            f_o, e_o = oracle.first_error_batch(data, offsets)
            flags, ferr = u8.validate_batch(dev(data), dev(offsets))
            torch.cuda.synchronize()
            assert np.array_equal(ferr.cpu().numpy(), e_o), it
            assert np.array_equal(flags.cpu().numpy(), f_o), it
        else:
            n = int(rng.integers(1, 2**20))
            b = synth.text(n, "latin", it)
            if rng.random() < 0.5:
                synth.inject_random(b, int(rng.integers(2**40)))
            td = dev(b)
            cuts = np.sort(rng.integers(0, n + 1, int(rng.integers(1, 20))))
            bounds = [0] + cuts.tolist() + [n]
            with u8.Stream() as s:
                for a, e in zip(bounds[:-1], bounds[1:]):
                    s.update(td[a:e])
                assert s.finish() == oracle.first_error(b), (it, n)
