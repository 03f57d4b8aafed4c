"""GPU tests of the serving loop: every request bit-exact vs the oracle, alone and in a mix."""
import sys

import numpy as np
import pytest

import oracle
from paper_2010_03090_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_03090_amd as u8
    u8.load()
    from paper_2010_03090_amd import serve
    return serve


def make_pool(serve, sizes, seed, base_every=3):
    rng = np.random.default_rng(seed)
    pool, expect = [], []
    for i, m in enumerate(sizes):
        lens = synth.lengths(m, "lognormal", 64, 1.2, 1, 65536, seed * 1000 + i) if m else np.zeros(0, np.int64)
        variant = ["mixed", "cjk", "random", "emoji"][i % 4] if m else "mixed"
        base = int(rng.integers(1, 40)) if i % base_every == 1 else 0
        data, offsets, _ = synth.batch_from_lengths(lens, variant, seed * 7 + i, err_frac=0.05, base=base)
        pool.append(serve.Request(data, offsets))
        expect.append(oracle.first_error_batch(data, offsets))
    return pool, expect


def check(req, exp, what):
    f, e = req.results()
    assert np.array_equal(e, exp[1]), what
    assert np.array_equal(f, exp[0]), what


@pytest.mark.parametrize("tile", [4, 8])
def test_serve_alone_equals_in_the_mix(sv, tile):
    """Each request's results are the oracle's alone and in a mix (batch tiles of 4 and 8 KiB)."""
    import paper_2010_03090_amd as u8
    old = u8.get_config()
    u8.set_config(batch_unroll=tile)
    try:
        _alone_and_in_the_mix(sv)
    finally:
        u8.set_config(**old)


def _alone_and_in_the_mix(sv):
    sizes = [0, 1, 2, 3, 17, 100, 1000, 4096, 2500, 64, 1, 0, 333, 4000, 7, 900, 2048, 5, 3000, 12] * 2
    pool, expect = make_pool(sv, sizes, 41)
    probe = [1, 7, 13, 19]
    with sv.Server() as srv:
        alone = {}
        for k in probe:
            say(f"case: serve alone request {k} n {pool[k].n}")
            pool[k].reset()
            srv.wait(srv.submit(pool[k]))
            check(pool[k], expect[k], f"alone {k}")
            alone[k] = pool[k].results()
        for rep in range(2):
            say(f"case: serve mix rep {rep} ({len(pool)} requests)")
            for r in pool:
                r.reset()
            tickets = [srv.submit(r) for r in pool]
            for t in tickets:
                srv.wait(t)
            for k, (r, e) in enumerate(zip(pool, expect)):
                check(r, e, f"mix {rep} request {k}")
            for k in probe:
                f, e = pool[k].results()
                assert np.array_equal(f, alone[k][0]) and np.array_equal(e, alone[k][1])
        st = srv.stats()
        assert st["requests_done"] == len(probe) + 2 * len(pool)
        assert st["batches"] >= 1


def test_serve_small_ring_admission(sv):
    """A ring that holds only a few batches: admission waits for space, results stay exact."""
    cfg = sv.default_config(max_batch_bytes=1 << 20, max_batch_strings=1 << 16, max_batch_requests=64,
                            max_inflight=8, streams=3)
    for budget in (1 << 21, 1 << 22):
        cfg.budget_bytes = budget
        try:
            srv = sv.Server(cfg)
            break
        except Exception:
            continue
    else:
        pytest.fail("no small budget accepted")
    pool, expect = make_pool(sv, [2000, 3000, 1500, 4000, 10, 2500, 3500, 1, 3900, 2222] * 3, 42)
    with srv:
        say(f"case: small ring budget {cfg.budget_bytes}")
        for rep in range(2):
            for r in pool:
                r.reset()
            tickets = [srv.submit(r) for r in pool]
            for t in tickets:
                srv.wait(t)
            for k, (r, e) in enumerate(zip(pool, expect)):
                check(r, e, f"small ring rep {rep} request {k}")


@pytest.mark.parametrize("mode", [0, 1])
def test_serve_replay(sv, mode):
    pool, expect = make_pool(sv, [5, 4096, 300, 1, 2000, 77, 3000, 1024], 43)
    arrivals = sv.poisson_arrivals(20_000, 400, 5)
    picks = np.random.default_rng(6).integers(0, len(pool), arrivals.size)
    for r in pool:
        r.reset()
    say(f"case: replay mode {mode}")
    lat, span = sv.replay(pool, arrivals, picks, mode)
    assert (lat > 0).all() and span > 0
    for k in set(picks.tolist()):
        check(pool[k], expect[k], f"replay mode {mode} request {k}")


def test_serve_rejects_oversize_and_bad_requests(sv):
    """A request larger than the batch limits is rejected with a status; the server keeps serving."""
    cfg = sv.default_config(max_batch_bytes=1 << 20, max_batch_strings=1 << 12, max_batch_requests=8,
                            budget_bytes=1 << 24)
    big_data, big_offsets, _ = synth.batch_from_lengths(np.array([(1 << 20) + 1]), "ascii", 5)
    many_data, many_offsets, _ = synth.batch_from_lengths(np.ones(1 << 12, np.int64), "ascii", 6)
    ok_pool, ok_expect = make_pool(sv, [3, 100, 0], 44)
    with sv.Server(cfg) as srv:
        for data, offsets in ((big_data, big_offsets), (many_data, many_offsets)):
            req = sv.Request(data, offsets)
            with pytest.raises(Exception) as ei:
                srv.submit(req)
            assert "invalid argument" in str(ei.value)
        for r, e in zip(ok_pool, ok_expect):
            r.reset()
            srv.wait(srv.submit(r))
            check(r, e, "after rejections")
