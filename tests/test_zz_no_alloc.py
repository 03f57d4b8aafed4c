"""The allocation-free batch entry point against the allocating one (needs an MI355X).

utf8v_validate_batch_noalloc keeps the batch kernel's cross-wave slots in a fixed
device array instead of a per-stream workspace.  Called through the C-ABI twice in a
row -- a batch whose strings run across waves (so the slots are used), then a smaller
one -- its flags and first-error offsets equal those of utf8v_validate_batch_async and
the oracle's, element by element.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2010_03090_amd import _native, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).copy()).cuda()


def _run(lib, fn, td, to, n, stream):
    flags = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    ferr = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    assert fn(td.data_ptr(), to.data_ptr(), n, flags.data_ptr(), ferr.data_ptr(), stream) == 0, \
        lib.utf8v_last_status()
    return flags, ferr


@pytest.mark.parametrize("waves", [16, 64, 3])
def test_noalloc_equals_the_allocating_entry_point(waves):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_03090_amd as u8
    lib = _native.load()
    rng = np.random.default_rng(90 + waves)
    # strings across tiles and waves (up to 6 MB), errors in about half of them
    big = np.concatenate([rng.integers(0, 200, 3000), rng.integers(4000, 90_000, 200),
                          [6_000_001, 2_500_000, 0, 1, 3_999_999]]).astype(np.int64)
    rng.shuffle(big)
    small = rng.integers(0, 300, 5000).astype(np.int64)
    old = u8.get_config()
    try:
        u8.set_config(batch_waves_per_cu=waves, batch_unroll=8 if waves == 3 else 4)  # 4 and 8 KiB tiles
        stream = torch.cuda.current_stream().cuda_stream or None
        for i, (lens, err) in enumerate(((big, 0.5), (small, 0.2))):
            data, offsets, expected = synth.batch_from_lengths(lens, "mixed", 100 + waves + i, err_frac=err, base=3)
            f_o, e_o = oracle.first_error_batch(data, offsets)
            assert np.array_equal(e_o[expected >= 0], expected[expected >= 0])
            n = offsets.size - 1
            td, to = dev(data), dev(offsets)
            say(f"case: noalloc waves {waves} call {i} n {n} bytes {data.size}")
            f_a, e_a = _run(lib, lib.utf8v_validate_batch_noalloc, td, to, n, stream)
            f_b, e_b = _run(lib, lib.utf8v_validate_batch_async, td, to, n, stream)
            torch.cuda.synchronize()
            assert np.array_equal(e_a.cpu().numpy(), e_b.cpu().numpy())
            assert np.array_equal(f_a.cpu().numpy(), f_b.cpu().numpy())
            assert np.array_equal(e_a.cpu().numpy(), e_o)
            assert np.array_equal(f_a.cpu().numpy(), f_o)
    finally:
        u8.set_config(**old)
