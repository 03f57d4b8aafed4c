"""The C-ABI entry points called through ctypes with device data (needs an MI355X).

The synchronous functions of the boundary -- utf8_validate(buf, len) -> bool and
utf8_validate_batch(data, offsets, n, out_flags, out_first_err) -- and the offsets
checker, against the oracle element by element.
"""
import ctypes
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


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return _native.load()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).copy()).cuda()


def _cases():
    """Valid and invalid buffers of several sizes, every error class, and the empty buffer."""
    out = [np.zeros(0, np.uint8), np.frombuffer(b"\xc3", np.uint8), np.frombuffer("é€😀".encode(), np.uint8)]
    for i, (n, variant) in enumerate(((1, "ascii"), (17, "mixed"), (4099, "cjk"), (300_001, "emoji"),
                                      (1_000_003, "mixed"), (2_000_000, "latin"))):
        b = synth.text(n, variant, 40 + i)
        out.append(b)
        for cls in range(7):
            c = b.copy()
            if synth.inject(c, (n * cls) // 7, cls, 50 + 7 * i + cls) >= 0:
                out.append(c)
    return out


def test_utf8_validate_on_device_data(lib):
    torch.cuda.synchronize()
    for b in _cases():
        say(f"case: utf8_validate len {b.size}")
        t = dev(b)
        torch.cuda.synchronize()
        got = lib.utf8_validate(t.data_ptr() if b.size else None, b.size)
        assert lib.utf8v_last_status() == 0
        assert got == (oracle.first_error(b) < 0), b.size


def _batch(seed, base):
    data, offsets, _ = synth.batch_from_lengths(
        np.array([0, 1, 3, 4, 0, 17, 64, 5000, 0, 2, 70_000, 1, 0] * 40, np.int64),
        "mixed", seed, err_frac=0.3, base=base)
    return data, offsets


def test_utf8_validate_batch_on_device_data(lib):
    for seed, base in ((61, 0), (62, 5), (63, 4093)):
        say(f"case: utf8_validate_batch seed {seed} offsets[0] {base}")
        data, offsets = _batch(seed, base)
        f_o, e_o = oracle.first_error_batch(data, offsets)
        assert (f_o == 0).any() and (f_o == 1).any()
        n = offsets.size - 1
        td, to = dev(data), dev(offsets)
        flags = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        ferr = torch.full((n,), -7, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        assert lib.utf8_validate_batch(td.data_ptr(), to.data_ptr(), n, flags.data_ptr(), ferr.data_ptr()) == 0
        assert np.array_equal(ferr.cpu().numpy(), e_o)
        assert np.array_equal(flags.cpu().numpy(), f_o)
    # n == 0 is a no-op and touches nothing
    assert lib.utf8_validate_batch(td.data_ptr(), to.data_ptr(), 0, flags.data_ptr(), ferr.data_ptr()) == 0


def test_utf8_validate_batch_rejects_host_pointers(lib):
    data, offsets = _batch(64, 0)
    n = offsets.size - 1
    td, to = dev(data), dev(offsets)
    flags = torch.empty(n, dtype=torch.uint8, device="cuda")
    ferr_host = np.empty(n, np.int64)   # pageable host memory: not reachable by the GPU
    rc = lib.utf8_validate_batch(td.data_ptr(), to.data_ptr(), n, flags.data_ptr(), ferr_host.ctypes.data)
    assert rc == _native.UTF8V_ENOTDEVICE


def test_check_offsets(lib):
    good = [np.array([0], np.int64), np.array([3, 3, 3], np.int64), np.arange(0, 10_000_000, 7, dtype=np.int64)]
    bad = [np.array([-1, 4], np.int64), np.array([0, 5, 4, 9], np.int64),
           np.concatenate([np.arange(0, 1_000_000, 3), [5], np.arange(3_000_000, 3_000_100)]).astype(np.int64)]
    for o in good:
        say(f"case: check_offsets good n {o.size - 1}")
        assert lib.utf8v_check_offsets(dev(o).data_ptr(), o.size - 1, None) == 1
    for o in bad:
        say(f"case: check_offsets bad n {o.size - 1}")
        assert lib.utf8v_check_offsets(dev(o).data_ptr(), o.size - 1, None) == 0
    assert lib.utf8v_check_offsets(None, 3, None) == _native.UTF8V_EINVAL


def test_release_then_fresh_calls(lib):
    """utf8v_release frees the workspaces; the next calls make new ones and stay exact."""
    b = synth.text(500_001, "cjk", 70)
    synth.inject(b, 333_333, "surrogate", 71)
    exp = oracle.first_error(b)
    data, offsets = _batch(72, 9)
    f_o, e_o = oracle.first_error_batch(data, offsets)
    t, td, to = dev(b), dev(data), dev(offsets)
    n = offsets.size - 1
    for rep in range(2):
        say(f"case: release round {rep}")
        torch.cuda.synchronize()
        out = ctypes.c_int64(0)
        assert lib.utf8v_validate_ex(t.data_ptr(), b.size, ctypes.byref(out), None) == 0 and out.value == exp
        flags = torch.empty(n, dtype=torch.uint8, device="cuda")
        ferr = torch.empty(n, dtype=torch.int64, device="cuda")
        assert lib.utf8_validate_batch(td.data_ptr(), to.data_ptr(), n, flags.data_ptr(), ferr.data_ptr()) == 0
        assert np.array_equal(ferr.cpu().numpy(), e_o) and np.array_equal(flags.cpu().numpy(), f_o)
        torch.cuda.synchronize()
        assert lib.utf8v_release() == 0

