"""The CPU oracle against its pins (no GPU needed)."""
import pytest

import oracle
import _pins


@pytest.fixture(scope="module")
def lib():
    return oracle.load_library()


@pytest.mark.parametrize("pin", _pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(lib, pin):
    pin(lib)


def test_oracle_rejects_bad_arguments(lib):
    import numpy as np
    v = np.zeros((4, 2, 3), np.uint8)
    with pytest.raises(RuntimeError):
        oracle.xcorr(v, 4, 4, 2, 3, chans=[2], lib=lib)      # channel out of range
    with pytest.raises(ValueError):
        oracle.xcorr(v, 4, 5, 2, 3, lib=lib)                 # wrong buffer size
    with pytest.raises(RuntimeError):
        oracle.xcorr_pair(v, 4, 4, 2, 3, 0, 1, 2, lib=lib)   # j > i


def test_tiny_golden_regression(lib):
    """The stored oracle output for the tiny workload (written by
    tests/golden/make_golden.py) still matches: guards generator and oracle
    against silent changes."""
    import hashlib
    import numpy as np
    from paper_2406_19013_amd import synth
    g = _pins.golden("tiny_expected.json")
    v = synth.tiny().numpy()
    assert hashlib.sha256(v.tobytes()).hexdigest() == g["input_sha256"]
    out = oracle.to_int32(oracle.xcorr(v, 4, 256, 8, 16, lib=lib))
    assert hashlib.sha256(out.tobytes()).hexdigest() == g["output_sha256"]
    for key, val in g["samples"].items():
        f, p = map(int, key.split(","))
        assert out[f, p].tolist() == val
