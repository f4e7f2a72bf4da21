"""The hardware-ceiling kernels behind the benchmark's measured roofline: they
run, report the work they do, and the MFMA one really multiplies its operands
(its checksum matches a host computation)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2406_19013_amd import xcorr as X  # noqa: E402


def _volts(T, F, N, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randint(0, 256, (T, F, N), generator=g, dtype=torch.uint8)


def test_mfma_ceiling_checksum():
    """Each wave multiplies four 1 KB operand fragments of the input (offset
    wave * 4096 modulo the span); the sum of all its accumulator entries after
    `iters` rounds is iters * sum over the 16 products of
    sum_k (sum_i A[i][k]) (sum_j B[k][j]), which only needs which lanes share
    a K half (lanes l and l + 32 hold the two halves of row l % 32)."""
    T, F, N = 64, 4, 192
    v = _volts(T, F, N, 11)
    dev = torch.device("cuda:0")
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    out = torch.zeros(512 * cus, dtype=torch.int32, device=dev)
    iters = 3
    ops = X.xcorr_ceiling(X.CEILING_MFMA_I8, v.to(dev), T, F, N, iters, out)
    torch.cuda.synchronize()
    assert ops == cus * 8 * iters * 16 * 65536
    raw = v.numpy().reshape(-1).view(np.int8).astype(np.int64)
    span = (raw.size - 4096) // 16 * 16 + 16
    got = out.cpu().numpy().astype(np.int64).reshape(cus * 8, 64)
    pairs = [(m & 3, (m + 1) & 3) for m in range(8)] + [((m + 2) & 3, (m + 3) & 3) for m in range(8)]
    for wid in list(range(8)) + [cus * 8 - 1]:
        base = (wid * 4096) % span
        frag = raw[base:base + 4096].reshape(4, 64, 16)          # [operand][lane][byte]
        halves = frag.reshape(4, 2, 32, 16).sum(axis=2)          # [operand][K half][byte]
        want = sum(int((halves[a] * halves[b]).sum()) for a, b in pairs) * iters
        assert (int(got[wid].sum()) - want) % (1 << 32) == 0, wid


def test_stream_ceiling_runs_and_counts_bytes():
    T, F, N = 200, 40, 192
    dev = torch.device("cuda:0")
    v = _volts(T, F, N, 12).to(dev)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    out = torch.zeros(512 * cus, dtype=torch.int32, device=dev)
    ops = X.xcorr_ceiling(X.CEILING_STREAM, v, T, F, N, 1, out)
    torch.cuda.synchronize()
    assert ops == T * F * N


def test_ceiling_refusals():
    dev = torch.device("cuda:0")
    v = torch.zeros((4, 8, 192), dtype=torch.uint8, device=dev)
    out = torch.zeros(8, dtype=torch.int32, device=dev)
    with pytest.raises(X.XcorrError):
        X.xcorr_ceiling(X.CEILING_STREAM, v, 4, 8, 192, 1, out)      # output too short
    big = torch.zeros(512 * 1024, dtype=torch.int32, device=dev)
    with pytest.raises(X.XcorrError):
        X.xcorr_ceiling(7, v, 4, 8, 192, 1, big)                      # unknown kind
    with pytest.raises(X.XcorrError):
        X.xcorr_ceiling(X.CEILING_STREAM, v, 4, 8, 100, 1, big)       # N not a multiple of 16
