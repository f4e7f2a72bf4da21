"""Input generator and sample-format facts (no GPU needed)."""
import numpy as np
import torch

from paper_2406_19013_amd import synth
import _pins


def test_pack_roundtrip_all_values():
    vals = torch.arange(-8, 8)
    re, im = torch.meshgrid(vals, vals, indexing="ij")
    b = synth.pack4(re, im)
    r2, i2 = synth.unpack4(b)
    assert torch.equal(r2, re.int()) and torch.equal(i2, im.int())
    assert len(set(b.flatten().tolist())) == 256


def test_high_nibble_is_real():
    b = synth.pack4(torch.tensor([3]), torch.tensor([-2]))
    assert int(b[0]) == 0x3E


def test_generators_are_deterministic_and_seeded():
    a = synth.tiny()
    b = synth.tiny()
    assert torch.equal(a, b) and a.shape == (256, 8, 16) and a.dtype == torch.uint8
    c = synth.gaussian_volts(8, 4, 64, sigma=2.5, bits=4, seed=(1, 2), tone=synth.Tone())
    d = synth.gaussian_volts(8, 4, 64, sigma=2.5, bits=4, seed=(1, 2), tone=synth.Tone())
    e = synth.gaussian_volts(8, 4, 64, sigma=2.5, bits=4, seed=(1, 3), tone=synth.Tone())
    assert torch.equal(c, d) and not torch.equal(c, e)


def test_chunked_generation_matches_unchunked():
    a = synth.gaussian_volts(8, 4, 100, sigma=2.5, bits=4, seed=(5,), chunk_t=7)
    b = synth.gaussian_volts(8, 4, 100, sigma=2.5, bits=4, seed=(5,), chunk_t=7)
    assert torch.equal(a, b)


def test_8bit_range_and_shape():
    v = synth.gaussian_volts(4, 3, 500, sigma=60.0, bits=8, seed=(9,))
    assert v.shape == (500, 3, 4, 2) and v.dtype == torch.int8
    assert int(v.min()) >= -127 and int(v.max()) <= 127


def test_gaussian_statistics_of_tianlai_recipe():
    v = synth.gaussian_volts(16, 8, 512, sigma=2.5, bits=4, seed=(2,), tone=None)
    re, im = synth.unpack4(v)
    x = torch.cat([re.flatten(), im.flatten()]).double()
    assert abs(x.mean().item()) < 0.05
    assert abs(x.std().item() - 2.5) < 0.1   # rounding adds ~1/12, clipping removes a little


def test_one_byte_per_sample_reproduces_link_rates():
    """Section 2.2's printed port rates follow from one byte per (input, channel,
    spectrum) for the 4+4-bit format, plus a small packet-header overhead."""
    g = _pins.golden("link_rates.json")
    bytes_per_sample = 1
    roach = g["inputs_per_board"] * g["channels_per_roach2_port"] * g["spectra_per_s"] * 8 * bytes_per_sample
    gpu = g["n_inputs"] * g["channels_per_gpu_port"] * g["spectra_per_s"] * 8 * bytes_per_sample
    for payload, printed in ((roach, g["roach2_port_gbps"]), (gpu, g["gpu_port_gbps"])):
        ovh = printed * 1e9 / payload - 1
        assert 0 <= ovh < g["max_header_overhead"]
    assert abs(6 * 4 * g["roach2_port_gbps"] - g["total_gbps"]) < 1e-9
    # both printed figures carry the same overhead factor
    r1 = g["roach2_port_gbps"] * 1e9 / roach
    r2 = g["gpu_port_gbps"] * 1e9 / gpu
    assert abs(r1 - r2) < 1e-4
