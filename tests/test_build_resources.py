"""The compiler's resource report of the last build: the kernels on the hot
paths (16-byte-aligned inputs, 64-row chunks) must not spill registers to
scratch memory; a spill there has cost an order of magnitude in time.

One bounded exception: the three-product kernel at D = 6 (the 192-input
triangle) spills at most 96 bytes per lane, all in its chunk-issue and
per-channel epilogue code, none in the K-step body; the variants that
removed the spill (channel offset in the scalar base, or at most 8
accumulators per wave) moved it into the K loop and ran 27 % slower."""
import os
import re

import pytest

from paper_2406_19013_amd import build

REPORT = os.path.join(os.path.dirname(build.__file__), "_build", build.RESOURCES)

HOT = [
    re.compile(r"xc_gauss4_kernelILi[1-5]ELi0E"),          # 4+4-bit default kernel, one launch per integration
    re.compile(r"xc_mfma4f_kernelILi[1-6]ELi1E"),         # 4+4-bit fused kernel (inputs not a multiple of 16)
    re.compile(r"xc_mfma4_kernelILi\dELi64ELi1E"),        # 4+4-bit per-role kernel, every D
    re.compile(r"xc_mfma8_kernelILi\dELb[01]ELi64ELi1E"),  # 8+8-bit int8 and FP16, LDS-DMA
    re.compile(r"xc_batch4_kernelILi1E"),                  # batched, LDS-DMA
]


@pytest.mark.skipif(not os.path.exists(REPORT), reason="no build report (run the build first)")
def test_hot_kernels_do_not_spill():
    res = build.read_resources(REPORT)
    hot = {k: v for k, v in res.items() if any(p.search(k) for p in HOT)}
    assert len(hot) >= 10 + 6 + 6 + 12 + 1, sorted(hot)
    spills = {k: v["ScratchSize"] for k, v in hot.items() if v.get("ScratchSize", 0)}
    assert not spills, spills
    for k, v in hot.items():
        assert v["VGPRs"] + v.get("AGPRs", 0) <= 512, k


@pytest.mark.skipif(not os.path.exists(REPORT), reason="no build report (run the build first)")
def test_three_product_kernel_d6_spill_is_bounded():
    res = build.read_resources(REPORT)
    d6 = {k: v for k, v in res.items() if re.search(r"xc_gauss4_kernelILi6ELi0E", k)}
    assert len(d6) == 2, sorted(d6)
    for k, v in d6.items():
        assert v.get("ScratchSize", 0) <= 96, (k, v)
