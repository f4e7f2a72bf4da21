"""The compiler's resource report of the last build: the kernels on the hot
paths (16-byte-aligned inputs, 64-row chunks) must not spill registers to
scratch memory; a spill there has cost an order of magnitude in time."""
import os
import re

import pytest

from paper_2406_19013_amd import build

REPORT = os.path.join(os.path.dirname(build.__file__), "_build", build.RESOURCES)

HOT = [
    re.compile(r"xc_gauss4_kernelILi[1-6]ELi[012]ELi[01]ELi[01]E"),   # 4+4-bit default kernel, every shape
    re.compile(r"xc_mfma4f_kernelILi[1-6]ELi1E"),         # 4+4-bit fused kernel (inputs not a multiple of 16)
    re.compile(r"xc_mfma4_kernelILi\dELi64ELi1E"),        # 4+4-bit per-role kernel, every D
    re.compile(r"xc_mfma8_kernelILi\dELb[01]ELi64ELi1E"),  # 8+8-bit int8 and FP16, LDS-DMA
    re.compile(r"xc_batch4_kernelILi1E"),                  # batched, LDS-DMA
]


@pytest.mark.skipif(not os.path.exists(REPORT), reason="no build report (run the build first)")
def test_hot_kernels_do_not_spill():
    res = build.read_resources(REPORT)
    hot = {k: v for k, v in res.items() if any(p.search(k) for p in HOT)}
    assert len(hot) >= 52 + 6 + 6 + 12 + 1, sorted(hot)
    spills = {k: v["ScratchSize"] for k, v in hot.items() if v.get("ScratchSize", 0)}
    assert not spills, spills
    for k, v in hot.items():
        assert v["VGPRs"] + v.get("AGPRs", 0) <= 512, k
