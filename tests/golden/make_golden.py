"""Write tests/golden/tiny_expected.json from the CPU oracle alone.

The workload is the 16-input, 8-channel, 256-sample uniform 4+4-bit case.
Run:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2406_19013_amd import synth  # noqa: E402


def main():
    v = synth.tiny().numpy()
    out = oracle.to_int32(oracle.xcorr(v, 4, 256, 8, 16))
    doc = {
        "workload": "16 inputs, 8 channels, 256 samples, re/im iid uniform on [-8,7], 4+4-bit, seed (240619013, 1)",
        "written_by": "tests/golden/make_golden.py (CPU oracle only)",
        "input_sha256": hashlib.sha256(v.tobytes()).hexdigest(),
        "output_sha256": hashlib.sha256(out.tobytes()).hexdigest(),
        "output_shape": list(out.shape),
        "samples": {f"{f},{p}": out[f, p].tolist() for f, p in ((0, 0), (0, 1), (3, 77), (7, 135))},
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_expected.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
