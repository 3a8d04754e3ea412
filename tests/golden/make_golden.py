"""Write the small text fixtures in this folder.  Calls only the oracle.

The paper prints no worked numeric example, so these fixtures are regression
pins of the oracle itself: small integer-valued inputs (listed in the file)
and the oracle's FP64 fused outputs, printed with 17 significant digits.  A
later change to the oracle's arithmetic that moves any of them must say which
passage of the paper justifies it.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def case(wavelet, H, W, B, seed, gain):
    rng = np.random.Generator(np.random.PCG64(seed))
    pan = rng.integers(0, 256, (H, W)).astype(np.float64)
    ms = rng.integers(0, 256, (B, H // 2, W // 2)).astype(np.float64)
    out = oracle.fuse(wavelet, pan, ms, gain)
    return {
        "wavelet": wavelet, "H": H, "W": W, "B": B, "gain": gain,
        "pan": pan.astype(int).tolist(), "ms": ms.astype(int).tolist(),
        "out": [[["%.17g" % v for v in row] for row in band] for band in out],
    }


def main():
    cases = [
        case("haar", 4, 6, 1, 11, None),
        case("d4", 8, 8, 2, 12, [1.0, 0.5]),
        case("d4", 6, 10, 1, 13, None),
        case("d4", 2, 4, 1, 14, None),
    ]
    with open(os.path.join(HERE, "oracle_fuse_small.json"), "w") as f:
        json.dump({"generator": "tests/golden/make_golden.py", "cases": cases}, f, indent=0)
        f.write("\n")


if __name__ == "__main__":
    main()
