"""Writes space_counts.json: valid-configuration counts and a SHA-256 of the
valid raw-index list (uint32 little-endian) for the full-size synthetic
spaces, computed by the oracle only.  Run from the repository root:

    python tests/golden/make_space_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import space as SP  # noqa: E402


def main():
    out = {"_source": "oracle.space.enumerate_valid on the synth spaces; see this script"}
    spaces = {"c1": synth.space_c1(), "c2": synth.space_c2(), "c5": synth.space_c5()}
    for s in range(64):
        spaces[f"batch{s}"] = synth.space_batch(s)
    for name, sp in spaces.items():
        v = SP.enumerate_valid(sp.radix, sp.values, sp.constraints)
        out[name] = {
            "n_raw": sp.n_raw,
            "n_valid": int(len(v)),
            "sha256_valid_u32le": hashlib.sha256(v.astype("<u4").tobytes()).hexdigest(),
        }
        print(name, out[name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "space_counts.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
