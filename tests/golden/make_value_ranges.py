"""Writes value_ranges.json: the stored value range (scale, offset) of each
named random-init INR, computed by the CPU oracle only.  Section 4.1 keeps the
data's value range with the model for normalisation at render time; for a
random-init network the range is the 2nd..98th percentile of its raw output
over a fixed Halton probe set.

Run: python tests/golden/make_value_ranges.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2504_18001_amd import configs, synth  # noqa: E402

ARCHS = {"small": configs.ARCH_SMALL, "inr512": configs.ARCH_512, "tera": configs.ARCH_TERA}


def main():
    out = {}
    for name, arch in ARCHS.items():
        for seed in range(4):
            t, w = synth.random_inr_params(arch, seed)
            s, o = O.value_normalization(arch, t, w)
            out[f"{name}/{seed}"] = {"value_scale": s, "value_offset": o}
            print(name, seed, s, o, flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "value_ranges.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
