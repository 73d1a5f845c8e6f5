"""Write the stored expected values under tests/golden/ from the oracle only.

Run from the repository root:  python tests/golden/make_golden.py

strict_seeds.json
    Seeds of the plain blob workload at 256 x 256 (50 blobs, same density
    and value distributions as the 512 x 512 workload) for which no voxel's
    candidate decision lies within 1e-4 of the threshold or of a window
    neighbour (oracle.ambiguous == 0).  On these, blob lists must agree bit
    for bit.  The full-size 512 x 512 workload has about ten such near-ties
    per image (two pixels straddling a blob centre), so no seed of it passes.
plain_512_counts.json
    Oracle candidate and blob counts of the 512 x 512 plain workload for
    seeds 0..7 (sigma 1..10, truncate 4, tau 0.1, overlap 0.5): a regression
    record of the oracle itself.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2108_12050_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    sig = oracle.linear_sigmas(10, 1.0, 10.0)
    strict = []
    seed = 0
    while len(strict) < 8:
        st = oracle.log_stack(synth.blob_field(seed, 256, 256), sig)
        if oracle.ambiguous(st, 0.1, 1e-4) == 0:
            strict.append(seed)
        seed += 1
    with open(os.path.join(HERE, "strict_seeds.json"), "w") as f:
        json.dump({"workload": "blob_field 256x256, 50 blobs", "sigmas": sig.tolist(),
                   "truncate": 4.0, "tau": 0.1, "eps": 1e-4, "scanned": seed,
                   "seeds": strict}, f, indent=1)
    rec = []
    for s in range(8):
        d = oracle.detect(synth.plain_tile(s), sig, tau=0.1, theta=0.5)
        rec.append({"seed": s, "candidates": int(len(d["cand"])), "blobs": d["count"]})
    with open(os.path.join(HERE, "plain_512_counts.json"), "w") as f:
        json.dump({"workload": "plain_tile 512x512", "sigmas": sig.tolist(), "truncate": 4.0,
                   "tau": 0.1, "overlap": 0.5, "records": rec}, f, indent=1)


if __name__ == "__main__":
    main()
