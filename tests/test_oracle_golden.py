"""The stored expected values under tests/golden/ still follow from the oracle
(they were written by tests/golden/make_golden.py, which calls only oracle/)."""
import json
import os

import pytest

from paper_2108_12050_amd import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_strict_seeds_have_no_ambiguous_decisions(ora):
    d = json.load(open(os.path.join(GOLD, "strict_seeds.json")))
    assert len(d["seeds"]) == 8
    for s in d["seeds"][:3]:
        st = ora.log_stack(synth.blob_field(s, 256, 256), d["sigmas"], d["truncate"])
        assert ora.ambiguous(st, d["tau"], d["eps"]) == 0


@pytest.mark.parametrize("i", [0, 5])
def test_plain_512_counts(ora, i):
    d = json.load(open(os.path.join(GOLD, "plain_512_counts.json")))
    rec = d["records"][i]
    out = ora.detect(synth.plain_tile(rec["seed"]), d["sigmas"], d["truncate"], d["tau"], d["overlap"])
    assert len(out["cand"]) == rec["candidates"] and out["count"] == rec["blobs"]
