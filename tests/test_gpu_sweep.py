"""The sensitivity sweep runs end to end on a small genome and its numbers
behave as the filter's definition implies: a larger error tolerance lowers the
threshold, so read existence never falls as e grows; every candidate that
passes at some e still passes at a larger e."""

from __future__ import annotations

import json

import pytest

from paper_1708_04329_amd import sweep

pytestmark = pytest.mark.gpu


def test_sweep_small(tmp_path, capsys):
    out = tmp_path / "s.json"
    sweep.main(["--genome-len", "3000000", "--reads", "200", "--bins-64k", "1,2", "--q", "4,5", "--cap", "256",
                "--json", str(out)])
    d = json.loads(out.read_text())
    for q in (4, 5):
        for b in ("1x64k", "2x64k"):
            xs = sorted((x for x in d["read_existence"] if x["q"] == q and x["bins"] == b), key=lambda x: x["e_pct"])
            assert len(xs) == 6
            vals = [x["read_existence"] for x in xs]
            assert all(0.0 <= v <= 1.0 for v in vals) and vals == sorted(vals)
    for b in ("1x64k", "2x64k"):
        xs = sorted((x for x in d["false_negative_rate"] if x["bins"] == b), key=lambda x: x["e_pct"])
        passing = [x["passing"] for x in xs]
        mapping = [x["mapping"] for x in xs]
        assert passing == sorted(passing) and mapping == sorted(mapping)
        assert all(x["passing"] <= x["candidates"] for x in xs)
