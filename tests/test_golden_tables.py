"""Counting conventions and storage formulas checked against the paper's
tables (tests/golden/paper_tables.json)."""
import json
import os
import re

import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def storage_words(name):
    """Extra storage per unknown: BiCGStab 8, GMRES(m) (m+1)+4, rGCROT(m,k)
    m + 2k + 3, rBiCGStab(k) 8 + 2k (Sec. 2.2-2.3: GMRES(m) (m+1)N + 4N,
    BiCGStab 8N, recycling adds 2kN)."""
    m = re.match(r"(\w+)(?:\((\d+)(?:,(\d+))?\))?", name)
    kind, a, b = m.group(1), m.group(2), m.group(3)
    if kind == "BiCGStab":
        return 8
    if kind == "GMRES":
        return int(a) + 1 + 4
    if kind == "rGCROT":
        return int(a) + 2 * int(b) + 3
    if kind == "rBiCGStab":
        return 8 + 2 * int(a)
    raise ValueError(name)


@pytest.mark.parametrize("table", ["storage_channel", "storage_porous"])
def test_storage_formulas(table):
    for name, words in GOLD[table].items():
        if name.startswith("_"):
            continue
        assert storage_words(name) == words


@pytest.mark.parametrize("table", ["channel_start", "channel_stationary"])
def test_counting_convention(table):
    """A cycle is m matvecs, a BiCGStab iteration 2; total time = steps x
    units per step x seconds per unit."""
    t = GOLD[table]
    for name, row in t.items():
        if name.startswith("_") or name == "steps":
            continue
        assert t["steps"] * row["per_step"] * row["s_per_unit"] == pytest.approx(row["total_s"], rel=0.06)
        m = re.match(r"\w+\((\d+)", name)
        per_unit = 2 if name == "BiCGStab" else int(m.group(1))
        if name.startswith("GMRES") or name == "BiCGStab":
            assert row["per_step"] * per_unit == pytest.approx(row["matvecs_per_step"], rel=0.02)
