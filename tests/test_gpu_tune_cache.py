"""Tuning decisions saved to a file and loaded by a new context (GPU).

A context that loads the file of another context finds every launch shape
of the same solve in it: the solve adds no shape to the table (the timing
runs of a shape happen exactly when it is added), and, every tile
configuration summing in the same order, it gives the same bits.  Files of
another build or device, or malformed ones, are refused.
"""

import numpy as np
import pytest

from synth import make_problem

pytestmark = pytest.mark.gpu


def _solve(rid, ctx, p):
    prob = rid.Problem.from_synth(ctx, p)
    out = prob.eigen(5, "rpa", "ris", "mixed")
    prob.close()
    return out


def test_tuning_file_round_trip(tmp_path):
    import paper_2404_17133_amd as rid

    p = make_problem(20, 80, 400, 90, seed=0).to("cuda:0")
    path = str(tmp_path / "tune.txt")
    a = rid.Context(0)
    first_a = _solve(rid, a, p)
    n = a.tune_save(path)
    assert n > 0
    assert a.tune_save(path) == n
    second_a = _solve(rid, a, p)
    assert a.tune_save(path) == n  # a second solve adds no shape
    assert np.array_equal(first_a["omega"], second_a["omega"])
    a.close()

    b = rid.Context(0)
    assert b.tune_save(str(tmp_path / "empty.txt")) == 0
    assert b.tune_load(path) == n
    first_b = _solve(rid, b, p)
    assert np.array_equal(first_b["omega"], first_a["omega"])
    assert b.tune_save(str(tmp_path / "again.txt")) == n  # no new shapes
    b.close()


def test_foreign_or_malformed_files_are_refused(tmp_path):
    import paper_2404_17133_amd as rid
    from paper_2404_17133_amd import _binding as B

    ctx = rid.Context(0)
    good = str(tmp_path / "good.txt")
    ctx.tune_save(good)
    lines = open(good).read().splitlines()
    head = lines[0].split()
    assert head[:2] == ["rid-tune", "1"] and head[3].startswith("gfx950")
    other = str(tmp_path / "other.txt")
    open(other, "w").write("rid-tune 1 0000000000000000 %s\n3 4 4000 800 1 20 800 1 5 4\n" % head[3])
    bad = [lines[0] + "\n" + body for body in (
        "3 4 4000 800 1 20 800 7 5 4\n",   # tile configuration 7 does not exist
        "3 8 4000 800 1 20 800 -1 5 4\n",  # a negative tile configuration
        "3 4 4000 800 1 20 800 0 2 4\n",   # 2 splits of 4 batches do not cover 20
        "9 4 4000 800 1 20 800 0 5 4\n",   # no family 9
        "3 4 4000 800 1 20 800 0 5\n",     # a field missing
        "3 4 4000 800 1 20 800 0 5 4\n3 6 4000 800 1 20 800 0 5 4\n")]  # 6-byte elements
    paths = [other, str(tmp_path / "missing.txt")]
    for j, text in enumerate(bad):
        paths.append(str(tmp_path / ("bad%d.txt" % j)))
        open(paths[-1], "w").write(text)
    for path in paths:
        with pytest.raises(rid.RidError) as e:
            ctx.tune_load(path)
        assert e.value.status == B.RID_ERR_INVALID_ARG
    assert ctx.tune_save(str(tmp_path / "after.txt")) == 0  # nothing of a refused file was kept
    ctx.close()
