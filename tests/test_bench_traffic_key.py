"""The key of the recorded HBM byte counts in bench.py: a hash of the sweep
sources' code, with comments and blank space removed, so that a comment edit
keeps the counts and a code edit drops them."""
from __future__ import annotations

import bench


def test_code_only_drops_comments_and_blank_space():
    src = "int x = 1; // one\n/* a block\n   comment */ int  y=2;\n\n"
    assert bench._code_only(src) == "int x = 1; int y=2;"


def test_code_edits_change_the_code_only_form():
    assert bench._code_only("s = fma(a, b, s);") != bench._code_only("s = fma(b, a, s);")
    assert bench._code_only("p + nx") != bench._code_only("p - nx")


def test_sweep_hash_covers_every_sweep_source():
    names = {p.rsplit("/", 1)[-1] for p in bench.SWEEP_SRCS}
    assert {"ntd_sweep.h", "ntd_apply.h", "ntd_apply_multi.h", "ntd_vec.hip"} <= names
    assert len(bench.sweep_hash()) == 16
