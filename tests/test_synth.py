"""The seeded generator draws the same bytes whether a matrix is drawn at once
or in column ranges (the large workloads are drawn in ranges with progress)."""
import numpy as np

import synth


def test_column_ranges_reproduce_the_whole_draw(monkeypatch):
    whole = synth.config("c5", n=301, p=1237)
    monkeypatch.setattr(synth, "PROGRESS_COLUMNS", 100)
    seen = []
    chunked = synth.config("c5", n=301, p=1237, progress=seen.append)
    assert np.array_equal(whole.packed, chunked.packed)
    assert len(seen) == 13 and seen[-1].startswith("[synth] 1,237 of 1,237")


def test_ranges_with_padding_and_relatedness(monkeypatch):
    a = synth.config("c2", n=203, p=901, pad_mode=-1)
    monkeypatch.setattr(synth, "PROGRESS_COLUMNS", 77)
    b = synth.config("c2", n=203, p=901, pad_mode=-1, progress=lambda m: None)
    assert np.array_equal(a.packed, b.packed)
