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


def test_paper_model_packed_matches_codes():
    # the packed draw of the Section 2 model is the code-matrix draw, packed
    rows, cols = 203, 517
    M = synth.algorithm1_codes(rows, cols, 10, rows * cols, 0.017, 9)
    g = synth.algorithm1(rows, cols, r=10, rkins=0.017, seed=9)
    assert np.array_equal(synth.pack_codes(M), g.packed)
    assert set(np.unique(M)) <= {0, 1, 2}
    # at most round(rkins rows) rows are copies (a row drawn twice keeps its last source)
    assert 1 <= g.meta["copied_rows"] <= round(0.017 * rows)
    # with nsignal = rows x cols an entry escapes every signal draw with
    # probability (1 - 1/N)^N ~ 1/e; a hit entry is uniform on {0, 1, 2}, so the
    # share of entries equal to 1 is at least (1 - 1/e) / 3
    assert np.mean(M == 1) >= 0.9 * (1 - np.exp(-1)) / 3
