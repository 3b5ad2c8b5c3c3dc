"""Host logic of the per-mode warm start: systems are grouped by harmonic, a
group whose rows are contiguous is passed as a slice, any other as its row
list, and a harmonic without a model is an error (no GPU needed)."""
import numpy as np
import pytest

from paper_2009_06725_amd import scvs


def _routing(models):
    obj = scvs.ModeWarmStarts.__new__(scvs.ModeWarmStarts)
    obj.ws = {k: f"model{k}" for k in models}
    return obj


def test_groups_by_harmonic():
    mw = _routing([1, 2, 3])
    modes = np.array([1, 1, 2, 2, 2, 3])
    got = [(w, rows.tolist(), sl) for w, rows, sl in mw._groups(modes)]
    assert got == [("model1", [0, 1], slice(0, 2)), ("model2", [2, 3, 4], slice(2, 5)),
                   ("model3", [5], slice(5, 6))]


def test_interleaved_rows_are_gathered():
    mw = _routing([1, 2])
    modes = np.array([1, 2, 1, 2])
    got = [(w, rows.tolist(), sl) for w, rows, sl in mw._groups(modes)]
    assert got == [("model1", [0, 2], None), ("model2", [1, 3], None)]
    # every system is routed exactly once
    rows = np.concatenate([r for _, r, _ in mw._groups(modes)])
    assert sorted(rows.tolist()) == [0, 1, 2, 3]


def test_unknown_harmonic_is_an_error():
    mw = _routing([1])
    with pytest.raises(scvs.ScvsError):
        list(mw._groups(np.array([1, 4])))
