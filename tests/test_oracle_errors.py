"""The oracle refuses a matrix without full column rank where the paper's
assumption (Section 1: A has full column rank) fails: the scaling QR of an
interface holding two identical columns is numerically rank deficient."""
import numpy as np
import pytest

from oracle import spaqr as osp
from rankdef import duplicated_column_problem


def test_duplicated_column_is_rank_deficient():
    p, j1, j2 = duplicated_column_problem()
    A = p.dense()
    assert np.array_equal(A[:, j1], A[:, j2]) and np.abs(A[:, j1]).sum() > 0
    assert (np.abs(A) > 0).any(axis=0).all()          # every column still has a nonzero
    an = osp.analyze(p, 4)
    with pytest.raises(osp.SpaqrError, match="rank deficient"):
        osp.factorize(an, 1e-2, 1)


def test_full_rank_twin_is_accepted():
    # the same construction without the copy factorizes (control)
    from synth import grid_ls
    p = grid_ls((32, 32), 1024, 0)
    osp.factorize(osp.analyze(p, 4), 1e-2, 1)
