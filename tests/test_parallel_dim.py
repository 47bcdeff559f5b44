"""Choice of the parallel dimension of an updated array (Sec. "Division of
Multidimensional Arrays"): the oracle pinned by the paper's NPB-BT example
and hand cases, and the library's helper equal to the oracle."""
import json
import os

import pytest
from hypothesis import given, settings, strategies as st

from oracle import plan as P
from paper_2110_14340_amd import jacc


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "npb_bt_lhsY_parallel_dim.json")


def test_golden_npb_bt_fixture():
    g = json.load(open(GOLDEN))
    par = [sum(1 for it in d if it in g["parallel_iterators"]) for d in g["dims_index_iterators"]]
    seq = [sum(1 for it in d if it in g["sequential_iterators"]) for d in g["dims_index_iterators"]]
    assert P.parallel_dim(par, seq) == g["expected_dim_row_major"]
    assert P.parallel_dim(par, seq, column_major=True) == g["expected_dim_column_major"]
    assert jacc.parallel_dim(par, seq) == g["expected_dim_row_major"]


def test_npb_bt_example_chooses_the_i_dimension():
    # lhsY[n][m][BB][jsize][i][k] inside loops over i, k (parallel) and m, n
    # (sequential): dims 4 and 5 tie; C picks the leftmost, Fortran the rightmost
    par = [0, 0, 0, 0, 1, 1]
    seq = [1, 1, 0, 0, 0, 0]
    assert P.parallel_dim(par, seq) == 4
    assert P.parallel_dim(par, seq, column_major=True) == 5


def test_more_parallel_iterators_win_then_fewer_sequential():
    assert P.parallel_dim([1, 2, 1], [0, 3, 0]) == 1          # a[i][i+k][k]: most parallel
    assert P.parallel_dim([1, 1, 1], [2, 0, 1]) == 1          # tie broken by sequential count
    assert P.parallel_dim([1, 1], [0, 0]) == 0
    assert P.parallel_dim([0, 0, 0], [1, 0, 2]) is None       # no parallel dimension: duplicate


def test_library_helper_cases_and_errors():
    assert jacc.parallel_dim([0, 0, 0, 0, 1, 1], [1, 1, 0, 0, 0, 0]) == 4
    assert jacc.parallel_dim([0, 0, 0, 0, 1, 1], [1, 1, 0, 0, 0, 0], column_major=True) == 5
    assert jacc.parallel_dim([0, 0], [1, 1]) == -1
    with pytest.raises(jacc.JaccError):
        jacc.parallel_dim([1, -1], [0, 0])
    with pytest.raises(jacc.JaccError):
        jacc.parallel_dim([], [])


@settings(max_examples=300, deadline=None)
@given(st.integers(1, 8).flatmap(lambda n: st.tuples(st.lists(st.integers(0, 3), min_size=n, max_size=n),
                                                     st.lists(st.integers(0, 3), min_size=n, max_size=n),
                                                     st.booleans())))
def test_library_matches_oracle(case):
    par, seq, cm = case
    ref = P.parallel_dim(par, seq, cm)
    assert jacc.parallel_dim(par, seq, cm) == (-1 if ref is None else ref)
