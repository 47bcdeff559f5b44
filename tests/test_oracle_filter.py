"""Pins of the oracle of the paper's predicate-filtering example (Sec.
"Predicate-Based Filtering", Fig. conv-code): the plain statement chain and
its K-replica filtered form.

* Two hand-worked cases on a of 8 and b of 6 elements split in two (owner
  blocks a: [0,4) [4,8), b: [0,3) [3,6)), whose only element in b's block but
  not in a's is 3.  Case 1 writes a[3] from partition 1 only because b[3]
  reads it (the closure of a's write guard); case 2 reads c on partition 1
  only because b[3] depends on it (the closure of the read guard).  Dropping
  either closure changes the gathered b[3].
* The chain evaluated statement by statement over all iterations at once
  (numpy fancy indexing), equal to the sequential chain because no element is
  touched by two iterations.
* The filtered K-replica run equals the plain run for many K, uneven block
  sizes and skipped iterations.
* The aliased chain (a and b one array) against its hand-derived effect.
"""
import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import inputs


def _hand_case(i, j, k, x):
    a = np.arange(8, dtype=np.float64) - 10.0
    b = np.arange(6, dtype=np.float64) - 20.0
    c = np.arange(10, dtype=np.float64) * 100.0
    idx = np.array([[i, j, k]], dtype=np.int32)
    xs = np.array([x])
    return a, b, c, idx, xs


def test_hand_case_closure_of_the_write_guard():
    # t: i=3, j=2, k=5, x=7.  Plain: a[3]=7, b[3]=7, x=c[2]=200, a[5]=200, b[5]=200.
    a, b, c, idx, xs = _hand_case(3, 2, 5, 7.0)
    want_a, want_b = a.copy(), b.copy()
    want_a[3], want_b[3], want_a[5], want_b[5] = 7.0, 7.0, 200.0, 200.0
    for fn in (lambda: oracle.pred_chain(a, b, c, idx, xs), lambda: oracle.pred_chain_partitioned(a, b, c, idx, xs, 2)):
        ra, rb = fn()
        assert np.array_equal(ra, want_a) and np.array_equal(rb, want_b)
    # partition 1 (a: [4,8), b: [3,6)) sees i=3 only in b's block: a[3] = 7
    # must still be written there, else the gathered b[3] would be a's old -7
    ra, rb = oracle.pred_chain_partitioned(a, b, c, idx, xs, 2)
    assert rb[3] == 7.0 and a[3] == -7.0


def test_hand_case_closure_of_the_read_guard():
    # t: i=0, j=6, k=3, x=5.  Plain: a[0]=5, b[0]=5, x=c[6]=600, a[3]=600, b[3]=600.
    a, b, c, idx, xs = _hand_case(0, 6, 3, 5.0)
    want_a, want_b = a.copy(), b.copy()
    want_a[0], want_b[0], want_a[3], want_b[3] = 5.0, 5.0, 600.0, 600.0
    for K in (1, 2):
        ra, rb = oracle.pred_chain_partitioned(a, b, c, idx, xs, K)
        assert np.array_equal(ra, want_a) and np.array_equal(rb, want_b), K
    ra, rb = oracle.pred_chain(a, b, c, idx, xs)
    assert np.array_equal(ra, want_a) and np.array_equal(rb, want_b)
    # k=3 lies only in b's block on partition 1: c[6] must be read there
    # (x would be 0 otherwise and the gathered b[3] 0)


def _vectorised(a, b, c, idx, xs):
    a, b = a.copy(), b.copy()
    nab = min(a.size, b.size)
    i, j, k = (idx[:, n].astype(np.int64) for n in range(3))
    ok = (i >= 0) & (i < nab) & (k >= 0) & (k < nab) & (j >= 0) & (j < c.size)
    i, j, k, x = i[ok], j[ok], k[ok], xs[ok]
    a[i] = x
    b[i] = a[i]
    x = c[j]
    a[k] = x
    b[k] = a[k]
    return a, b


@pytest.mark.parametrize("na,nb,nc,T,skipped", [(100, 100, 50, 40, 0), (1000, 700, 333, 300, 9), (64, 200, 7, 31, 5)])
def test_plain_chain_equals_statementwise_evaluation(na, nb, nc, T, skipped):
    a, b, c, idx, xs = inputs.pred_chain_inputs(na, nb, nc, T, seed=na + T, skipped=skipped)
    ra, rb = oracle.pred_chain(a, b, c, idx, xs)
    va, vb = _vectorised(a, b, c, idx, xs)
    assert np.array_equal(ra, va) and np.array_equal(rb, vb)
    # iterations with an out-of-range index change nothing
    sa, sb = oracle.pred_chain(a, b, c, idx[skipped:], xs[skipped:])
    assert np.array_equal(ra, sa) and np.array_equal(rb, sb)


@pytest.mark.parametrize("na,nb,T", [(1000, 700, 300), (701, 1000, 333), (97, 64, 30), (8, 6, 3)])
def test_filtered_replicas_equal_plain_run(na, nb, T):
    a, b, c, idx, xs = inputs.pred_chain_inputs(na, nb, 50, T, seed=T, skipped=4)
    ra, rb = oracle.pred_chain(a, b, c, idx, xs)
    for K in (1, 2, 3, 5, 6):
        pa, pb = oracle.pred_chain_partitioned(a, b, c, idx, xs, K)
        assert np.array_equal(pa, ra) and np.array_equal(pb, rb), K
    pa, pb = oracle.pred_chain_partitioned(a, b, c, idx, xs, 3, rows=(10, T - 5))
    qa, qb = oracle.pred_chain(a, b, c, idx, xs, rows=(10, T - 5))
    assert np.array_equal(pa, qa) and np.array_equal(pb, qb)


def test_aliased_chain():
    """a and b one array: a[i] = x, then a[i] = a[i], x = c[j], a[k] = x,
    a[k] = a[k] — the effect is a[i] = xs[t] and a[k] = c[j]."""
    a, _, c, idx, xs = inputs.pred_chain_inputs(500, 500, 40, 120, seed=3, skipped=6)
    ra, rb = oracle.pred_chain(a, a, c, idx, xs)
    assert ra is rb
    want = a.copy()
    for t in range(xs.size):
        i, j, k = (int(v) for v in idx[t])
        if 0 <= i < a.size and 0 <= k < a.size and 0 <= j < c.size:
            want[i] = xs[t]
            want[k] = c[j]
    assert np.array_equal(ra, want)
