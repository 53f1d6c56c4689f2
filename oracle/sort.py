"""Quicksort of the paper's collection API (Section 4, Listing 3), in plain numpy.

The listing sorts a vector by recursion: the pivot is the item at index count // 2 of the
current collection; three filters keep, in order, the items less than, equal to and greater
than the pivot; the result is quicksort(less) followed by the equal items followed by
quicksort(greater) (concatenate, Table 2).  Its postcondition says the result is sorted and has
the input's count.

Readings (the listing as printed does not run as is):
* An empty partition would be passed back into a routine that requires count > 0; an empty
  collection is returned as it is (a second base case next to count = 1).
* Indices are 0-based: the pivot of a collection of count c is the item at position c // 2.
* Comparisons are IEEE comparisons in the element type: an item that is NaN is neither less
  than, equal to nor greater than any pivot, so every filter drops it, and a NaN pivot drops
  its whole collection.  The postcondition count = old count then fails, which is how the
  contract reports such input.
* filter is stable, so items that compare equal (e.g. -0.0 and +0.0) keep their input order.
"""
from __future__ import annotations

import sys

import numpy as np


def quicksort(a: np.ndarray) -> np.ndarray:
    """The listing's recursion on a float32 or int32 vector; returns a new vector."""
    a = np.asarray(a)
    if a.dtype not in (np.float32, np.int32):
        raise TypeError("quicksort sorts float32 or int32 vectors")
    limit = sys.getrecursionlimit()
    sys.setrecursionlimit(max(limit, 20000))
    try:
        return _qs(a)
    finally:
        sys.setrecursionlimit(limit)


def _qs(a: np.ndarray) -> np.ndarray:
    if a.size <= 1:  # count 1: the collection itself; count 0: nothing to sort
        return a.copy()
    pivot = a[a.size // 2]
    with np.errstate(invalid="ignore"):
        left = a[a < pivot]
        mid = a[a == pivot]
        right = a[a > pivot]
    return np.concatenate([_qs(left), mid, _qs(right)]).astype(a.dtype, copy=False)
