"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Nearest-rank percentile: the q-quantile of n values is the value at rank
ceil(q n) (1-based) of the sorted list.
"""
import math


def percentile(values, q):
    v = sorted(values)
    if not v:
        raise ValueError("empty")
    r = max(1, math.ceil(q * len(v)))
    return v[r - 1]
