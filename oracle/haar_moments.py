"""Haar frame potential of U(d) by counting permutations.

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

The paper states F_Haar^(k) = k! (Sec. I.A, after the diamond-norm bound).
That holds for d >= k.  In general E_Haar |Tr U|^{2k} over U(d) equals the
number of permutations of k elements whose longest increasing subsequence
has length <= d (Rains 1998; Diaconis-Shahshahani 1994 for d >= k).  The
Supplementary "Validation of sampling Haar random two-qubit unitaries" runs
n = 2, l = 1 (d = 4) at k = 6 and 8, where the count is 694 and 33324, not
720 and 40320.  Both readings are recorded; the count is what is computed.
"""

import itertools
import math


def lis_length(perm):
    """Longest strictly increasing subsequence (patience sorting)."""
    tails = []
    for x in perm:
        lo, hi = 0, len(tails)
        while lo < hi:
            mid = (lo + hi) // 2
            if tails[mid] < x:
                lo = mid + 1
            else:
                hi = mid
        if lo == len(tails):
            tails.append(x)
        else:
            tails[lo] = x
    return len(tails)


def haar_frame_potential(k, d):
    """#{pi in S_k : LIS(pi) <= d} by enumeration (k <= 9 is instant)."""
    if k == 0:
        return 1
    if d >= k:
        return math.factorial(k)
    return sum(1 for p in itertools.permutations(range(k)) if lis_length(p) <= d)
