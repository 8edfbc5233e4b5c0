"""Integer enumeration of the ACE product-basis index list.

Each basis function is one row of six int32 (n1, l1, n2, l2, n3, l3), with -1 in
unused slots:
  order 1: (n, 0, -1, -1, -1, -1)
  order 2: (n1, l, n2, l, -1, -1) with n1 <= n2
  order 3: (n1, l1, n2, l2, n3, l3) with (n1,l1) <= (n2,l2) <= (n3,l3)
           lexicographically, |l1-l2| <= l3 <= l1+l2 and l1+l2+l3 even.
Rows are ordered by order, then lexicographically by the tuple.
"""
import numpy as np


def ace_basis(n_max, l_max, n1_cap=None, n2_cap=None, l2_cap=None, n3_cap=None, l3_cap=None):
    """Return the int32 array [n_funcs, 6]. Caps restrict n (exclusive) and l (inclusive)
    per body order; None means n_max / l_max."""
    n1_cap = n_max if n1_cap is None else n1_cap
    n2_cap = n_max if n2_cap is None else n2_cap
    n3_cap = n_max if n3_cap is None else n3_cap
    l2_cap = l_max if l2_cap is None else l2_cap
    l3_cap = l_max if l3_cap is None else l3_cap
    rows = []
    for n in range(n1_cap):
        rows.append((n, 0, -1, -1, -1, -1))
    for l in range(l2_cap + 1):
        for n1 in range(n2_cap):
            for n2 in range(n1, n2_cap):
                rows.append((n1, l, n2, l, -1, -1))
    ch = sorted((n, l) for n in range(n3_cap) for l in range(l3_cap + 1))
    o3 = []
    for a in range(len(ch)):
        for b in range(a, len(ch)):
            for c in range(b, len(ch)):
                (n1, l1), (n2, l2), (n3, l3) = ch[a], ch[b], ch[c]
                if (l1 + l2 + l3) % 2 or not (abs(l1 - l2) <= l3 <= l1 + l2):
                    continue
                o3.append((n1, l1, n2, l2, n3, l3))
    rows.extend(o3)
    return np.array(rows, dtype=np.int32).reshape(-1, 6)


def basis_counts(func_nl):
    """(order-1, order-2, order-3) row counts of a basis index list."""
    f = np.asarray(func_nl)
    o1 = int(((f[:, 2] < 0)).sum())
    o3 = int((f[:, 4] >= 0).sum())
    return o1, len(f) - o1 - o3, o3
