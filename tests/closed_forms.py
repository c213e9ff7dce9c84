"""Closed forms used by the tests (each pinned against brute force in tests/test_oracle.py)."""
from math import comb

import numpy as np

import graphgen as gg

# complement pairs of Table 1 (graphlet id -> id of its complement)
COMPLEMENT = {1: 2, 2: 1, 3: 6, 6: 3, 4: 5, 5: 4, 7: 17, 17: 7, 8: 16, 16: 8, 9: 15, 15: 9,
              10: 14, 14: 10, 11: 13, 13: 11, 12: 12}


def cocktail_party(k):
    """K_k minus a perfect matching (2i, 2i+1), k even: every vertex has degree k - 2."""
    iu = np.triu_indices(k, 1)
    keep = ~((iu[1] == iu[0] + 1) & (iu[0] % 2 == 0))
    return gg.csr_from_pairs(k, iu[0][keep], iu[1][keep])


def cocktail_party_counts(k):
    """(X1..X17, the 13 per-edge counts shared by every edge) of cocktail_party(k).
    Globals through the complement, a perfect matching of p = k/2 edges: it has p edges,
    p(k - 2) single-edge triples, C(p, 2) 2K2 quadruples and p (C(k-2, 2) - (p - 1))
    quadruples holding exactly one matching edge.  Per edge (u, v): T is everything but u, v
    and their mates (t = k - 4), S_u = {mate of v}, S_v = {mate of u}, D is empty, the edges
    inside T number C(t, 2) - t/2, each mate is adjacent to all of T, and the mates are
    adjacent to each other."""
    p = k // 2
    Xc = [0] * 18
    Xc[1] = p
    Xc[2] = comb(k, 2) - p
    Xc[5] = p * (k - 2)
    Xc[6] = comb(k, 3) - p * (k - 2)
    Xc[14] = comb(p, 2)
    Xc[16] = p * (comb(k - 2, 2) - (p - 1))
    Xc[17] = comb(k, 4) - Xc[14] - Xc[16]
    X = [Xc[COMPLEMENT[i]] for i in range(1, 18)]
    t = k - 4
    K = comb(t, 2) - t // 2
    per_edge = [t, 2, 0, K, comb(t, 2) - K + 2 * t, 0, 1, 0, 0, 0, 0, 0, 0]
    return X, per_edge
