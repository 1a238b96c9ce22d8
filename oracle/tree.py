"""Binary index tree (Sec. 2.7 "A binary tree structure", Fig. 1).

The root holds ``I_1 = [0, N)``; a node's interval is split into two roughly
equal halves, children of node t are 2t and 2t+1 (Fig. 1 numbering), and
intervals holding more than ``m`` indices keep being split.  Reading taken
where the paper leaves freedom: every leaf sits on the same level
``L = ceil(log2(N/m))`` (the loops "over leaf boxes" and ``A^(L)`` of
Fig. 2/4 assume that), and the left child gets ``ceil(n/2)`` indices.
"""
from __future__ import annotations

import math


class Tree:
    def __init__(self, n: int, leaf: int):
        if n < 1 or leaf < 1:
            raise ValueError("n and leaf size must be positive")
        self.n = n
        self.leaf = leaf
        self.L = 0 if n <= leaf else int(math.ceil(math.log2(n / leaf)))
        size = 2 ** (self.L + 1)
        self.lo = [0] * size
        self.hi = [0] * size
        self.lo[1], self.hi[1] = 0, n
        for t in range(1, 2 ** self.L):
            a, b = self.lo[t], self.hi[t]
            mid = a + (b - a + 1) // 2
            self.lo[2 * t], self.hi[2 * t] = a, mid
            self.lo[2 * t + 1], self.hi[2 * t + 1] = mid, b

    # --- navigation -------------------------------------------------------
    def level_nodes(self, lev: int):
        return range(2 ** lev, 2 ** (lev + 1))

    def leaves(self):
        return self.level_nodes(self.L)

    @staticmethod
    def children(t: int):
        return 2 * t, 2 * t + 1

    @staticmethod
    def sibling(t: int) -> int:
        return t ^ 1

    @staticmethod
    def level(t: int) -> int:
        return t.bit_length() - 1

    def I(self, t: int) -> slice:
        """Index vector I_t as a slice of [0, N)."""
        return slice(self.lo[t], self.hi[t])

    def size(self, t: int) -> int:
        return self.hi[t] - self.lo[t]

    def J(self, child: int) -> slice:
        """Relative positions J_child of I_child inside I_parent (Sec. 4.1)."""
        p = child // 2
        return slice(self.lo[child] - self.lo[p], self.hi[child] - self.lo[p])

    def nmax(self) -> int:
        return max(self.size(t) for t in self.leaves())
