"""Cluster tree and block cluster tree of an H^2 matrix (Section II).

The paper fixes a binary cluster tree whose root is level 0, with leaves of at
most `leafsize` indices and 2^l clusters at level l, and a block partition
decided by the strong admissibility condition (equation admCond): a block
(t, s) is admissible when max(diam t, diam s) <= eta * dist(t, s).
Admissible blocks are leaves of the block tree at any level; inadmissible
blocks are only kept as dense leaves at the leaf level; every other block is a
non-leaf block whose four children are the products of the clusters'
children.

Readings where the paper leaves details open:
  * bisection: every cluster of a level is split while ceil(N / 2^l) exceeds
    the leaf size, so all leaves sit at depth L = ceil(log2(N / leafsize));
    the split is at the median along the longest axis of the cluster's tight
    bounding box (ties to the lower axis), after a stable sort by that
    coordinate and then by original index; the first child gets floor(n/2).
  * diam and dist are taken on tight axis-aligned bounding boxes: diam is the
    box diagonal, dist the Euclidean gap between the boxes; a block with a
    zero gap is never admissible.
"""
import numpy as np

R, F, NL = 0, 1, 2
TYPE_NAMES = {R: "R", F: "F", NL: "NL"}


class ClusterTree:
    """Complete binary cluster tree over a point set.

    perm[p] is the original index of the point at tree position p; cluster c
    of level l covers tree positions [start(l, c), stop(l, c)).
    """

    def __init__(self, points, leaf_size):
        pts = np.asarray(points, dtype=np.float64)
        n = pts.shape[0]
        if n < 1 or leaf_size < 1:
            raise ValueError("need at least one point and leaf_size >= 1")
        depth = 0
        while -(-n // (1 << depth)) > leaf_size:
            depth += 1
        perm = np.arange(n, dtype=np.int64)
        ranges = [(0, n)]
        for _ in range(depth):
            nxt = []
            for s, e in ranges:
                idx = perm[s:e]
                p = pts[idx]
                ext = p.max(axis=0) - p.min(axis=0)
                axis = int(np.argmax(ext))
                order = np.lexsort((idx, p[:, axis]))
                perm[s:e] = idx[order]
                m = s + (e - s) // 2
                nxt.append((s, m))
                nxt.append((m, e))
            ranges = nxt
        self.points = pts
        self.n = n
        self.leaf_size = leaf_size
        self.L = depth
        self.perm = perm
        self.leaf_off = np.array([r[0] for r in ranges] + [n], dtype=np.int64)
        # tight bounding boxes per level
        self.lo = []
        self.hi = []
        for lev in range(depth + 1):
            nc = 1 << lev
            lo = np.empty((nc, 3))
            hi = np.empty((nc, 3))
            for c in range(nc):
                s, e = self.start(lev, c), self.stop(lev, c)
                p = pts[perm[s:e]]
                lo[c] = p.min(axis=0)
                hi[c] = p.max(axis=0)
            self.lo.append(lo)
            self.hi.append(hi)

    def start(self, lev, c):
        return int(self.leaf_off[c << (self.L - lev)])

    def stop(self, lev, c):
        return int(self.leaf_off[(c + 1) << (self.L - lev)])

    def size(self, lev, c):
        return self.stop(lev, c) - self.start(lev, c)

    def indices(self, lev, c):
        """Original point indices of cluster c at level lev, in tree order."""
        return self.perm[self.start(lev, c):self.stop(lev, c)]

    def diam(self, lev, c):
        return float(np.linalg.norm(self.hi[lev][c] - self.lo[lev][c]))

    def dist(self, lev, t, s):
        gap = np.maximum(0.0, np.maximum(self.lo[lev][s] - self.hi[lev][t],
                                         self.lo[lev][t] - self.hi[lev][s]))
        return float(np.linalg.norm(gap))


class BlockTree:
    """Block cluster tree: per level, the (row cluster, column cluster, type)
    triples of its nodes, sorted by (row, column)."""

    def __init__(self, tree, eta):
        self.L = tree.L
        self.eta = eta
        self.rows, self.cols, self.types = [], [], []
        cand = [(0, 0)]
        for lev in range(tree.L + 1):
            cand.sort()
            rows, cols, types, nxt = [], [], [], []
            for t, s in cand:
                d = tree.dist(lev, t, s)
                adm = d > 0.0 and max(tree.diam(lev, t), tree.diam(lev, s)) <= eta * d
                if adm:
                    typ = R
                elif lev == tree.L:
                    typ = F
                else:
                    typ = NL
                    for a in (2 * t, 2 * t + 1):
                        for b in (2 * s, 2 * s + 1):
                            nxt.append((a, b))
                rows.append(t)
                cols.append(s)
                types.append(typ)
            self.rows.append(np.array(rows, dtype=np.int64))
            self.cols.append(np.array(cols, dtype=np.int64))
            self.types.append(np.array(types, dtype=np.int8))
            cand = nxt

    @classmethod
    def from_arrays(cls, rows, cols, types, eta=float("nan")):
        self = cls.__new__(cls)
        self.L = len(rows) - 1
        self.eta = eta
        self.rows = [np.asarray(r, dtype=np.int64) for r in rows]
        self.cols = [np.asarray(c, dtype=np.int64) for c in cols]
        self.types = [np.asarray(t, dtype=np.int8) for t in types]
        return self

    def count(self, typ):
        return int(sum(int((t == typ).sum()) for t in self.types))

    def same_as(self, other):
        if self.L != other.L:
            return False
        for lev in range(self.L + 1):
            for a, b in ((self.rows, other.rows), (self.cols, other.cols),
                         (self.types, other.types)):
                if not np.array_equal(a[lev], b[lev]):
                    return False
        return True

    def min_admissible_level(self):
        """Lowest level number that holds an admissible block (L if none)."""
        for lev in range(self.L + 1):
            if (self.types[lev] == R).any():
                return lev
        return self.L

    def sparsity_constant(self):
        """Largest number of blocks any single cluster forms at one level,
        counting row and column roles separately."""
        best = 0
        for lev in range(self.L + 1):
            if self.rows[lev].size:
                best = max(best, int(np.bincount(self.rows[lev]).max()),
                           int(np.bincount(self.cols[lev]).max()))
        return best
