"""In-memory H^2 matrix (Section II) and its flat interchange format.

An H^2 matrix over a cluster tree stores
  * leaf row bases V_t (#t x k_t) and, for every non-root cluster t', the
    transfer matrix E_t' (k_t' x k_parent) with V_parent restricted to the
    rows of t' equal to V_t' E_t' (the nested property);
  * the same for the column side (W, E^col);
  * a coupling matrix S_ts (k^row_t x k^col_s) for every admissible block,
    which represents V_t S_ts W_s^T;
  * a dense matrix F_ts for every inadmissible leaf block.
Matrices are in tree order (rows and columns permuted by tree.perm).

The flat format lays everything out in one set of arrays so that the C-ABI
library and the CPU checker read the same input:
  n, L, is_complex, leaf_off[2^L+1], perm[n],
  node_off[L+2], node_row[], node_col[], node_type[]   (level-major),
  krow[2^(L+1)-1], kcol[...]                          (cluster (l,c) at 2^l-1+c),
  V / W: leaf bases, column-major, offsets V_off[2^L+1] (in elements),
  Er / Ec: transfers of cluster (l,c), l>=1, at flat cluster index, offsets
           Er_off[2^(L+1)] (root slot empty),
  S: per node (empty unless admissible), offsets S_off[nnodes+1],
  F: per node (empty unless dense), offsets F_off[nnodes+1].
Complex matrices are stored as complex128 (interleaved re, im).
"""
import numpy as np

from .structure import BlockTree, R, F


def cluster_index(lev, c):
    return (1 << lev) - 1 + c


class H2Matrix:
    def __init__(self, tree, blocks, V, Er, W, Ec, S, Fd):
        self.tree = tree
        self.blocks = blocks
        self.V = V      # list over leaf clusters
        self.Er = Er    # list over levels; Er[0] = [None]; Er[l][c] k(l,c) x k(l-1,c//2)
        self.W = W
        self.Ec = Ec
        self.S = S      # list over levels of lists aligned with block nodes
        self.F = Fd     # list aligned with level-L block nodes
        dt = np.result_type(*[v.dtype for v in V]) if V else np.float64
        self.dtype = np.dtype(np.complex128 if np.issubdtype(dt, np.complexfloating)
                              else np.float64)

    @property
    def L(self):
        return self.tree.L

    @property
    def n(self):
        return self.tree.n

    def krow(self, lev, c):
        if lev == self.L:
            return self.V[c].shape[1]
        return self.Er[lev + 1][2 * c].shape[1]

    def kcol(self, lev, c):
        if lev == self.L:
            return self.W[c].shape[1]
        return self.Ec[lev + 1][2 * c].shape[1]

    # ------------------------------------------------------------------ flat
    def to_flat(self):
        L = self.L
        t = self.tree
        cdt = self.dtype
        nclus = (1 << (L + 1)) - 1
        krow = np.zeros(nclus, dtype=np.int64)
        kcol = np.zeros(nclus, dtype=np.int64)
        for lev in range(L + 1):
            for c in range(1 << lev):
                krow[cluster_index(lev, c)] = self.krow(lev, c)
                kcol[cluster_index(lev, c)] = self.kcol(lev, c)

        def pack(mats):
            offs = [0]
            parts = []
            for m in mats:
                if m is None or m.size == 0:
                    offs.append(offs[-1])
                    continue
                parts.append(np.asarray(m, dtype=cdt).ravel(order="F"))
                offs.append(offs[-1] + m.size)
            data = np.concatenate(parts) if parts else np.zeros(0, dtype=cdt)
            return data, np.array(offs, dtype=np.int64)

        def transfers(E):
            mats = [None]
            for lev in range(1, L + 1):
                mats.extend(E[lev])
            return mats

        node_off = [0]
        for lev in range(L + 1):
            node_off.append(node_off[-1] + len(self.blocks.rows[lev]))
        S_all, F_all = [], []
        for lev in range(L + 1):
            S_all.extend(self.S[lev])
            F_all.extend(self.F if lev == L else [None] * len(self.blocks.rows[lev]))
        V, V_off = pack(self.V)
        W, W_off = pack(self.W)
        Er, Er_off = pack(transfers(self.Er))
        Ec, Ec_off = pack(transfers(self.Ec))
        S, S_off = pack(S_all)
        Fd, F_off = pack(F_all)
        return dict(
            n=np.int64(t.n), L=np.int64(L),
            is_complex=np.int64(1 if cdt == np.complex128 else 0),
            leaf_size=np.int64(t.leaf_size), eta=np.float64(self.blocks.eta),
            leaf_off=t.leaf_off.astype(np.int64), perm=t.perm.astype(np.int64),
            node_off=np.array(node_off, dtype=np.int64),
            node_row=np.concatenate(self.blocks.rows).astype(np.int32),
            node_col=np.concatenate(self.blocks.cols).astype(np.int32),
            node_type=np.concatenate(self.blocks.types).astype(np.int32),
            krow=krow, kcol=kcol,
            V=V, V_off=V_off, W=W, W_off=W_off,
            Er=Er, Er_off=Er_off, Ec=Ec, Ec_off=Ec_off,
            S=S, S_off=S_off, F=Fd, F_off=F_off,
        )

    @classmethod
    def from_flat(cls, d, tree=None):
        """Rebuild from the flat format. `tree` may supply a ClusterTree with
        points; otherwise a point-free tree shell is made from leaf_off/perm."""
        L = int(d["L"])
        if tree is None:
            tree = TreeShell(int(d["n"]), L, d["leaf_off"], d["perm"],
                             int(d.get("leaf_size", 0)))
        node_off = d["node_off"]
        rows, cols, types = [], [], []
        for lev in range(L + 1):
            a, b = int(node_off[lev]), int(node_off[lev + 1])
            rows.append(d["node_row"][a:b].astype(np.int64))
            cols.append(d["node_col"][a:b].astype(np.int64))
            types.append(d["node_type"][a:b].astype(np.int8))
        blocks = BlockTree.from_arrays(rows, cols, types, float(d.get("eta", np.nan)))
        krow, kcol = d["krow"], d["kcol"]
        cdt = np.complex128 if int(d["is_complex"]) else np.float64

        def get(data, off, i, r, c):
            a, b = int(off[i]), int(off[i + 1])
            return np.asarray(data[a:b], dtype=cdt).reshape((r, c), order="F").copy()

        def nrows(c):
            return tree.stop(L, c) - tree.start(L, c)

        V = [get(d["V"], d["V_off"], c, nrows(c), int(krow[cluster_index(L, c)]))
             for c in range(1 << L)]
        W = [get(d["W"], d["W_off"], c, nrows(c), int(kcol[cluster_index(L, c)]))
             for c in range(1 << L)]
        Er, Ec = [[None]], [[None]]
        for lev in range(1, L + 1):
            er, ec = [], []
            for c in range(1 << lev):
                i = cluster_index(lev, c)
                p = cluster_index(lev - 1, c // 2)
                er.append(get(d["Er"], d["Er_off"], i, int(krow[i]), int(krow[p])))
                ec.append(get(d["Ec"], d["Ec_off"], i, int(kcol[i]), int(kcol[p])))
            Er.append(er)
            Ec.append(ec)
        S, Fd = [], []
        for lev in range(L + 1):
            sl = []
            for q in range(len(rows[lev])):
                g = int(node_off[lev]) + q
                if types[lev][q] == R:
                    t_, s_ = int(rows[lev][q]), int(cols[lev][q])
                    sl.append(get(d["S"], d["S_off"], g,
                                  int(krow[cluster_index(lev, t_)]),
                                  int(kcol[cluster_index(lev, s_)])))
                else:
                    sl.append(None)
            S.append(sl)
        for q in range(len(rows[L])):
            g = int(node_off[L]) + q
            if types[L][q] == F:
                t_, s_ = int(rows[L][q]), int(cols[L][q])
                Fd.append(get(d["F"], d["F_off"], g, nrows(t_), nrows(s_)))
            else:
                Fd.append(None)
        return cls(tree, blocks, V, Er, W, Ec, S, Fd)

    def save(self, path):
        np.savez(path, **self.to_flat())

    @classmethod
    def load(cls, path):
        with np.load(path, allow_pickle=False) as z:
            d = {k: z[k] for k in z.files}
        return cls.from_flat(d)


class TreeShell:
    """Cluster tree ranges without the point coordinates."""

    def __init__(self, n, L, leaf_off, perm, leaf_size=0):
        self.n = n
        self.L = L
        self.leaf_off = np.asarray(leaf_off, dtype=np.int64)
        self.perm = np.asarray(perm, dtype=np.int64)
        self.leaf_size = leaf_size

    def start(self, lev, c):
        return int(self.leaf_off[c << (self.L - lev)])

    def stop(self, lev, c):
        return int(self.leaf_off[(c + 1) << (self.L - lev)])

    def size(self, lev, c):
        return self.stop(lev, c) - self.start(lev, c)
