"""Algorithmic work of the H^2 matrix-matrix product at the actual ranks,
counted from the structure and the ranks of A, B and C (Sections III and IV):

  triple  one contraction per evaluated block product (an A node (I,J) and a
          B node (J,K) of one level, not both non-leaf): 2 n_i n_j n_k for a
          dense target (Section III-A); for an admissible or temporary
          target, at the leaves (equation leafcoup_simple)
            dense x dense          2 kC_i n_j kC_k   (V^C_i^H F^A_ij)(F^B_jk W^C_k)
            dense x admissible     2 kC_i kB_j kB_k  Ahat_ij S^B_jk
            admissible x dense     2 kA_i kA_j kC_k  S^A_ij Bhat_jk
            admissible x admiss.   2 kA_i kB_j kB_k  (S^A_ij Pi_j) S^B_jk
          and above them (equation nonleafcoup_simple, the per-target
          projection applied once)
            non-leaf x admissible  2 kC_I kB_J kB_K  Ahat_IJ S^B_JK
            admissible x any       2 kA_I kA_J kC_K  S^A_IJ Bhat_JK;
  target  per target the products that apply the projections: X2 P^B,
          P^A X3 and P^A (X4 P^B) at the leaves, W P^B and P^A W above
          them, and T^C_I^H M_IK T^C_K for a merged target (case 1);
  gram    2 d^2 per column contributed to a row or column Gram sum of
          dimension d (Gr1L, Gr2L, Gr3L, case1-ch ... case3-ch-nl);
  eig     9 d^3 per Gram matrix.
Complex products count four real ones (eight for the eigen-decompositions,
which run on the real embedding of twice the dimension).  Plain Python over
the oracle's symbolic phase.

Part of the CPU checker: test infrastructure only.
"""
from h2inputs.structure import F, NL

from .mmp import BLUE, Symbolic


def flop_counts(A, B, info):
    """dict(triple, target, gram, eig, total) for C = A B with the ranks of C
    in `info` (as returned by oracle.mmp.h2_mmp)."""
    sym = Symbolic(A.blocks)
    L, lmin = A.L, info["lmin"]
    cr, cc = info["ranks_row"], info["ranks_col"]
    t = A.tree

    def n(c):
        return t.size(L, c)

    out = dict(triple=0.0, target=0.0, gram=0.0, eig=0.0)
    acc = set()
    for lev in range(L, lmin - 1, -1):
        ncl = 1 << lev
        ar = [A.krow(lev, c) for c in range(ncl)]
        ac = [A.kcol(lev, c) for c in range(ncl)]
        br = [B.krow(lev, c) for c in range(ncl)]
        bc = [B.kcol(lev, c) for c in range(ncl)]
        if lev == L:
            dr = [n(c) for c in range(ncl)]
            dc = list(dr)
        else:
            dr = [cr[lev + 1][2 * c] + cr[lev + 1][2 * c + 1] for c in range(ncl)]
            dc = [cc[lev + 1][2 * c] + cc[lev + 1][2 * c + 1] for c in range(ncl)]
        rcols = list(ar)     # old row bases (Gr3L, case3-ch-nl)
        ccols = list(bc)
        for (i, j), (q, typ) in sym.nodes[lev].items():
            if typ in (F, NL):
                rcols[i] += br[j]    # F^A_ij V^B_j / Acoll_IJ T^B_J
                ccols[j] += ac[i]    # mirror on B's node (i, j)
        case1 = {(a >> 1, b >> 1) for (a, b) in acc} if lev < L else set()
        nxt = set()
        flags = {}
        for (i, j, k, qa, qb, ta, tb) in sym.triples(lev):
            tg, _ = sym.target(lev, i, k)
            if tg == F:
                out["triple"] += 2.0 * n(i) * n(j) * n(k)
                continue
            if tg == BLUE:
                nxt.add((i, k))
            bit = 0
            if lev == L:
                if ta == F and tb == F:
                    out["triple"] += 2.0 * cr[lev][i] * n(j) * cc[lev][k]
                    rcols[i] += n(k)
                    ccols[k] += n(i)
                elif ta == F:
                    out["triple"] += 2.0 * cr[lev][i] * br[j] * bc[k]
                    bit = 1
                elif tb == F:
                    out["triple"] += 2.0 * ar[i] * ac[j] * cc[lev][k]
                    bit = 2
                else:
                    out["triple"] += 2.0 * ar[i] * br[j] * bc[k]
                    bit = 4
            elif ta == NL:
                out["triple"] += 2.0 * cr[lev][i] * br[j] * bc[k]
                bit = 1
            else:
                out["triple"] += 2.0 * ar[i] * ac[j] * cc[lev][k]
                bit = 2
            if bit:
                flags[(i, k)] = flags.get((i, k), 0) | bit
        for (i, k), b in flags.items():
            if b & 1:
                out["target"] += 2.0 * cr[lev][i] * bc[k] * cc[lev][k]
            if b & 4:
                out["target"] += 2.0 * ar[i] * bc[k] * cc[lev][k]
            if b & 6:
                out["target"] += 2.0 * cr[lev][i] * ar[i] * cc[lev][k]
        for (i, k) in case1:
            out["target"] += 2.0 * cr[lev][i] * dr[i] * dc[k] + 2.0 * cr[lev][i] * dc[k] * cc[lev][k]
            rcols[i] += dc[k]
            ccols[k] += dr[i]
            if sym.nodes[lev].get((i, k)) is None:
                nxt.add((i, k))
        for c in range(ncl):
            out["gram"] += 2.0 * dr[c] ** 2 * rcols[c] + 2.0 * dc[c] ** 2 * ccols[c]
            out["eig"] += 9.0 * (dr[c] ** 3 + dc[c] ** 3)
        acc = nxt
    if A.dtype.kind == "c":
        for key in ("triple", "target", "gram"):
            out[key] *= 4.0
        out["eig"] *= 8.0
    out["total"] = out["triple"] + out["target"] + out["gram"] + out["eig"]
    return out
