"""Accuracy-controlled, structure-preserving H^2 matrix-matrix product
C = A B with change of cluster bases (Ma and Jiao, Sections III and IV).

Plain FP64 / complex128 NumPy, one block at a time, in the paper's order:

  0. cluster-basis products Pi_j = (W^A_j)^T V^B_j, leaf then nested
     (equation nonleafproduct; the paper calls them B_j);
  leaf level L (Section III):
  1. new leaf row basis of C from three normalised Gram sums: dense-dense
     products whose target is admissible at this or an upper level
     (equation Gr1L), F^A_ij V^B_j for every dense block of A in the row
     (Gr2L), and V^A_i V^A_i^H (Gr3L); the column basis from the mirror
     sums (case1-ch, case2-ch, case3-ch); truncation of the summed Gram's
     eigen-decomposition at eps;
  2. projections P^A, P^B (leafproj) and collected blocks (Fcollect);
  3. the products: dense targets exactly, admissible targets through
     leafcoup_simple; targets that lie inside an upper-level admissible
     block of C are kept as temporary couplings ("blue" blocks of Fig. 3);
  non-leaf levels l = L-1 ... l_min (Section IV, the six steps of its
  summary):
  4. collect the four children of each non-leaf block of A and of B, and
     merge the four children's temporary couplings of each admissible or
     blue target (nonleafA);
  5. new transfer matrices from the normalised Grams case1-ch-nl,
     case2-ch-nl, case3-ch-nl and their column mirrors;
  6. projections (nonleafproj) and collected blocks (NLcollect);
  7. the products nonleafcoup_simple, routed to admissible blocks of C, to
     temporary couplings, or to couplings attached to non-leaf blocks;
  8. a top-down split of the couplings attached to non-leaf blocks into the
     admissible and dense blocks below them (end of Section IV).

FIXED mode is the fixed-basis ("formatted") product the paper compares
against (Section I; Table IV, "existing" row): C keeps the row bases of A and
the column bases of B, orthonormalised (each new basis is the numerical
range of the third Gram component alone, eigenvalues above 1e-12 lambda_1),
so no contribution changes the bases and the error of C is not controlled
by eps (which FIXED mode ignores); every other step is the same.

Readings of points the paper leaves open (each also listed in the design
notes): "normalize" divides a Gram sum by its trace and skips empty sums;
"normalized singular values greater than eps" keeps eigenvalues with
lambda_m > tau * lambda_1 where tau = eps in PAPER mode (the Gram's own
singular values, which reproduces the paper's error of about sqrt(eps)) and
tau = (theta*eps/n_t)^2 in ACCURACY mode (the default, aimed at
||C - AB||_F <= eps ||AB||_F): singular values of the stacked normalised
contributions above theta*eps/n_t, where n_t = L - l_min + 1 is the number
of levels whose bases are truncated.  Each level's truncation adds its own
error to C and these errors add up over the levels (measured: the error at
theta*eps per level grows about linearly with n_t), so the budget eps is
split evenly over the levels; theta = 1 was fixed once by
`calibrate_theta.py` on small members of each input family.  At least one
vector is kept; EXACT mode keeps every eigenvector; the non-leaf column
"original basis" term is Q Q^H with Q = diag(P^B_k'^T) T^B_K; blocks enter
the case-1 Gram one product at a time at the leaf level and one merged
target at a time above it; every dense (or non-leaf) block of A in a row
enters the case-2 Gram whatever its target.

Part of the CPU checker: test infrastructure only.
"""
import numpy as np

from h2inputs.h2data import H2Matrix
from h2inputs.structure import R, F, NL

BLUE = 3
EXACT, ACCURACY, PAPER, FIXED = "exact", "accuracy", "paper", "fixed"
THETA = 1.0
# FIXED mode: relative eigenvalue floor of the numerical rank of an old basis
FIXED_TAU = 1e-12


def _h(x):
    return x.conj().T


def truncated_levels(L, lmin):
    """Number of levels whose bases are truncated: the leaves and every
    non-leaf level down to l_min."""
    return max(1, L - lmin + 1)


def threshold(eps, mode, theta=THETA, levels=1):
    """Relative eigenvalue threshold tau (lambda_m > tau * lambda_1 is kept)."""
    if mode == EXACT:
        return None
    if mode == FIXED:
        return FIXED_TAU
    if mode == PAPER:
        return float(eps)
    if mode == ACCURACY:
        return float(theta * eps / levels) ** 2
    raise ValueError(mode)


def truncated_basis(components, tau):
    """Orthonormal basis from normalised Gram components.

    components: list of (Gram sum, trace) with Gram in row-space form
    (Z Z^H).  Each non-empty component is divided by its trace, the results
    are summed, and the eigenvectors of the sum whose eigenvalues exceed
    tau * lambda_1 are returned in descending order (all of them when tau is
    None), at least one."""
    d = components[0][0].shape[0]
    G = np.zeros((d, d), dtype=np.result_type(*[c[0].dtype for c in components]))
    for Gc, tr in components:
        if tr > 0.0:
            G += Gc / tr
    G = 0.5 * (G + _h(G))
    lam, U = np.linalg.eigh(G)
    lam = lam[::-1]
    U = U[:, ::-1]
    if tau is None:
        k = d
    else:
        k = int(np.count_nonzero(lam > tau * lam[0])) if lam[0] > 0 else 1
        k = max(1, min(k, d))
    return np.ascontiguousarray(U[:, :k]), lam


class _Gram:
    """Running Gram sum with its trace; `row` form adds Z Z^H, column form
    adds Z^T Z^*."""

    def __init__(self, d, dtype):
        self.G = np.zeros((d, d), dtype=dtype)
        self.tr = 0.0

    def add_row(self, Z):
        self.G += Z @ _h(Z)
        self.tr += float(np.vdot(Z, Z).real)

    def add_col(self, Z):
        self.G += Z.T @ Z.conj()
        self.tr += float(np.vdot(Z, Z).real)

    def comp(self):
        return (self.G, self.tr)


def _blockdiag(a, b):
    out = np.zeros((a.shape[0] + b.shape[0], a.shape[1] + b.shape[1]),
                   dtype=np.result_type(a, b))
    out[:a.shape[0], :a.shape[1]] = a
    out[a.shape[0]:, a.shape[1]:] = b
    return out


class Symbolic:
    """Per-level node maps, triples and target classes (shared structure of
    A, B and C)."""

    def __init__(self, blocks):
        self.L = blocks.L
        self.nodes = []
        self.brow = []
        for lev in range(self.L + 1):
            d, br = {}, {}
            for q, (i, j, t) in enumerate(zip(blocks.rows[lev], blocks.cols[lev],
                                              blocks.types[lev])):
                d[(int(i), int(j))] = (q, int(t))
                br.setdefault(int(i), []).append((int(j), q, int(t)))
            self.nodes.append(d)
            self.brow.append(br)
        self.lmin = blocks.min_admissible_level()

    def target(self, lev, i, k):
        hit = self.nodes[lev].get((i, k))
        if hit is not None:
            return hit[1], hit[0]
        up, a, b = lev, i, k
        while up > 0:
            up, a, b = up - 1, a >> 1, b >> 1
            hit = self.nodes[up].get((a, b))
            if hit is not None:
                assert hit[1] == R, "a non-node target must lie inside an admissible block"
                return BLUE, -1
        raise AssertionError("target outside the block tree")

    def triples(self, lev):
        """(i, j, k, qa, qb, ta, tb) for every A node (i,j) and B node (j,k)
        of this level that are not both non-leaf."""
        out = []
        for (i, j), (qa, ta) in self.nodes[lev].items():
            for (k, qb, tb) in self.brow[lev].get(j, ()):
                if ta == NL and tb == NL:
                    continue
                out.append((i, j, k, qa, qb, ta, tb))
        out.sort()
        return out


def h2_mmp(A, B, eps, mode=ACCURACY, theta=THETA):
    """C = A B.  Returns (C, info) with info holding the rank profile."""
    if not A.blocks.same_as(B.blocks) or A.n != B.n or \
            not np.array_equal(A.tree.leaf_off, B.tree.leaf_off):
        raise ValueError("A and B must share the cluster tree and block partition")
    if eps < 0:
        raise ValueError("eps must be >= 0")
    if eps == 0 and mode != FIXED:
        mode = EXACT
    fixed = mode == FIXED

    def comps(c1, c2, c3):
        """Gram components entering a new basis: all three, or in FIXED mode
        only the old basis (whose span the new one then equals)."""
        return [c3] if fixed else [c1, c2, c3]
    L = A.L
    T = A.tree
    sym = Symbolic(A.blocks)
    lmin = sym.lmin
    tau = threshold(eps, mode, theta, truncated_levels(L, lmin))
    cdt = np.result_type(A.dtype, B.dtype)

    # ---- step 0: cluster-basis products Pi_j = (W^A_j)^T V^B_j
    Pi = [None] * (L + 1)
    Pi[L] = [A.W[j].T @ B.V[j] for j in range(1 << L)]
    for lev in range(L - 1, -1, -1):
        Pi[lev] = [sum(A.Ec[lev + 1][c].T @ Pi[lev + 1][c] @ B.Er[lev + 1][c]
                       for c in (2 * j, 2 * j + 1)) for j in range(1 << lev)]

    # ---- outputs
    VC = [None] * (1 << L)
    WC = [None] * (1 << L)
    ErC = [[None]] + [[None] * (1 << lev) for lev in range(1, L + 1)]
    EcC = [[None]] + [[None] * (1 << lev) for lev in range(1, L + 1)]
    SC = [[None] * len(A.blocks.rows[lev]) for lev in range(L + 1)]
    SNL = [[None] * len(A.blocks.rows[lev]) for lev in range(L + 1)]
    FC = [None] * len(A.blocks.rows[L])
    for q, t in enumerate(A.blocks.types[L]):
        if t == F:
            r, c = A.blocks.rows[L][q], A.blocks.cols[L][q]
            FC[q] = np.zeros((T.size(L, r), T.size(L, c)), dtype=cdt)
    PA = [None] * (L + 1)
    PB = [None] * (L + 1)
    Ahat = [None] * (L + 1)
    Bhat = [None] * (L + 1)
    Acc = [dict() for _ in range(L + 1)]

    def add_to(store, lev, q, val):
        if store[lev][q] is None:
            store[lev][q] = val.copy()
        else:
            store[lev][q] += val

    def route(lev, i, k, val):
        tg, qc = sym.target(lev, i, k)
        if tg == R:
            add_to(SC, lev, qc, val)
        elif tg == NL:
            add_to(SNL, lev, qc, val)
        elif tg == BLUE:
            if (i, k) in Acc[lev]:
                Acc[lev][(i, k)] += val
            else:
                Acc[lev][(i, k)] = val.copy()
        else:
            raise AssertionError("dense target at a non-leaf level")

    # ================================================================ leaf
    lev = L
    trip = sym.triples(L)
    nl = 1 << L

    def dense_a(q, i, j):
        if A.blocks.types[L][q] == F:
            return A.F[q]
        return A.V[i] @ A.S[L][q] @ A.W[j].T

    def dense_b(q, j, k):
        if B.blocks.types[L][q] == F:
            return B.F[q]
        return B.V[j] @ B.S[L][q] @ B.W[k].T

    # step 1: Gram sums for the new leaf bases
    g1r = [_Gram(T.size(L, c), cdt) for c in range(nl)]
    g1c = [_Gram(T.size(L, c), cdt) for c in range(nl)]
    for (i, j, k, qa, qb, ta, tb) in trip:
        if ta == F and tb == F and sym.target(L, i, k)[0] in (R, BLUE):
            P = A.F[qa] @ B.F[qb]
            g1r[i].add_row(P)
            g1c[k].add_col(P)
    g2r = [_Gram(T.size(L, c), cdt) for c in range(nl)]
    g2c = [_Gram(T.size(L, c), cdt) for c in range(nl)]
    for (i, j), (q, t) in sym.nodes[L].items():
        if t == F:
            g2r[i].add_row(A.F[q] @ B.V[j])
    for (j, k), (q, t) in sym.nodes[L].items():
        if t == F:
            g2c[k].add_col(A.W[j].T @ B.F[q])
    for c in range(nl):
        g3r = _Gram(T.size(L, c), cdt)
        g3r.add_row(A.V[c])
        VC[c], _ = truncated_basis(comps(g1r[c].comp(), g2r[c].comp(), g3r.comp()), tau)
        g3c = _Gram(T.size(L, c), cdt)
        g3c.add_row(B.W[c])          # enters as W^B_k (W^B_k)^H
        WC[c], _ = truncated_basis(comps(g1c[c].comp(), g2c[c].comp(), g3c.comp()), tau)

    # step 2: projections and collected blocks
    PA[L] = [_h(VC[i]) @ A.V[i] for i in range(nl)]
    PB[L] = [B.W[k].T @ WC[k].conj() for k in range(nl)]
    Ahat[L] = [None] * len(A.blocks.rows[L])
    Bhat[L] = [None] * len(A.blocks.rows[L])
    for (i, j), (q, t) in sym.nodes[L].items():
        if t == F:
            Ahat[L][q] = _h(VC[i]) @ A.F[q] @ B.V[j]
            Bhat[L][q] = A.W[i].T @ B.F[q] @ WC[j].conj()
        else:
            Ahat[L][q] = PA[L][i] @ A.S[L][q] @ Pi[L][j]
            Bhat[L][q] = Pi[L][i] @ B.S[L][q] @ PB[L][j]

    # step 3: products
    for (i, j, k, qa, qb, ta, tb) in trip:
        tg, qc = sym.target(L, i, k)
        if tg == F:
            FC[qc] += dense_a(qa, i, j) @ dense_b(qb, j, k)
            continue
        if ta == F and tb == F:
            val = (_h(VC[i]) @ A.F[qa]) @ (B.F[qb] @ WC[k].conj())
        elif ta == F:
            val = Ahat[L][qa] @ B.S[L][qb] @ PB[L][k]
        elif tb == F:
            val = PA[L][i] @ A.S[L][qa] @ Bhat[L][qb]
        else:
            val = PA[L][i] @ A.S[L][qa] @ Pi[L][j] @ B.S[L][qb] @ PB[L][k]
        route(L, i, k, val)

    # ============================================================ non-leaf
    def stack2(E, lev, c):
        return np.vstack([E[lev + 1][2 * c], E[lev + 1][2 * c + 1]])

    for lev in range(L - 1, lmin - 1, -1):
        ch = lev + 1
        kr = [VC[c].shape[1] if ch == L else ErC[ch + 1][2 * c].shape[1]
              for c in range(1 << ch)]
        kc = [WC[c].shape[1] if ch == L else EcC[ch + 1][2 * c].shape[1]
              for c in range(1 << ch)]

        def acoll(i, j):
            rows = []
            for a in (2 * i, 2 * i + 1):
                rows.append(np.hstack([Ahat[ch][sym.nodes[ch][(a, b)][0]]
                                       for b in (2 * j, 2 * j + 1)]))
            return np.vstack(rows)

        def bcoll(j, k):
            rows = []
            for a in (2 * j, 2 * j + 1):
                rows.append(np.hstack([Bhat[ch][sym.nodes[ch][(a, b)][0]]
                                       for b in (2 * k, 2 * k + 1)]))
            return np.vstack(rows)

        def merged(i, k):
            rows = []
            for a in (2 * i, 2 * i + 1):
                row = []
                for b in (2 * k, 2 * k + 1):
                    v = Acc[ch].get((a, b))
                    row.append(v if v is not None else np.zeros((kr[a], kc[b]), dtype=cdt))
                rows.append(np.hstack(row))
            return np.vstack(rows)

        # step 4: merged children couplings of admissible / blue targets
        case1 = sorted({(a >> 1, b >> 1) for (a, b) in Acc[ch]})
        M = {}
        for (i, k) in case1:
            tg, _ = sym.target(lev, i, k)
            assert tg in (R, BLUE)
            M[(i, k)] = merged(i, k)

        # step 5: new transfer matrices
        ncl = 1 << lev
        Kr = [kr[2 * c] + kr[2 * c + 1] for c in range(ncl)]
        Kc = [kc[2 * c] + kc[2 * c + 1] for c in range(ncl)]
        g1r = [_Gram(Kr[c], cdt) for c in range(ncl)]
        g1c = [_Gram(Kc[c], cdt) for c in range(ncl)]
        for (i, k), m in M.items():
            g1r[i].add_row(m)
            g1c[k].add_col(m)
        g2r = [_Gram(Kr[c], cdt) for c in range(ncl)]
        g2c = [_Gram(Kc[c], cdt) for c in range(ncl)]
        Acol = {}
        Bcol = {}
        for (i, j), (q, t) in sym.nodes[lev].items():
            if t == NL:
                Acol[q] = acoll(i, j)
                g2r[i].add_row(Acol[q] @ stack2(B.Er, lev, j))
                Bcol[q] = bcoll(i, j)
                g2c[j].add_col(stack2(A.Ec, lev, i).T @ Bcol[q])
        TCr = [None] * ncl
        TCc = [None] * ncl
        for c in range(ncl):
            g3r = _Gram(Kr[c], cdt)
            g3r.add_row(_blockdiag(PA[ch][2 * c], PA[ch][2 * c + 1]) @ stack2(A.Er, lev, c))
            TCr[c], _ = truncated_basis(comps(g1r[c].comp(), g2r[c].comp(), g3r.comp()), tau)
            g3c = _Gram(Kc[c], cdt)
            Q = _blockdiag(PB[ch][2 * c].T, PB[ch][2 * c + 1].T) @ stack2(B.Ec, lev, c)
            g3c.add_row(Q)            # enters as Q Q^H
            TCc[c], _ = truncated_basis(comps(g1c[c].comp(), g2c[c].comp(), g3c.comp()), tau)
            ErC[ch][2 * c] = TCr[c][:kr[2 * c]]
            ErC[ch][2 * c + 1] = TCr[c][kr[2 * c]:]
            EcC[ch][2 * c] = TCc[c][:kc[2 * c]]
            EcC[ch][2 * c + 1] = TCc[c][kc[2 * c]:]

        # step 6: projections and collected blocks
        PA[lev] = [_h(TCr[c]) @ _blockdiag(PA[ch][2 * c], PA[ch][2 * c + 1])
                   @ stack2(A.Er, lev, c) for c in range(ncl)]
        PB[lev] = [stack2(B.Ec, lev, c).T @ _blockdiag(PB[ch][2 * c], PB[ch][2 * c + 1])
                   @ TCc[c].conj() for c in range(ncl)]
        Ahat[lev] = [None] * len(A.blocks.rows[lev])
        Bhat[lev] = [None] * len(A.blocks.rows[lev])
        for (i, j), (q, t) in sym.nodes[lev].items():
            if t == NL:
                Ahat[lev][q] = _h(TCr[i]) @ Acol[q] @ stack2(B.Er, lev, j)
                Bhat[lev][q] = stack2(A.Ec, lev, i).T @ Bcol[q] @ TCc[j].conj()
            elif t == R:
                Ahat[lev][q] = PA[lev][i] @ A.S[lev][q] @ Pi[lev][j]
                Bhat[lev][q] = Pi[lev][i] @ B.S[lev][q] @ PB[lev][j]

        # step 7: products of this level
        for (i, j, k, qa, qb, ta, tb) in sym.triples(lev):
            if ta == NL:
                val = Ahat[lev][qa] @ B.S[lev][qb] @ PB[lev][k]
            elif tb == NL:
                val = PA[lev][i] @ A.S[lev][qa] @ Bhat[lev][qb]
            else:
                val = PA[lev][i] @ A.S[lev][qa] @ Pi[lev][j] @ B.S[lev][qb] @ PB[lev][k]
            route(lev, i, k, val)
        for (i, k), m in M.items():
            route(lev, i, k, _h(TCr[i]) @ m @ TCc[k].conj())

    # ================================================ step 8: top-down split
    for lev in range(lmin, L):
        ch = lev + 1
        for (i, k), (q, t) in sym.nodes[lev].items():
            if t != NL or SNL[lev][q] is None:
                continue
            S = SNL[lev][q]
            for a in (2 * i, 2 * i + 1):
                for b in (2 * k, 2 * k + 1):
                    qq, tt = sym.nodes[ch][(a, b)]
                    Y = ErC[ch][a] @ S @ EcC[ch][b].T
                    if tt == R:
                        add_to(SC, ch, qq, Y)
                    elif tt == NL:
                        add_to(SNL, ch, qq, Y)
                    else:
                        FC[qq] += VC[a] @ Y @ WC[b].T

    # ================================================ assemble C
    # above l_min no admissible block of C needs a basis: rank zero there
    def rank_r(lev, c):
        if lev == L:
            return VC[c].shape[1]
        return ErC[lev + 1][2 * c].shape[1] if lev >= lmin else 0

    def rank_c(lev, c):
        if lev == L:
            return WC[c].shape[1]
        return EcC[lev + 1][2 * c].shape[1] if lev >= lmin else 0

    for lev in range(1, lmin + 1):
        for c in range(1 << lev):
            ErC[lev][c] = np.zeros((rank_r(lev, c), 0), dtype=cdt)
            EcC[lev][c] = np.zeros((rank_c(lev, c), 0), dtype=cdt)
    for lev in range(L + 1):
        for q, t in enumerate(A.blocks.types[lev]):
            if t == R and SC[lev][q] is None:
                i, k = int(A.blocks.rows[lev][q]), int(A.blocks.cols[lev][q])
                SC[lev][q] = np.zeros((rank_r(lev, i), rank_c(lev, k)), dtype=cdt)
    C = H2Matrix(A.tree, A.blocks, VC, ErC, WC, EcC, SC, FC)
    ranks_r = [[C.krow(lev, c) for c in range(1 << lev)] for lev in range(L + 1)]
    ranks_c = [[C.kcol(lev, c) for c in range(1 << lev)] for lev in range(L + 1)]
    info = dict(lmin=lmin, tau=tau, mode=mode, ranks_row=ranks_r, ranks_col=ranks_c)
    return C, info
