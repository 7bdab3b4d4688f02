"""Recompression of an input H^2 matrix: new orthonormal nested bases of
the smallest ranks that keep each cluster's whole far field to a relative
accuracy, with the couplings projected onto them.  The partition and the
dense leaf blocks stay as they are.

The paper builds its inputs with a construction it cites but does not
describe (Section VI); this is a standard algebraic H^2 compression, written
here from its definition:

  * far field of a row cluster t: every admissible block (t', s) with t'
    equal to t or one of its ancestors, restricted to the rows of t.  In the
    nested bases that block row is V_t Z_t, and its Gram matrix is
    V_t K_t V_t^H with the weight
        K_t = sum_{(t,s) admissible} S_ts (W_s^T W_s^*) S_ts^H
              + E_t K_parent(t) E_t^H,
    the column-basis Grams W_s^T W_s^* taken through the transfers;
  * leaves: the new basis is the dominant eigenvectors of V_t K_t V_t^H;
    P_t = V'_t^H V_t maps old coefficients to new ones;
  * above the leaves (up to l_min): the old basis of t written in the
    children's new bases is Z_t = [P_t1 E_t1; P_t2 E_t2]; the new stacked
    transfer [E'_t1; E'_t2] is the dominant eigenvectors of
    Z_t K_t Z_t^H and P_t = [E'_t1; E'_t2]^H Z_t;
  * the column side is the row side of the transpose (bases W, transfers
    E^col, couplings S_ts^T, other-side Grams V_t^T V_t^*);
  * new couplings S'_ts = P^row_t S_ts (P^col_s)^T.

Truncation follows the product's ACCURACY reading: eigenvalues above
(theta eps / n_t)^2 lambda_1 of each Gram are kept (at least one vector),
n_t = L - l_min + 1 truncated levels, and never more than the old rank
(the far field lies in the old basis' span, so further directions are
rounding noise).  The eigenvalues of a Gram matrix are the squared singular
values of the far field, so FP64 resolves singular values down to about
1e-8 of the largest: eps below EPS_FLOOR = 1e-8 is rejected.  Levels above
l_min carry no basis (rank zero), as in a product.  Plain FP64 / complex128
NumPy.

Part of the CPU checker: test infrastructure only.
"""
import numpy as np

from h2inputs.h2data import H2Matrix
from h2inputs.structure import R
from .mmp import ACCURACY, THETA, threshold, truncated_basis, truncated_levels

EPS_FLOOR = 1e-8


def _h(x):
    return x.conj().T


def basis_grams(X, E, L):
    """G[l][c] = X_t^T X_t^* of the expanded bases, through the nested
    property: G_parent = sum_children E_c^T G_c E_c^*."""
    G = [None] * (L + 1)
    G[L] = [x.T @ x.conj() for x in X]
    for lev in range(L - 1, -1, -1):
        G[lev] = [E[lev + 1][2 * c].T @ G[lev + 1][2 * c] @ E[lev + 1][2 * c].conj()
                  + E[lev + 1][2 * c + 1].T @ G[lev + 1][2 * c + 1] @ E[lev + 1][2 * c + 1].conj()
                  for c in range(1 << lev)]
    return G


def far_field_weights(E, couplings, other, L, lmin, ranks, dtype):
    """K[l][t] for l >= l_min, top-down: the cluster's own admissible blocks
    S (other Gram) S^H plus the parent's weight carried down by E_t."""
    K = [None] * (L + 1)
    for lev in range(lmin, L + 1):
        Kl = []
        for t in range(1 << lev):
            k = ranks(lev, t)
            if lev > lmin:
                Et = E[lev][t]
                Kl.append(Et @ K[lev - 1][t // 2] @ _h(Et))
            else:
                Kl.append(np.zeros((k, k), dtype=dtype))
        for t, s, S in couplings[lev]:
            Kl[t] = Kl[t] + S @ other[lev][s] @ _h(S)
        K[lev] = Kl
    return K


def new_side(X, E, couplings, other, L, lmin, tau, ranks, dtype):
    """New leaf bases, transfers (levels l_min+1 .. L) and coefficient maps
    P[l][t] of one side."""
    K = far_field_weights(E, couplings, other, L, lmin, ranks, dtype)
    Xn = [None] * (1 << L)
    En = [[None] * (1 << lev) for lev in range(L + 1)]
    P = [None] * (L + 1)
    P[L] = []
    for t in range(1 << L):
        U, _ = truncated_basis([(X[t] @ K[L][t] @ _h(X[t]), 1.0)], tau)
        U = U[:, :max(1, min(U.shape[1], X[t].shape[1]))]
        Xn[t] = U
        P[L].append(_h(U) @ X[t])
    for lev in range(L - 1, lmin - 1, -1):
        P[lev] = []
        for t in range(1 << lev):
            a, b = 2 * t, 2 * t + 1
            Z = np.vstack([P[lev + 1][a] @ E[lev + 1][a], P[lev + 1][b] @ E[lev + 1][b]])
            U, _ = truncated_basis([(Z @ K[lev][t] @ _h(Z), 1.0)], tau)
            U = U[:, :max(1, min(U.shape[1], Z.shape[1]))]
            k1 = P[lev + 1][a].shape[0]
            En[lev + 1][a] = U[:k1]
            En[lev + 1][b] = U[k1:]
            P[lev].append(_h(U) @ Z)
    return Xn, En, P


def recompress(M, eps, theta=THETA):
    """Recompressed copy of M at accuracy eps (>= EPS_FLOOR).  Returns (M', info)
    with the new rank profiles."""
    if not eps >= EPS_FLOOR:
        raise ValueError("eps must be >= %g" % EPS_FLOOR)
    L = M.L
    lmin = M.blocks.min_admissible_level()
    tau = threshold(eps, ACCURACY, theta, truncated_levels(L, lmin))
    BV = basis_grams(M.V, M.Er, L)
    BW = basis_grams(M.W, M.Ec, L)
    row_c = [[] for _ in range(L + 1)]
    col_c = [[] for _ in range(L + 1)]
    for lev in range(L + 1):
        for q, (t, s, typ) in enumerate(zip(M.blocks.rows[lev], M.blocks.cols[lev],
                                            M.blocks.types[lev])):
            if typ == R:
                row_c[lev].append((int(t), int(s), M.S[lev][q]))
                col_c[lev].append((int(s), int(t), M.S[lev][q].T))
    V2, Er2, PR = new_side(M.V, M.Er, row_c, BW, L, lmin, tau, M.krow, M.dtype)
    W2, Ec2, PC = new_side(M.W, M.Ec, col_c, BV, L, lmin, tau, M.kcol, M.dtype)

    def rank(side, lev, c):
        P = PR if side == 0 else PC
        return P[lev][c].shape[0] if lev >= lmin else 0

    # above l_min no block needs a basis: transfers into those levels are
    # empty (k x 0) and the clusters there have rank zero
    for lev in range(1, lmin + 1):
        for c in range(1 << lev):
            Er2[lev][c] = np.zeros((rank(0, lev, c), 0), dtype=M.dtype)
            Ec2[lev][c] = np.zeros((rank(1, lev, c), 0), dtype=M.dtype)
    Er2[0] = [None]
    Ec2[0] = [None]
    S2 = []
    for lev in range(L + 1):
        sl = []
        for q, (t, s, typ) in enumerate(zip(M.blocks.rows[lev], M.blocks.cols[lev],
                                            M.blocks.types[lev])):
            sl.append(PR[lev][t] @ M.S[lev][q] @ PC[lev][s].T if typ == R else None)
        S2.append(sl)
    F2 = [None if f is None else f.copy() for f in M.F]
    out = H2Matrix(M.tree, M.blocks, V2, Er2, W2, Ec2, S2, F2)
    info = dict(lmin=lmin, tau=tau,
                ranks_row=[[out.krow(lev, c) for c in range(1 << lev)] for lev in range(L + 1)],
                ranks_col=[[out.kcol(lev, c) for c in range(1 << lev)] for lev in range(L + 1)])
    return out, info
