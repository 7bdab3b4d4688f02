"""Exact operations on an H^2 matrix: expansion to dense and the matrix-vector
product (the exact H^2 mat-vec the accuracy criterion, equation `error` of
Section VI, relies on).  FP64 / complex128, plain NumPy.

Part of the CPU checker: test infrastructure only.
"""
import numpy as np

from h2inputs.structure import R, F


def expanded_row_basis(M, lev, c):
    """V_t for cluster (lev, c), assembled through the nested property
    (Section II): V_t = diag(V_t1, V_t2) [E_t1; E_t2]."""
    if lev == M.L:
        return M.V[c]
    a = expanded_row_basis(M, lev + 1, 2 * c) @ M.Er[lev + 1][2 * c]
    b = expanded_row_basis(M, lev + 1, 2 * c + 1) @ M.Er[lev + 1][2 * c + 1]
    return np.vstack([a, b])


def expanded_col_basis(M, lev, c):
    if lev == M.L:
        return M.W[c]
    a = expanded_col_basis(M, lev + 1, 2 * c) @ M.Ec[lev + 1][2 * c]
    b = expanded_col_basis(M, lev + 1, 2 * c + 1) @ M.Ec[lev + 1][2 * c + 1]
    return np.vstack([a, b])


def to_dense_tree_order(M):
    """Dense matrix in tree order: V_t S_ts W_s^T for admissible blocks, the
    stored block for dense leaves."""
    n = M.n
    D = np.zeros((n, n), dtype=M.dtype)
    t_ = M.tree
    for lev in range(M.L + 1):
        for q, (t, s, typ) in enumerate(zip(M.blocks.rows[lev], M.blocks.cols[lev],
                                            M.blocks.types[lev])):
            rs = slice(t_.start(lev, t), t_.stop(lev, t))
            cs = slice(t_.start(lev, s), t_.stop(lev, s))
            if typ == R:
                D[rs, cs] = expanded_row_basis(M, lev, t) @ M.S[lev][q] @ \
                    expanded_col_basis(M, lev, s).T
            elif typ == F:
                D[rs, cs] = M.F[q]
    return D


def to_dense(M):
    """Dense matrix in the original point order."""
    D = to_dense_tree_order(M)
    out = np.empty_like(D)
    p = M.tree.perm
    out[np.ix_(p, p)] = D
    return out


def matvec(M, x):
    """y = M x for x in the original point order (n or n x nrhs): forward
    transform x^_s = W_s^T x_s up the tree, couplings y^_t += S_ts x^_s,
    backward transform down the tree, then the dense near field."""
    x = np.asarray(x)
    vec = x.ndim == 1
    X = x.reshape(M.n, -1)
    dt = np.result_type(M.dtype, X.dtype)
    p = M.tree.perm
    xt = X[p].astype(dt)
    L = M.L
    t_ = M.tree
    xh = [None] * (L + 1)
    xh[L] = [M.W[c].T @ xt[t_.start(L, c):t_.stop(L, c)] for c in range(1 << L)]
    for lev in range(L - 1, -1, -1):
        xh[lev] = [M.Ec[lev + 1][2 * c].T @ xh[lev + 1][2 * c]
                   + M.Ec[lev + 1][2 * c + 1].T @ xh[lev + 1][2 * c + 1]
                   for c in range(1 << lev)]
    yh = [[np.zeros((M.krow(lev, c), X.shape[1]), dtype=dt) for c in range(1 << lev)]
          for lev in range(L + 1)]
    yt = np.zeros((M.n, X.shape[1]), dtype=dt)
    for lev in range(L + 1):
        for q, (t, s, typ) in enumerate(zip(M.blocks.rows[lev], M.blocks.cols[lev],
                                            M.blocks.types[lev])):
            if typ == R:
                yh[lev][t] += M.S[lev][q] @ xh[lev][s]
            elif typ == F:
                yt[t_.start(lev, t):t_.stop(lev, t)] += \
                    M.F[q] @ xt[t_.start(lev, s):t_.stop(lev, s)]
    for lev in range(1, L + 1):
        for c in range(1 << lev):
            yh[lev][c] += M.Er[lev][c] @ yh[lev - 1][c // 2]
    for c in range(1 << L):
        yt[t_.start(L, c):t_.stop(L, c)] += M.V[c] @ yh[L][c]
    y = np.empty_like(yt)
    y[p] = yt
    return y[:, 0] if vec else y


def relative_error(C, A, B, x):
    """epsilon_rel of equation `error`: ||C x - A (B x)|| / ||A (B x)||."""
    ref = matvec(A, matvec(B, x))
    return float(np.linalg.norm(matvec(C, x) - ref) / np.linalg.norm(ref))
