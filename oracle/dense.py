"""Brute-force linear algebra on tiny problems (test infrastructure).

* ``big_J``            -- the TD x TD residual Jacobian of eq. big_j: identity blocks on the
                          diagonal, -A_t on the block sub-diagonal (t = 2..T).
* ``J_inv_by_products`` -- eq. J_inv: block (t, u) of J^{-1} is A_t A_{t-1} ... A_{u+1}
                          for t >= u, zero above the diagonal.
* ``newton_step_dense`` -- Delta = -J^{-1} r by a dense linear solve (eq. deer_full_update).
* ``lm_step_dense``     -- Delta_LM = -(J^T J + lambda I)^{-1} J^T r (Ch. 4, the minimiser of
                          eq. lagrangian).
* ``all_bracketings``   -- every way to parenthesise a product with a binary operator; with
                          the affine composition of eq. bin_op_affine they must all agree.
* ``tree_scan_trace``   -- the up-sweep / down-sweep inclusive scan of Tabs. upsweep and
                          downsweep, run on interval labels so its contents can be compared
                          with the tables.
"""
import numpy as np


def big_J(At):
    T, D, _ = At.shape
    J = np.eye(T * D)
    for t in range(1, T):
        J[t * D:(t + 1) * D, (t - 1) * D:t * D] = -At[t]
    return J


def J_inv_by_products(At):
    T, D, _ = At.shape
    Ji = np.zeros((T * D, T * D))
    for u in range(T):
        P = np.eye(D)
        for t in range(u, T):
            if t > u:
                P = At[t] @ P
            Ji[t * D:(t + 1) * D, u * D:(u + 1) * D] = P
    return Ji


def newton_step_dense(At, r):
    T, D = r.shape
    return -np.linalg.solve(big_J(At), r.ravel()).reshape(T, D)


def lm_step_dense(At, r, lam):
    T, D = r.shape
    J = big_J(At)
    M = J.T @ J + lam * np.eye(T * D)
    return -np.linalg.solve(M, J.T @ r.ravel()).reshape(T, D)


def affine_op(ei, ej):
    """eq. bin_op_affine: (A_i, b_i) (x) (A_j, b_j) = (A_j A_i, b_j + A_j b_i); i before j."""
    Ai, bi = ei
    Aj, bj = ej
    return (Aj @ Ai, bj + Aj @ bi)


def all_bracketings(elems, op):
    """Results of every full parenthesisation of op(e_1, ..., e_n) (a Catalan number of them)."""
    memo = {}

    def go(i, j):
        if (i, j) in memo:
            return memo[(i, j)]
        if i == j:
            out = [elems[i]]
        else:
            out = []
            for k in range(i, j):
                for left in go(i, k):
                    for right in go(k + 1, j):
                        out.append(op(left, right))
        memo[(i, j)] = out
        return out

    return go(0, len(elems) - 1)


def tree_scan_trace(T):
    """Up-sweep then down-sweep inclusive scan over positions 1..T (T a power of two).

    Each cell holds the 1-based closed interval (lo, hi) of the product it contains, so a
    combine of (lo, m) with (m + 1, hi) yields (lo, hi).  Returns (up_rows, down_rows), the
    array contents after every level of each sweep, the first up row being the leaves.
    """
    assert T > 0 and T & (T - 1) == 0
    cells = [(t, t) for t in range(1, T + 1)]
    up_rows = [list(cells)]

    def comb(a, b):
        assert a[1] + 1 == b[0], (a, b)
        return (a[0], b[1])

    stride = 1
    while stride < T:
        for pos in range(2 * stride, T + 1, 2 * stride):          # 1-based positions
            cells[pos - 1] = comb(cells[pos - 1 - stride], cells[pos - 1])
        up_rows.append(list(cells))
        stride *= 2
    down_rows = []
    stride = T // 4
    while stride >= 1:
        for pos in range(3 * stride, T + 1, 2 * stride):
            cells[pos - 1] = comb(cells[pos - 1 - stride], cells[pos - 1])
        down_rows.append(list(cells))
        stride //= 2
    return up_rows, down_rows
