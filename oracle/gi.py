"""Graph isomorphism as QUBO and as an integer Ising model.  Test infrastructure.

Variables: x[u, i] = 1 when vertex u of graph 2 is mapped to vertex i of graph 1
(Section 4.1, after Eq. 8).  Spin index p = u * n + i, so N = n * n spins.

Eq. 8 has two one-hot penalties (weight C1: every vertex of graph 2 maps to
exactly one vertex of graph 1 and vice versa) and two edge-inconsistency
penalties (weight C2: mapping an edge of one graph onto a non-edge of the
other).  Readings taken where the paper is silent:

* C1 = C2 = 1 unless given.
* Each unordered spin pair {(u, i), (v, j)} with u != v, i != j and exactly one of
  A1[i, j], A2[u, v] set is penalised once by C2.  Summing the printed double
  sums over ordered pairs visits every such spin pair twice, so the literal
  evaluation below halves them.

QUBO (Eq. 7) keeps Q upper triangular: H(x) = sum_{p <= q} Q[p, q] x_p x_q.
Ising mapping (Section 4.2): sigma = 2x - 1,
    h_p = -Q_pp / 2 - (1/4) sum_{q != p} Q_pq,   J_pq = J_qp = -Q_pq / 4,
so H_Ising(sigma) = H_QUBO(x) - c with c = sum_p Q_pp / 2 + sum_{p<q} Q_pq / 4.
Everything is multiplied by an integer scale S (a multiple of 4) to keep the
quarter-integers exact: h~ = S h, J~ = S J, E~ = S E.
"""

from __future__ import annotations

from fractions import Fraction
from itertools import permutations

import numpy as np


def spin_index(u: int, i: int, n: int) -> int:
    return u * n + i


def qubo_gi(a1: np.ndarray, a2: np.ndarray, c1: int = 1, c2: int = 1):
    """Upper-triangular integer Q (N x N) and the constant 2 n C1 of Eq. 8, so
    that Eq. 8 = x^T Q x (upper triangular sum) + const.

    Q_pp = -2 C1 (-C1 from the row penalty, -C1 from the column penalty);
    for p < q with p = (u, i), q = (v, j):
      2 C1 if exactly one of u == v, i == j holds (two ones in a row or a column);
      C2   if u != v, i != j and A1[i, j] != A2[u, v] (an edge onto a non-edge);
      0    otherwise.
    """
    n = a1.shape[0]
    N = n * n
    p = np.arange(N)
    u, i = p // n, p % n
    same_u = u[:, None] == u[None, :]
    same_i = i[:, None] == i[None, :]
    one_hot = same_u != same_i
    inconsistent = (~same_u) & (~same_i) & (a1[i[:, None], i[None, :]] != a2[u[:, None], u[None, :]])
    Q = np.where(one_hot, 2 * c1, 0) + np.where(inconsistent, c2, 0)
    Q = np.triu(Q, 1).astype(np.int64)
    Q[p, p] = -2 * c1
    return Q, 2 * n * c1


def eq8_direct(a1: np.ndarray, a2: np.ndarray, x: np.ndarray, c1: int = 1, c2: int = 1) -> Fraction:
    """Eq. 8 evaluated term by term for an assignment x[u, i] (n x n, 0/1)."""
    n = a1.shape[0]
    x = np.asarray(x, dtype=np.int64).reshape(n, n)
    val = Fraction(0)
    for u in range(n):
        val += c1 * (1 - int(x[u, :].sum())) ** 2
    for i in range(n):
        val += c1 * (1 - int(x[:, i].sum())) ** 2
    edge_sum = 0
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            for u in range(n):
                for v in range(n):
                    if u == v:
                        continue
                    if a1[i, j] == 0 and a2[u, v] == 1:
                        edge_sum += x[u, i] * x[v, j]
                    if a1[i, j] == 1 and a2[u, v] == 0:
                        edge_sum += x[u, i] * x[v, j]
    # ordered (i, j) and (u, v): each unordered spin pair counted twice
    val += Fraction(c2 * edge_sum, 2)
    return val


def qubo_value(Q: np.ndarray, x: np.ndarray) -> int:
    """Eq. 7 with upper-triangular Q: sum_{p <= q} Q_pq x_p x_q."""
    x = np.asarray(x, dtype=np.int64).reshape(-1)
    return int(x @ np.triu(Q) @ x)


def ising_from_qubo(Q: np.ndarray, scale: int):
    """Integer Ising coefficients at scale S from an upper-triangular Q.

    Returns (h~ int64 [N], J~ int64 [N, N] symmetric, zero diagonal, S * c) with
    S * H_QUBO(x) = E~(sigma) + S * c for sigma = 2x - 1.
    """
    if scale % 4:
        raise ValueError("scale must be a multiple of 4 for exact quarter-integers")
    N = Q.shape[0]
    Qu = np.triu(Q, 1)
    Qsym = Qu + Qu.T                           # Q_pq for both orders, zero diagonal
    diag = np.diag(Q)
    h = -(scale // 2) * diag - (scale // 4) * Qsym.sum(axis=1)
    J = -(scale // 4) * Qsym
    c_scaled = (scale // 2) * int(diag.sum()) + (scale // 4) * int(Qu.sum())
    return h.astype(np.int64), J.astype(np.int64), c_scaled


def gi_ising(a1: np.ndarray, a2: np.ndarray, scale: int = 12, c1: int = 1, c2: int = 1):
    """GI pair -> (h~, J~, E*~): the integer Ising model at scale S and its ground
    energy, which is reached exactly by the permutation matrices of the
    isomorphisms (Eq. 8 is zero there)."""
    Q, const = qubo_gi(a1, a2, c1, c2)
    h, J, c_scaled = ising_from_qubo(Q, scale)
    e_star = scale * (0 - const) - c_scaled    # Eq. 8 = 0  =>  H_QUBO = -const
    return h, J, e_star


def ground_energy_closed_form(n: int, m: int, scale: int = 12, c1: int = 1, c2: int = 1) -> int:
    """E*~ for an isomorphic pair with n vertices and m edges, from counting Q's
    entries: N diagonal terms -2 C1; n^2 (n-1) one-hot pairs 2 C1; 4 m (P - m)
    inconsistent-edge pairs C2 with P = n(n-1)/2."""
    P = n * (n - 1) // 2
    diag_sum = -2 * c1 * n * n
    upper_sum = 2 * c1 * n * n * (n - 1) + c2 * 4 * m * (P - m)
    c_scaled = (scale // 2) * diag_sum + (scale // 4) * upper_sum
    return -scale * 2 * n * c1 - c_scaled


def assignment_from_perm(perm: np.ndarray) -> np.ndarray:
    """x[u, i] = 1 iff i = perm[u]; flattened to spins p = u n + i."""
    n = len(perm)
    x = np.zeros((n, n), dtype=np.int64)
    x[np.arange(n), perm] = 1
    return x.reshape(-1)


def automorphism_count(a: np.ndarray) -> int:
    """Number of vertex permutations f with a[f(u), f(v)] == a[u, v] (brute force)."""
    n = a.shape[0]
    count = 0
    for f in permutations(range(n)):
        f = np.asarray(f)
        if np.array_equal(a[np.ix_(f, f)], a):
            count += 1
    return count
