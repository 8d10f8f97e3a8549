"""Runge-Kutta tableaus and LTS stage-conversion weights (test infrastructure only).

Paper passages:
  * eq. rk_schemes (Sec. 3.4): explicit p-stage RK, stages k_i and weights w_i.
  * eq. rk_crrection (Sec. 3.6.2): linear relation between the stages K and the
    time derivatives d^j U / dt^j through a lower-triangular matrix C and the
    step-size matrix P_dt = diag(1, dt, ..., dt^{p-1}).
  * eqs. fc_1 / fc_2 (Sec. 3.6.2): stage corrections between a finer and a
    coarser block, M = (P C) B (P C)^{-1} with B an upper-triangular Taylor shift.

Readings (the printed factor order is dimensionally inconsistent):
  * The stage argument is u^n + dt * sum_q a_sq k_q (eq. rk_schemes omits dt in
    the stages but keeps it in the update); w_i are the usual weights b_i.
  * K = C P D (rows of C are stages, columns derivative orders), not P C D: with
    P on the left a stage would be scaled by dt^{i-1}, which does not match
    k_i = F(...).  The inverse used by the correction is then P^{-1} C^{-1}.
  * B_Delta is the Taylor shift (B)_{jm} = Delta^{m-j}/(m-j)!, truncated at p.
  * A ghost holds the receiver-step *stage state* Y_s built from converted
    stages, i.e. u(t_r) + dt_r sum_{q<s} a_sq k~_q, where u(t_r) is the source's
    Taylor polynomial at the receiver's step start and k~ the converted stages.

All weights are computed in exact rationals (fractions.Fraction); a float64
value is obtained from each rational by one correctly rounded division.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction as Fr
from math import factorial
from typing import Dict, List, Sequence, Tuple


@dataclass(frozen=True)
class Tableau:
    """Explicit RK tableau (eq. rk_schemes): a is strictly lower triangular."""
    name: str
    a: Tuple[Tuple[Fr, ...], ...]   # p x p
    b: Tuple[Fr, ...]               # p

    @property
    def p(self) -> int:
        return len(self.b)

    @property
    def c(self) -> Tuple[Fr, ...]:
        return tuple(sum(row, Fr(0)) for row in self.a)


def _tab(name: str, a: Sequence[Sequence], b: Sequence) -> Tableau:
    return Tableau(name, tuple(tuple(Fr(x) for x in row) for row in a), tuple(Fr(x) for x in b))


#: Classic fourth-order RK (the configurations' scheme).
RK4 = _tab("rk4",
           [[0, 0, 0, 0],
            [Fr(1, 2), 0, 0, 0],
            [0, Fr(1, 2), 0, 0],
            [0, 0, 1, 0]],
           [Fr(1, 6), Fr(1, 3), Fr(1, 3), Fr(1, 6)])

#: Third-order strong-stability-preserving RK of Shu and Osher (the paper's
#: experiments use a third-order RK scheme, Sec. 4.3).
SSPRK3 = _tab("ssprk3",
              [[0, 0, 0],
               [1, 0, 0],
               [Fr(1, 4), Fr(1, 4), 0]],
              [Fr(1, 6), Fr(1, 6), Fr(2, 3)])

TABLEAUS: Dict[str, Tableau] = {"rk4": RK4, "ssprk3": SSPRK3}


def c_matrix(tab: Tableau) -> List[List[Fr]]:
    """Matrix C of eq. rk_crrection.

    For a linear autonomous problem u' = L u every stage is a polynomial in
    dt L applied to u: k_i = sum_j C_ij dt^{j-1} L^j u.  Inserting this into
    k_i = L(u + dt sum_m a_im k_m) gives C_i1 = 1 and
    C_{i,j+1} = sum_m a_im C_{m,j}.
    """
    p = tab.p
    C = [[Fr(0)] * p for _ in range(p)]
    for i in range(p):
        C[i][0] = Fr(1)
    for j in range(1, p):
        for i in range(p):
            C[i][j] = sum((tab.a[i][m] * C[m][j - 1] for m in range(p)), Fr(0))
    return C


def lower_inverse(M: List[List[Fr]]) -> List[List[Fr]]:
    """Exact inverse of a lower-triangular rational matrix (forward substitution)."""
    n = len(M)
    inv = [[Fr(0)] * n for _ in range(n)]
    for col in range(n):
        for i in range(n):
            rhs = Fr(1) if i == col else Fr(0)
            acc = sum((M[i][k] * inv[k][col] for k in range(i)), Fr(0))
            if M[i][i] == 0:
                raise ZeroDivisionError("C is singular: the tableau does not reach order p on linear problems")
            inv[i][col] = (rhs - acc) / M[i][i]
    return inv


def converted_stages(tab: Tableau, delta: Fr, rho: Fr) -> List[List[Fr]]:
    """Matrix T with k~ = T K: a source's stages expressed as the stages of a step of
    size dt_r starting Delta later (eqs. fc_1, fc_2: M = C P_r B_Delta P_n^{-1} C^{-1}),
    in units where dt_r = 1 (delta = Delta/dt_r, rho = dt_n/dt_r)."""
    p = tab.p
    C = c_matrix(tab)
    Ci = lower_inverse(C)
    delta = Fr(delta)
    rho = Fr(rho)
    T = [[Fr(0)] * p for _ in range(p)]
    for q in range(p):
        for j in range(1, p + 1):
            cq = C[q][j - 1]
            if cq == 0:
                continue
            for m in range(j, p + 1):
                f = cq * delta ** (m - j) / factorial(m - j) * rho ** (1 - m)
                for i in range(p):
                    T[q][i] += f * Ci[m - 1][i]
    return T


def conversion_weights(tab: Tableau, delta: Fr, rho: Fr) -> List[List[Fr]]:
    """Stage-conversion weights w^_{s,i}(delta, rho) (eqs. rk_crrection, fc_1, fc_2).

    A source block holds a step record (U0, K_1..K_p) taken with step dt_n and
    starting Delta before the receiver's current step (receiver step dt_r).  With
    delta = Delta/dt_r and rho = dt_n/dt_r, the receiver's stage-s state is

        Y_s = U0 + dt_r * sum_i w^_{s,i} K_i ,

    obtained by
      D      = P_n^{-1} C^{-1} K                (derivatives at the source start)
      u(t_r) = U0 + sum_j Delta^j / j! D_j      (Taylor to order p)
      k~     = C P_r B_Delta D                  (receiver stages, eq. fc_1/fc_2)
      Y_s    = u(t_r) + dt_r sum_{q<s} a_sq k~_q.
    Dividing every dt by dt_r leaves only delta and rho.
    """
    p = tab.p
    C = c_matrix(tab)
    Ci = lower_inverse(C)
    delta = Fr(delta)
    rho = Fr(rho)
    # Taylor part: (u(t_r) - U0)/dt_r = sum_i taylor_i K_i
    taylor = [Fr(0)] * p
    for j in range(1, p + 1):          # derivative order j uses row j-1 of C^{-1}
        f = delta ** j * rho ** (1 - j) / factorial(j)
        for i in range(p):
            taylor[i] += f * Ci[j - 1][i]
    T = converted_stages(tab, delta, rho)
    W = []
    for s in range(p):
        row = list(taylor)
        for q in range(s):
            if tab.a[s][q] != 0:
                for i in range(p):
                    row[i] += tab.a[s][q] * T[q][i]
        W.append(row)
    return W


#: The four legal time cases of a ghost relation on a ghost-reach-balanced octree
#: (Sec. 3.6.3: adjacent blocks differ by at most one level and their time gap is
#: at most the finer step).  Index -> (delta, rho).
CASES: Tuple[Tuple[Fr, Fr], ...] = (
    (Fr(0), Fr(1)),        # 0: same level
    (Fr(0), Fr(1, 2)),     # 1: finer source, common start (eq. fc_1 direction f->c)
    (Fr(0), Fr(2)),        # 2: coarser source, common start (inverse of eq. fc_1)
    (Fr(1), Fr(2)),        # 3: coarser source, receiver's second fine step (eq. fc_2)
)


def weight_table(tab: Tableau) -> List[List[List[Fr]]]:
    """Exact weights [case][stage][i] for the four cases in CASES."""
    return [conversion_weights(tab, d, r) for (d, r) in CASES]


def to_float(x: Fr) -> float:
    """One correctly rounded division p/q (Python's int/int true division)."""
    return x.numerator / x.denominator


def weight_table_f64(tab: Tableau):
    """float64 weights [case][stage][i], each from one correctly rounded division."""
    import numpy as np
    W = weight_table(tab)
    return np.array([[[to_float(x) for x in row] for row in case] for case in W], dtype=np.float64)


def a_f64(tab: Tableau):
    import numpy as np
    return np.array([[to_float(x) for x in row] for row in tab.a], dtype=np.float64)


def b_f64(tab: Tableau):
    import numpy as np
    return np.array([to_float(x) for x in tab.b], dtype=np.float64)
