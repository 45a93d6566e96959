"""IMEX Runge-Kutta double Butcher tableaux (Section 3.1) and the three presets.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A tableau is (At, bt, A, b): At strictly lower triangular (explicit), A lower
triangular (diagonally implicit), weights bt / b.  Definitions of Section 3.1:
  type A   a_ii != 0 for all i;
  type CK  a_11 = 0 and the trailing (s-1)x(s-1) block of A invertible;
  ARS      type CK with a_i1 = 0 for all i;
  GSA      a_si = b_i for all i and at_si = bt_i for i < s (the last stage is the
           new time level).
Presets:
  euler1   first-order GSA IMEX Euler (Section 4.1);
  paper2   second-order GSA IMEX scheme with c = 9/4, gamma = (c - 1/2)/(c - 1)
           (Section 4.1);
  ars443   third-order ARS(4,4,3) of Ascher, Ruuth and Spiteri (1997), cited by the
           paper but not printed in it: the paper prints no third-order tableau.
Type-A presets (Theorem 3.4 covers type A without well-prepared data; the paper prints
no type-A tableau, so these are constructed here from the order conditions):
  typea1   first order: implicit A = I (2 x 2), explicit stage 2 from stage 1;
  typea2   second order, four stages, diagonally implicit with a_ii = 1/4 and weights
           b = (1/2, 0, 1/4, 1/4), explicit Heun-type part with weights (1/2, 1/2, 0, 0);
           it meets sum b = sum bt = 1 and b.c = bt.ct = b.ct = bt.c = 1/2 exactly.
Pins (tests/test_tableau.py): the printed coefficients (tests/golden/tableaux.json),
structural properties, and observed order of accuracy on a partitioned test ODE
against a high-accuracy reference.
"""

from fractions import Fraction as Fr

import numpy as np


class Tableau:
    def __init__(self, name, At, bt, A, b):
        self.name = name
        self.At = np.array(At, dtype=np.float64)
        self.bt = np.array(bt, dtype=np.float64)
        self.A = np.array(A, dtype=np.float64)
        self.b = np.array(b, dtype=np.float64)
        self.s = self.A.shape[0]

    @property
    def ct(self):
        return self.At.sum(axis=1)

    @property
    def c(self):
        return self.A.sum(axis=1)

    def is_explicit_part_ok(self):
        return bool(np.all(np.triu(self.At) == 0.0))

    def is_dirk(self):
        return bool(np.all(np.triu(self.A, 1) == 0.0))

    def is_type_a(self):
        return bool(np.all(np.diag(self.A) != 0.0))

    def is_type_ck(self):
        if self.A[0, 0] != 0.0:
            return False
        return bool(np.all(np.diag(self.A)[1:] != 0.0))

    def is_ars(self):
        return self.is_type_ck() and bool(np.all(self.A[:, 0] == 0.0))

    def is_gsa(self):
        s = self.s
        return (bool(np.all(self.A[s - 1, :] == self.b))
                and bool(np.all(self.At[s - 1, : s - 1] == self.bt[: s - 1]))
                and self.bt[s - 1] == 0.0)


def _frac_to_float(rows):
    return [[float(x) for x in r] for r in rows]


def euler1_fractions():
    At = [[0, 0], [1, 0]]
    bt = [1, 0]
    A = [[0, 0], [0, 1]]
    b = [0, 1]
    return At, bt, A, b


def paper2_fractions(c=Fr(9, 4)):
    g = (c - Fr(1, 2)) / (c - 1)
    At = [[0, 0, 0], [c, 0, 0], [1 - 1 / (2 * c), 1 / (2 * c), 0]]
    bt = [1 - 1 / (2 * c), 1 / (2 * c), 0]
    A = [[0, 0, 0], [0, c, 0], [0, 1 - g, g]]
    b = [0, 1 - g, g]
    return At, bt, A, b


def ars443_fractions():
    h = Fr(1, 2)
    A = [[0, 0, 0, 0, 0],
         [0, h, 0, 0, 0],
         [0, Fr(1, 6), h, 0, 0],
         [0, -h, h, h, 0],
         [0, Fr(3, 2), Fr(-3, 2), h, h]]
    At = [[0, 0, 0, 0, 0],
          [h, 0, 0, 0, 0],
          [Fr(11, 18), Fr(1, 18), 0, 0, 0],
          [Fr(5, 6), Fr(-5, 6), h, 0, 0],
          [Fr(1, 4), Fr(7, 4), Fr(3, 4), Fr(-7, 4), 0]]
    return At, list(At[4]), A, list(A[4])


def typea1_fractions():
    At = [[0, 0], [1, 0]]
    bt = [1, 0]
    A = [[1, 0], [0, 1]]
    b = [0, 1]
    return At, bt, A, b


def typea2_fractions():
    q, h = Fr(1, 4), Fr(1, 2)
    A = [[q, 0, 0, 0],
         [h, q, 0, 0],
         [q, 0, q, 0],
         [h, 0, q, q]]
    At = [[0, 0, 0, 0],
          [1, 0, 0, 0],
          [h, h, 0, 0],
          [h, h, 0, 0]]
    return At, [h, h, 0, 0], A, [h, 0, q, q]


def preset_fractions(name):
    return {"euler1": euler1_fractions, "paper2": paper2_fractions,
            "ars443": ars443_fractions, "typea1": typea1_fractions,
            "typea2": typea2_fractions}[name]()


def preset(name):
    At, bt, A, b = preset_fractions(name)
    return Tableau(name, _frac_to_float(At), [float(x) for x in bt],
                   _frac_to_float(A), [float(x) for x in b])


PRESETS = ("euler1", "paper2", "ars443")
TYPE_A_PRESETS = ("typea1", "typea2")
