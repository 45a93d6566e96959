"""Six-velocity (D2Q6) discrete velocity model of Section 2.1.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is here, each written from the definitions of Section 2.1:
  velocity_set        c_i = (cos(pi(i-1)/3), sin(pi(i-1)/3)), i = 1..6.
  moment_matrix       rows: 1, c_x, c_y, 1/2 - c_x^2, c_x c_y, c_x (c_y^2 - 1/4).
  equilibrium         F_i^eq = rho/6 + (1/3) c_i.u + (2/3)(c_i c_i - I/2):u u.
  bgk_collision       C(F) = -(1/tau)(F - F^eq(rho(F), u(F))).
  scaled <-> populations  the map between populations F_i and the scaled moments
                      (u1, u2, theta, v1, v2, q): R = 1 + 2 eps^2 theta, U = eps u,
                      V = eps^2 v, Q = eps^3 q with R, U, V, Q the unscaled moments.
  population_rhs      d/dt F_i of the scaled model  dF/dt + (1/eps) c.grad F =
                      -(1/(eps^2 tau))(F - F^eq).
  moment_rhs          the scaled closed moment system (Section 2.1, the six scalar
                      equations; vector form of Section 3).

Readings of the printed text (each one pinned by tests/test_d2q6.py):
  * v1 is the moment of (1/2 - c_x^2); the printed definition has the opposite sign,
    but the moment system, the definition of F(u) and the formal limit all require
    this one.
  * The q equation carries d_x v1 + d_y v2 (the printed equation repeats d_x).
  * The collision relaxes towards equilibrium: the printed scaled population
    equation puts a minus sign in front of C(F), which would anti-relax.
  * The rescaled moments are R = 1 + 2 eps^2 theta, U = eps u, V = eps^2 v,
    Q = eps^3 q (the printed rescaling drops the factor 1/6 of the Maxwellian).
Pins: equilibrium moment identities, collision invariants, Gram matrix of the
basis, and moments of population_rhs == moment_rhs for arbitrary smooth fields.
"""

import numpy as np


def velocity_set():
    """The six lattice velocities (Section 2.1).  Returns (cx, cy), each shape (6,)."""
    i = np.arange(1, 7)
    ang = np.pi * (i - 1) / 3.0
    return np.cos(ang), np.sin(ang)


def moment_matrix():
    """6x6 matrix M with rows m_k(c_i); M @ F gives (rho, U1, U2, V1, V2, Q).

    Rows follow the moment definitions of Section 2.1 (density, momentum, the two
    second-order moments v1, v2 and the third-order moment q), with v1 read as the
    moment of (1/2 - c_x^2).
    """
    cx, cy = velocity_set()
    return np.stack([
        np.ones(6),
        cx,
        cy,
        0.5 - cx * cx,
        cx * cy,
        cx * (cy * cy - 0.25),
    ])


def equilibrium(rho, u1, u2):
    """F_i^eq(rho, u) of Section 2.1.  Returns an array with a leading axis of 6."""
    cx, cy = velocity_set()
    rho = np.asarray(rho, dtype=np.float64)
    u1 = np.asarray(u1, dtype=np.float64)
    u2 = np.asarray(u2, dtype=np.float64)
    out = []
    for i in range(6):
        cu = cx[i] * u1 + cy[i] * u2
        # (c c - I/2) : (u u)
        quad = ((cx[i] * cx[i] - 0.5) * u1 * u1
                + 2.0 * cx[i] * cy[i] * u1 * u2
                + (cy[i] * cy[i] - 0.5) * u2 * u2)
        out.append(rho / 6.0 + cu / 3.0 + (2.0 / 3.0) * quad)
    return np.stack(out)


def raw_moments(F):
    """(rho, U1, U2, V1, V2, Q) = M @ F along the leading axis."""
    M = moment_matrix()
    return np.tensordot(M, F, axes=(1, 0))


def bgk_collision(F, tau):
    """C(F_i) = -(1/tau)(F_i - F_i^eq), with F^eq built from rho = sum F and
    u = sum c F of F itself (Section 2.1)."""
    m = raw_moments(F)
    return -(F - equilibrium(m[0], m[1], m[2])) / tau


def populations_from_scaled(u1, u2, theta, v1, v2, q, eps):
    """Populations F_i for given scaled moments (Section 2.1 scaling, reading above).

    Solves M F = (R, U1, U2, V1, V2, Q) with R = 1 + 2 eps^2 theta, U = eps u,
    V = eps^2 v, Q = eps^3 q.  M is invertible because its rows are orthogonal.
    """
    m = np.stack([
        1.0 + 2.0 * eps * eps * np.asarray(theta, dtype=np.float64),
        eps * np.asarray(u1, dtype=np.float64),
        eps * np.asarray(u2, dtype=np.float64),
        eps * eps * np.asarray(v1, dtype=np.float64),
        eps * eps * np.asarray(v2, dtype=np.float64),
        eps ** 3 * np.asarray(q, dtype=np.float64),
    ])
    M = moment_matrix()
    shape = m.shape[1:]
    F = np.linalg.solve(M, m.reshape(6, -1))
    return F.reshape((6,) + shape)


def scaled_from_populations(F, eps):
    """Inverse of populations_from_scaled: (u1, u2, theta, v1, v2, q)."""
    rho, U1, U2, V1, V2, Q = raw_moments(F)
    return (U1 / eps, U2 / eps, (rho - 1.0) / (2.0 * eps * eps),
            V1 / eps ** 2, V2 / eps ** 2, Q / eps ** 3)


def population_rhs(F, eps, tau, ddx, ddy):
    """dF_i/dt of the diffusively scaled DVM with relaxing BGK collision:
    dF/dt = -(1/eps) c_i.grad F_i - (1/(eps^2 tau)) (F_i - F_i^eq(rho, u)).

    ddx, ddy: callables returning the x / y derivative of a 2D field."""
    cx, cy = velocity_set()
    m = raw_moments(F)
    Feq = equilibrium(m[0], m[1], m[2])
    out = np.empty_like(F)
    for i in range(6):
        out[i] = (-(cx[i] * ddx(F[i]) + cy[i] * ddy(F[i])) / eps
                  - (F[i] - Feq[i]) / (eps * eps * tau))
    return out


def flux_F(u1, u2):
    """F(u) = (1/2 (u2^2 - u1^2), u1 u2) of the vector form (Section 3)."""
    return 0.5 * (u2 * u2 - u1 * u1), u1 * u2


def moment_rhs(u1, u2, theta, v1, v2, q, eps, tau, ddx, ddy):
    """Time derivatives of the scaled moments from the closed moment system of
    Section 2.1 (with the q-equation divergence read as d_x v1 + d_y v2).

    tau = 0 is not allowed here (the relaxation term is stiff-infinite)."""
    F1, F2 = flux_F(u1, u2)
    du1 = -(-ddx(v1) + ddy(v2) + ddx(theta))
    du2 = -(ddx(v2) + ddy(v1) + ddy(theta))
    dth = -(ddx(u1) + ddy(u2)) / (2.0 * eps * eps)
    dv1 = -(-ddx(u1) + ddy(u2)) / (4.0 * eps * eps) - ddx(q) - (v1 - F1) / (eps * eps * tau)
    dv2 = -(ddx(u2) + ddy(u1)) / (4.0 * eps * eps) - ddy(q) - (v2 - F2) / (eps * eps * tau)
    dq = -(ddx(v1) + ddy(v2)) / (2.0 * eps * eps) - q / (eps * eps * tau)
    return du1, du2, dth, dv1, dv2, dq
