"""Three-stage, third-order low-storage Runge-Kutta time integration (Sec. 3.1
names a third-order scheme with three stages; Eq. (6) is its one-stage analogue).

Test infrastructure only (see ``oracle/__init__``).

The paper names the order and the stage count only; the scheme read here is
Williamson's 2N-storage RK3 (J. Comput. Phys. 35, 1980), whose stage s is
    k <- A_s k + dt R(q, t + C_s dt),    q <- q + B_s k,
with A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15), C = (0, 1/3, 3/4).
Every three-stage third-order method has the stability polynomial
1 + z + z^2/2 + z^3/6.
"""
A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)
C = (0.0, 1.0 / 3.0, 3.0 / 4.0)


def rk3_step(q, dt, rhs, t=0.0):
    """One step q^n -> q^{n+1}; ``rhs(q, t)`` is the (corrected) right-hand side."""
    k = None
    for s in range(3):
        r = rhs(q, t + C[s] * dt)
        k = dt * r if s == 0 else A[s] * k + dt * r
        q = q + B[s] * k
    return q


def integrate(q, dt, n_steps, rhs, t0=0.0, callback=None):
    """n_steps RK3 steps from t0; ``callback(step, q)`` runs after each step."""
    for n in range(n_steps):
        q = rk3_step(q, dt, rhs, t0 + n * dt)
        if callback is not None:
            callback(n + 1, q)
    return q
