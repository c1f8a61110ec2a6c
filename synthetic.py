"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

This module holds no arithmetic of the method: it draws random numbers and
arranges them in the shapes the library boundary uses.  Both the CPU oracle
and the HIP path receive exactly these arrays.

* ``random_state``   a valid (positive density and pressure) conserved state
                     q[5][E][n_p] with the magnitudes of the Mach-0.1 Taylor-Green
                     vortex: rho ~ 1, momentum O(1), total energy ~ 178.7.
* ``mlp_init``       Gaussian weights (std 1/sqrt(fan_in)), zero biases, float32,
                     drawn layer by layer from one generator.
* ``request_stream`` the mixed stream of Taylor-Green solves used by the
                     serving workload (Poisson arrivals).
* ``epoch_permutation`` the minibatch shuffle of one training epoch.
"""
import numpy as np

# rho E of the Mach-0.1 TGV at rest pressure: p0/(gamma-1) + 1/8 with p0 = 1/(1.4 * 0.01).
TGV_ENERGY_LEVEL = 178.69642857142858


def random_state(N, P, seed, momentum=1.0, density_amp=0.05, energy_amp=2.0):
    """Nodal-noise conserved state, q[v][e][n] float64, e over N^3 elements."""
    rng = np.random.default_rng(seed)
    E, n_p = N ** 3, (P + 1) ** 3
    q = np.empty((5, E, n_p))
    q[0] = 1.0 + density_amp * rng.uniform(-1.0, 1.0, (E, n_p))
    q[1:4] = momentum * rng.uniform(-1.0, 1.0, (3, E, n_p))
    q[4] = TGV_ENERGY_LEVEL + energy_amp * rng.uniform(-1.0, 1.0, (E, n_p))
    return q


def constant_state(N, P, rho, mom, energy):
    E, n_p = N ** 3, (P + 1) ** 3
    q = np.empty((5, E, n_p))
    q[0] = rho
    q[1:4] = np.asarray(mom, dtype=np.float64)[:, None, None]
    q[4] = energy
    return q


def mlp_init(dims, seed=0):
    """[(W[out, in], b[out]), ...] float32: W ~ N(0, 1) / sqrt(fan_in), b = 0.
    The weights of layer 1, 2, ... are drawn in that order, row-major."""
    rng = np.random.default_rng(seed)
    layers = []
    for fan_in, fan_out in zip(dims[:-1], dims[1:]):
        W = (rng.standard_normal((fan_out, fan_in)) / np.sqrt(fan_in)).astype(np.float32)
        layers.append((W, np.zeros(fan_out, dtype=np.float32)))
    return layers


def random_rows(n_rows, n_cols, seed, scale=1.0, dtype=np.float32):
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal((n_rows, n_cols))).astype(dtype)


def epoch_permutation(n, rng):
    return rng.permutation(n)


def request_stream(n=64, seed=1, mean_gap=0.5, t_end=2.0):
    """Serving workload: for each request i, draw the gap to the previous
    arrival ~ Exp(mean_gap), then Re, the order choice and the mesh, uniformly,
    in that order.  Order choice "3+nn" means P = 3 with the forcing network."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for i in range(n):
        t += rng.exponential(mean_gap)
        Re = (30.0, 200.0, 1600.0)[rng.integers(3)]
        order = ("3+nn", "6", "8")[rng.integers(3)]
        N = (4, 8, 16)[rng.integers(3)]
        reqs.append({"id": i, "arrival": t, "Re": Re, "P": 3 if order == "3+nn" else int(order),
                     "use_nn": order == "3+nn", "N": N, "t_end": t_end})
    return reqs
