"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and lays out workload descriptions; it
holds none of the method's arithmetic (no quadrature, no operator, no solver).
Both the oracle and the library receive what it produces as plain data.

Workloads (the paper uses no public data set; these stand in for its f = 1 and
manufactured-sine test problems):
  * random residual: interior entries iid uniform[-1, 1], boundary entries 0;
  * manufactured sine: f = d*pi^2 * prod_a sin(pi x_a), exact u = prod_a sin(pi x_a);
  * Fourier field: f = sum_{m<16} c_m |kappa_m|^-2 prod_a sin(pi kappa_ma x_a),
    kappa_ma uniform in 1..8, c_m uniform in [-1, 1];
  * serving trace: Poisson arrivals, dimension uniform in {2, 3}, degree uniform
    in 1..7, level whose DoF count is closest (in log) to a log-uniform target
    in [1e4, 1e7].
"""
import math

import numpy as np


def n1d(k, level):
    return k * 2 ** level + 1


def random_interior(d, k, level, seed):
    """Full-grid vector, x0 fastest; interior entries iid U[-1, 1] from default_rng(seed), boundary 0."""
    n = n1d(k, level)
    rng = np.random.default_rng(seed)
    inner = rng.uniform(-1.0, 1.0, size=(n - 2,) * d)
    full = np.zeros((n,) * d)
    full[(slice(1, n - 1),) * d] = inner
    return full.reshape(-1)


def manufactured_sine(d):
    """(kappas, coefs) of f = d*pi^2 prod sin(pi x_a)."""
    return [[1] * d], [d * math.pi ** 2]


def fourier_modes(d, seed, n_modes=16, kappa_max=8):
    """(kappas, coefs) of a random smooth field with amplitudes decaying as |kappa|^-2."""
    rng = np.random.default_rng(seed)
    kappas = rng.integers(1, kappa_max + 1, size=(n_modes, d))
    c = rng.uniform(-1.0, 1.0, size=n_modes)
    coefs = c / np.sum(kappas.astype(np.float64) ** 2, axis=1)
    return kappas.tolist(), coefs.tolist()


def serving_trace(seed, n_requests, rate_per_s, dof_lo=1e4, dof_hi=1e7, degrees=range(1, 8)):
    """List of request dicts: arrival time, d, k, level, kappas, coefs (seeded)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        d = int(rng.integers(2, 4))
        k = int(rng.choice(list(degrees)))
        target = math.exp(rng.uniform(math.log(dof_lo), math.log(dof_hi)))
        best = None
        for level in range(1, 16):
            n = n1d(k, level) ** d
            if n > dof_hi * 1.0001:
                break
            if n < dof_lo * 0.9999:
                continue
            score = abs(math.log(n) - math.log(target))
            if best is None or score < best[0]:
                best = (score, level)
        if best is None:  # no level inside the window: take the smallest above dof_lo
            level = 1
            while n1d(k, level) ** d < dof_lo:
                level += 1
            best = (0.0, level)
        kap, coefs = fourier_modes(d, int(rng.integers(0, 2 ** 31)))
        out.append(dict(id=i, arrival=t, d=d, k=k, level=best[1], kappas=kap, coefs=coefs))
    return out
