"""Seeded synthetic inputs (random numbers only; none of the solver's
arithmetic).  Arrays are full node arrays, row-major with x fastest; entries at
boundary nodes are ignored for right-hand sides and used for Dirichlet data.

Recipe: numpy PCG64 ``default_rng(seed)``; right-hand sides i.i.d. uniform on
[-1, 1] or standard normal, drawn over the whole node array in row-major order.
"""
import numpy as np


def uniform(shape, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, shape)


def normal(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def normal_triplet(shape, seed):
    """f, Dirichlet data and loss weights drawn in that order from one generator."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape), rng.standard_normal(shape), rng.standard_normal(shape)


def sine_product(xs):
    """u = prod_a sin(pi x_a) on the tensor grid of the node coordinate arrays xs
    (x fastest) and its Laplacian -dim pi^2 u: a manufactured solution."""
    grids = np.meshgrid(*reversed(xs), indexing="ij")
    u = np.ones(grids[0].shape)
    for g in grids:
        u = u * np.sin(np.pi * g)
    return u, -len(xs) * np.pi ** 2 * u
