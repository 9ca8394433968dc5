"""Seeded synthetic inputs for the domain-wall multigrid path.

This module is shared by the CPU oracle and the HIP path and holds none of the
method's arithmetic: it only draws numbers.  Everything is deterministic for a
given seed (numpy PCG64).

Gauge fields stand in for the two-flavor Schwinger ensembles of the paper's
numerical section (Sec. 3): they are quenched U(1) fields drawn with a
checkerboard Metropolis update of the plaquette action
``S = -beta * sum_x cos(theta_P(x))`` from a cold start, with
``theta_P(x) = theta_0(x) + theta_1(x+0) - theta_0(x+1) - theta_1(x)``.

Array conventions (used throughout the package):
  * link angles ``theta[mu, y, x]`` (mu=0 is the x direction), float64;
  * links ``U[mu, y, x] = cos(theta) + i sin(theta)``, complex128;
  * 5-d fermion fields ``psi[rhs, s, y, x, spin]``, complex128, C-contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "GaugeField",
    "metropolis_u1",
    "links_from_theta",
    "gaussian_field",
    "random_theta",
    "random_phases",
    "gauge_seed",
    "rhs_seed",
    "null_start_seed",
]


def gauge_seed(cfg: int, L: int) -> int:
    """Seed of the gauge field of a named workload (10000*cfg + L)."""
    return 10000 * cfg + L


def rhs_seed(cfg: int, L: int, j: int) -> int:
    """Seed of right-hand side ``j`` of a named workload."""
    return 1_000_000 * cfg + 1000 * L + j


def null_start_seed(cfg: int, level: int) -> int:
    """Seed of the Gaussian starting vectors of the setup at ``level``."""
    return 7_000_000 + 100 * cfg + level


@dataclass
class GaugeField:
    theta: np.ndarray          # (2, Ly, Lx) float64
    U: np.ndarray              # (2, Ly, Lx) complex128
    beta: float
    sweeps: int
    seed: int
    acceptance: float
    topological_charge: float


def links_from_theta(theta: np.ndarray) -> np.ndarray:
    """U = cos(theta) + i sin(theta), evaluated once on the host."""
    theta = np.asarray(theta, dtype=np.float64)
    U = np.empty(theta.shape, dtype=np.complex128)
    U.real = np.cos(theta)
    U.imag = np.sin(theta)
    return U


def _wrap(a: np.ndarray) -> np.ndarray:
    """Map angles into [-pi, pi)."""
    return np.remainder(a + math.pi, 2.0 * math.pi) - math.pi


def _plaquette(theta: np.ndarray) -> np.ndarray:
    t0, t1 = theta[0], theta[1]
    return t0 + np.roll(t1, -1, axis=1) - np.roll(t0, -1, axis=0) - t1


def metropolis_u1(Lx: int, Ly: int, beta: float, sweeps: int, seed: int) -> GaugeField:
    """Quenched U(1) Metropolis run, cold start, one hit per link per sweep.

    A sweep updates the mu=0 links on even rows, then odd rows, then the mu=1
    links on even columns, then odd columns.  Links updated together share no
    plaquette, so each half-update is an exact single-link Metropolis step
    applied to many links at once.  Proposal ``theta + delta*(2u-1)`` with
    ``delta = min(pi, 2/sqrt(beta))``; acceptance ``u' < exp(-dS)``.
    Requires even Lx and Ly.
    """
    if Lx % 2 or Ly % 2:
        raise ValueError("metropolis_u1 needs even lattice extents")
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = np.zeros((2, Ly, Lx), dtype=np.float64)
    delta = min(math.pi, 2.0 / math.sqrt(beta)) if beta > 0 else math.pi
    yy, xx = np.meshgrid(np.arange(Ly), np.arange(Lx), indexing="ij")
    masks = [
        (0, (yy % 2) == 0),
        (0, (yy % 2) == 1),
        (1, (xx % 2) == 0),
        (1, (xx % 2) == 1),
    ]
    accepted = 0
    proposed = 0
    for _ in range(sweeps):
        for mu, mask in masks:
            step = delta * (2.0 * rng.random((Ly, Lx)) - 1.0)
            u_acc = rng.random((Ly, Lx))
            old_cos = np.cos(_plaquette(theta))
            trial = theta.copy()
            trial[mu] = np.where(mask, theta[mu] + step, theta[mu])
            new_cos = np.cos(_plaquette(trial))
            dcos = new_cos - old_cos
            # Each link touches two plaquettes: the one at its own site and the
            # one one step back in the orthogonal direction.
            if mu == 0:
                dS = -beta * (dcos + np.roll(dcos, 1, axis=0))
            else:
                dS = -beta * (dcos + np.roll(dcos, 1, axis=1))
            acc = mask & (u_acc < np.exp(np.minimum(-dS, 0.0)))
            theta[mu] = np.where(acc, _wrap(trial[mu]), theta[mu])
            accepted += int(acc.sum())
            proposed += int(mask.sum())
    Q = float(_wrap(_plaquette(theta)).sum() / (2.0 * math.pi))
    return GaugeField(theta=theta, U=links_from_theta(theta), beta=beta,
                      sweeps=sweeps, seed=seed,
                      acceptance=accepted / max(proposed, 1),
                      topological_charge=Q)


def random_theta(Lx: int, Ly: int, seed: int) -> np.ndarray:
    """Uniform link angles in [-pi, pi) (a 'hot' gauge field)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-math.pi, math.pi, size=(2, Ly, Lx))


def random_phases(shape, seed: int) -> np.ndarray:
    """exp(i*alpha) with alpha uniform, e.g. a U(1) gauge rotation g(x)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return links_from_theta(rng.uniform(-math.pi, math.pi, size=shape))


def gaussian_field(shape, seed: int) -> np.ndarray:
    """Complex Gaussian field: Re and Im independently N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty(shape, dtype=np.complex128)
    out.real = rng.standard_normal(shape)
    out.imag = rng.standard_normal(shape)
    return out
