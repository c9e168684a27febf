"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module only draws random numbers; it holds none of the method's
arithmetic.  Every random quantity the method consumes (the KL coefficients
xi of each random-field sample, the control z, training controls, initial
network weights) is drawn here and passed, as the same array, to both the CPU
oracle and the HIP library.

Workload recipe (the configurations of the semilinear elliptic source-control
problem, paper Sec. 4.2, eq. (elliptic_pde)):

* xi  ~ N(0, 1) i.i.d., shape (N, K1, K1) in 2D (j = x-frequency slow,
  k = y-frequency fast) or (N, K1, K1, K1) in 3D;
* z   ~ U[0, 1]^{d_Z} (one control shared by all samples of an SAA call);
* Z   ~ U[0, 1]^{N x d_Z} (per-sample controls for training data, the
  auxiliary control law nu_z of Sec. 3.1), or uniform over a box [lo, hi]
  (Sec. 4.2 trains over the admissible box [-4, 4]^{d_Z});
* network weights: Glorot-uniform matrices, zero biases.
"""
from __future__ import annotations

import numpy as np

# Seeds of the named workloads.
SEED_XI_SMALL = 2305     # n = 32, N = 64
SEED_Z_SMALL = 20053
SEED_XI_MEDIUM = 2306    # n = 128, N = 1024
SEED_XI_TRAIN = 2307     # training fields, N = 2048
SEED_Z_TRAIN = 2308      # training controls
SEED_XI_VALID = 2309
SEED_Z_VALID = 2310
SEED_XI_LARGE = 2311     # surrogate SAA, N = 65536
SEED_XI_HELDOUT = 2312   # held-out PDE samples for the surrogate error estimate
SEED_Z_EVAL = (101, 102, 103, 104, 105)
SEED_XI_3D = 2313        # 3D problem on 48^3, N = 256
SEED_Z_3D = 2314         # its control (64 sources)
SEED_XI_TRAIN3D = 2321   # 3D surrogate: training fields, N = 1024
SEED_Z_TRAIN3D = 2322    # its training controls
SEED_XI_HELDOUT3D = 2323 # held-out 3D PDE samples for the error estimate
SEED_XI_LARGE3D = 2324   # 3D surrogate SAA, N = 16384


def kl_coefficients(seed: int, n_samples: int, kl_per_dim: int, dim: int = 2) -> np.ndarray:
    """xi[i, j, k(, l)] ~ N(0, 1), float64, C-contiguous."""
    rng = np.random.default_rng(seed)
    shape = (n_samples,) + (kl_per_dim,) * dim
    return np.ascontiguousarray(rng.standard_normal(shape))


def control(seed: int, d_z: int = 25, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """z ~ U[lo, hi]^{d_z}, float64."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, d_z)


def controls(seed: int, n_samples: int, d_z: int = 25, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Per-sample controls Z[i, :] ~ U[lo, hi]^{d_z}, float64, (n_samples, d_z)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(lo, hi, (n_samples, d_z)))


def glorot_mlp(seed: int, widths: list[int]) -> list[tuple[np.ndarray, np.ndarray]]:
    """Glorot-uniform weights W_l (out x in) and zero biases for the layer
    widths [in, h1, ..., out]; float64."""
    rng = np.random.default_rng(seed)
    layers = []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        w = rng.uniform(-lim, lim, (fan_out, fan_in))
        layers.append((np.ascontiguousarray(w), np.zeros(fan_out)))
    return layers


def random_mlp(seed: int, widths: list[int], bias_scale: float = 0.1) -> list[tuple[np.ndarray, np.ndarray]]:
    """Glorot-uniform weights with non-zero N(0, bias_scale^2) biases, used by
    parity tests so that every bias term is exercised."""
    rng = np.random.default_rng(seed)
    layers = []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        w = rng.uniform(-lim, lim, (fan_out, fan_in))
        b = bias_scale * rng.standard_normal(fan_out)
        layers.append((np.ascontiguousarray(w), b))
    return layers


def permutation(seed: int, n: int) -> np.ndarray:
    """A random permutation of range(n), int64."""
    return np.random.default_rng(seed).permutation(n)
