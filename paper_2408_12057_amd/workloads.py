"""Seeded synthetic workloads shaped like the paper's (and the benchmark
configurations built on them).  Pure data generation with numpy PCG64: no part
of the method's arithmetic lives here, so both the HIP path and the CPU oracle
can take their inputs from it.

Data seed for configuration c is ``default_rng(240812057 + c)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

DATA_SEED = 240812057


@dataclass
class Workload:
    name: str
    family: str              # "gauss" | "logreg" | "gmm"
    d: int
    ref_sigma2: float
    move: str
    params: dict = field(default_factory=dict)  # mu/sigma2, X/y, means/log_scales (float32)
    N: int = 1024
    T: int = 64
    leapfrog: int = 5
    eps0: float = 0.1


def gaussian_d10(N: int = 1024, T: int = 64) -> Workload:
    """Isotropic Gaussian target exp(-|x - 2 1|^2 / (2 * 0.25)) in d = 10, eta = N(0, I);
    RWMH with proposal standard deviation 0.5 / sqrt(d)."""
    d = 10
    return Workload("gauss_d10_rwmh", "gauss", d, 1.0, "rwmh",
                    dict(mu=np.full(d, 2.0, dtype=np.float32), sigma2=0.25), N=N, T=T,
                    eps0=0.5 / np.sqrt(d))


def logreg_data(n: int, d: int, seed: int) -> tuple:
    """X iid N(0,1) (fp32), theta* ~ N(0, I), y ~ Bernoulli(sigmoid(X theta*))."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)).astype(np.float32)
    theta = rng.standard_normal(d)
    z = X.astype(np.float64) @ theta
    p = 1.0 / (1.0 + np.exp(-z))
    y = (rng.random(n) < p).astype(np.float32)
    return X, y, theta


def logreg_n10000_d50(N: int = 16384, n: int = 10000, d: int = 50) -> Workload:
    """Bayesian logistic regression, X in R^{10000 x 50}, prior eta = N(0, I_50), MALA."""
    X, y, _ = logreg_data(n, d, DATA_SEED + 2)
    return Workload("logreg_n10000_d50_mala", "logreg", d, 1.0, "mala", dict(X=X, y=y), N=N,
                    T=1000, eps0=0.5 * d ** (-1.0 / 6.0))


def logreg_n5000_d200(N: int = 8192, n: int = 5000, d: int = 200) -> Workload:
    """Bayesian logistic regression at the batch's widest size, X in
    R^{5000 x 200}, prior eta = N(0, I_200), MALA (the panel layout)."""
    X, y, _ = logreg_data(n, d, DATA_SEED + 3)
    return Workload("logreg_n5000_d200_mala", "logreg", d, 1.0, "mala", dict(X=X, y=y), N=N,
                    T=512, eps0=0.5 * d ** (-1.0 / 6.0))


def gmm8_d100(N: int = 65536) -> Workload:
    """Equal-weight mixture of 8 Gaussians in d = 100: means iid N(0, 16 I),
    covariance 0.1 I, eta = N(0, 25 I); HMC with 5 leapfrog steps."""
    rng = np.random.default_rng(DATA_SEED + 3)
    d, K = 100, 8
    means = (4.0 * rng.standard_normal((K, d))).astype(np.float32)
    ls = np.full(K, 0.5 * np.log(0.1), dtype=np.float32)
    return Workload("gmm8_d100_hmc", "gmm", d, 25.0, "hmc", dict(means=means, log_scales=ls),
                    N=N, T=2000, leapfrog=5, eps0=0.5 * 5.0 * d ** (-0.25))


def gmm4_d20(N: int = 8192) -> Workload:
    """Mixture of K = 4 Gaussians in d = 20, means iid N(0, 4 I), log-scales 0,
    eta = N(0, 9 I); MALA."""
    rng = np.random.default_rng(DATA_SEED + 4)
    d, K = 20, 4
    means = (2.0 * rng.standard_normal((K, d))).astype(np.float32)
    ls = np.zeros(K, dtype=np.float32)
    return Workload("gmm4_d20_mala", "gmm", d, 9.0, "mala", dict(means=means, log_scales=ls),
                    N=N, T=256, eps0=0.5 * 3.0 * d ** (-1.0 / 6.0))


def random_gauss(rng: np.random.Generator, d: int) -> dict:
    return dict(mu=rng.normal(size=d).astype(np.float32), sigma2=float(rng.uniform(0.2, 2.0)))


def random_gmm(rng: np.random.Generator, d: int, K: int) -> dict:
    return dict(means=(1.5 * rng.normal(size=(K, d))).astype(np.float32),
                log_scales=rng.uniform(-0.6, 0.2, size=K).astype(np.float32))


def synthetic_logw(rng: np.random.Generator, N: int, scale: float = 3.0) -> np.ndarray:
    return rng.normal(scale=scale, size=N)


def batch_problems(n_problems: int = 256, seed_offset: int = 5, d_max_logreg: int = 200):
    """Independent problems of uneven size: family by a fair coin (the d-dimensional
    Gaussian target exp(-|x - 2 1|^2 / 0.5) with RWMH, or the logistic-regression
    generator with MALA), d uniform in [5, 200] (logistic regression: [5, d_max_logreg]),
    n uniform in [100, 5000], N in {2^8, ..., 2^16}, T in {2^5, ..., 2^10}.
    Returns a list of dicts (family, d, N, T, params, eps0, eps_kappa)."""
    rng = np.random.default_rng(DATA_SEED + seed_offset)
    out = []
    for p in range(n_problems):
        fam = "gauss" if rng.random() < 0.5 else "logreg"
        N = int(2 ** rng.integers(8, 17))
        T = int(2 ** rng.integers(5, 11))
        if fam == "gauss":
            d = int(rng.integers(5, 201))
            out.append(dict(family="gauss", d=d, N=N, T=T, move="rwmh",
                            params=dict(mu=np.full(d, 2.0, dtype=np.float32), sigma2=0.25),
                            eps0=0.5 / np.sqrt(d), eps_adapt=False, eps_kappa=0.0))
        else:
            d = int(rng.integers(5, d_max_logreg + 1))
            n = int(rng.integers(100, 5001))
            X, y, _ = logreg_data(n, d, DATA_SEED + 1000 + p)
            out.append(dict(family="logreg", d=d, N=N, T=T, move="mala", params=dict(X=X, y=y),
                            eps0=0.5 * d ** (-1.0 / 6.0), eps_adapt=True, eps_kappa=n / 4.0))
    return out
