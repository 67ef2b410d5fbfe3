"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random data and builds the paper's ground-truth covariance
matrices; it holds none of the measures' arithmetic and imports neither the HIP
library nor the oracle.  Every array is FP64, sample-major [T][N] (or
[D][T][N] for several datasets).

Workloads (the draw order is part of the definition):

* ``planted_10`` -- N=10, T=1000, seed 0: variables 0-2 are redundant copies of
  one latent source (x_i = z + 0.3 e_i), variables 3-5 a synergistic triplet
  (x5 = x3 + x4 + 0.3 e), variables 6-9 independent N(0,1).
* ``latent_20`` -- N=20, T=10000, seed 1: 4-factor model with U(-1,1)
  loadings plus unit noise and three planted synergistic triplets
  x_k = x_i + x_j + 0.2 e for (i,j,k) = (0,1,2), (3,4,5), (6,7,8).
* ``ar1_30`` -- N=30, T=1200, seed 2: AR(1) (phi = 0.5) sources through a random
  30x30 mixing matrix with N(0, 1/30) entries (fMRI-like).
* ``uneven_many`` -- seed 3: D datasets with N ~ U{10..40}, T ~ U{500..5000},
  each a k-factor model (k ~ U{1..5}, loadings U(-1,1), unit noise).
* ``latent_100`` -- N=100, T=2000, seed 4: 8 factors plus unit noise and five
  planted synergistic groups x_{4g+3} = x_{4g} + x_{4g+1} + x_{4g+2} + 0.2 e;
  plus a seeded batch of n-plets with order ~ U{8..20}.

The paper's benchmark data (Results, "Enhanced performance") is N=30 i.i.d.
N(0,1) with T=1000; its real datasets (fMRI, the 920-dataset collection) are
not available, so these generators stand in for them with the same shapes.
"""
from __future__ import annotations

import numpy as np


def planted_10(seed: int = 0, T: int = 1000) -> np.ndarray:
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(T)
    E = rng.standard_normal((T, 10))
    X = E.copy()
    X[:, 0:3] = z[:, None] + 0.3 * E[:, 0:3]
    X[:, 5] = E[:, 3] + E[:, 4] + 0.3 * E[:, 5]
    return X


def latent_20(seed: int = 1, T: int = 10000, N: int = 20) -> np.ndarray:
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((T, 4))
    L = rng.uniform(-1.0, 1.0, (N, 4))
    X = F @ L.T + rng.standard_normal((T, N))
    for (i, j, k) in ((0, 1, 2), (3, 4, 5), (6, 7, 8)):
        X[:, k] = X[:, i] + X[:, j] + 0.2 * rng.standard_normal(T)
    return X


def ar1_30(seed: int = 2, T: int = 1200, N: int = 30, phi: float = 0.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    M = rng.normal(0.0, 1.0 / np.sqrt(N), (N, N))
    S = np.empty((T, N))
    S[0] = rng.standard_normal(N) / np.sqrt(1.0 - phi * phi)
    for t in range(1, T):
        S[t] = phi * S[t - 1] + rng.standard_normal(N)
    return S @ M.T


def factor_model(rng: np.random.Generator, T: int, N: int, k: int) -> np.ndarray:
    F = rng.standard_normal((T, k))
    L = rng.uniform(-1.0, 1.0, (N, k))
    return F @ L.T + rng.standard_normal((T, N))


def uneven_many(D: int = 1024, seed: int = 3, n_lo: int = 10, n_hi: int = 40,
                t_lo: int = 500, t_hi: int = 5000):
    """List of D datasets [T_d][N_d] of uneven shapes."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(D):
        N = int(rng.integers(n_lo, n_hi + 1))
        T = int(rng.integers(t_lo, t_hi + 1))
        k = int(rng.integers(1, 6))
        out.append(factor_model(rng, T, N, k))
    return out


def latent_100(seed: int = 4, T: int = 2000, N: int = 100, B: int = 100000,
               k_lo: int = 8, k_hi: int = 20):
    """(X [T][N], n-plets [B][k_hi] int32 padded with -1)."""
    rng = np.random.default_rng(seed)
    X = factor_model(rng, T, N, 8)
    for g in range(5):
        a = 4 * g
        X[:, a + 3] = X[:, a] + X[:, a + 1] + X[:, a + 2] + 0.2 * rng.standard_normal(T)
    idx = -np.ones((B, k_hi), dtype=np.int32)
    ks = rng.integers(k_lo, k_hi + 1, size=B)
    for b in range(B):
        idx[b, : ks[b]] = np.sort(rng.choice(N, size=int(ks[b]), replace=False))
    return X, idx


def replicas_20(D: int, seed: int = 1, T: int = 10000) -> np.ndarray:
    """D independent draws of the latent_20 model, stacked as [D][T][20]."""
    return np.stack([latent_20(seed=seed + 1000 * d, T=T) for d in range(D)])


# --------------------------------------------------------------------------- ground-truth covariances
def s_system(n: int, c: float) -> np.ndarray:
    """Synergy system (Supplementary, PGMs): X_1..X_n independent, Y depends on all.

    Sigma = [[I_n, c 1], [c 1^T, n c^2 + 1]].
    """
    S = np.eye(n + 1)
    S[:n, n] = c
    S[n, :n] = c
    S[n, n] = n * c * c + 1.0
    return S


def r_system(n: int, c: float) -> np.ndarray:
    """Redundancy system (Supplementary, PGMs): X_i conditionally independent given Y.

    Sigma = [[c^2 11^T + I_n, c 1], [c 1^T, 1]].
    """
    S = np.full((n + 1, n + 1), c * c)
    S[np.arange(n), np.arange(n)] = c * c + 1.0
    S[:n, n] = c
    S[n, :n] = c
    S[n, n] = 1.0
    return S


def block_diag(*blocks: np.ndarray) -> np.ndarray:
    n = sum(b.shape[0] for b in blocks)
    out = np.zeros((n, n))
    o = 0
    for b in blocks:
        m = b.shape[0]
        out[o:o + m, o:o + m] = b
        o += m
    return out


def concatenated_100() -> np.ndarray:
    """The 100-variable concatenated system: weak/strong R, weak/strong S (c = 0.5 / 1,
    each 19 X's + Y) and 20 independent variables."""
    return block_diag(r_system(19, 0.5), r_system(19, 1.0), s_system(19, 0.5), s_system(19, 1.0), np.eye(20))


def random_spd(rng: np.random.Generator, n: int, cond: float = 100.0) -> np.ndarray:
    """A random symmetric positive-definite matrix with the given condition number."""
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.exp(rng.uniform(0.0, np.log(cond), n))
    ev[0], ev[-1] = 1.0, cond
    A = (Q * ev) @ Q.T
    return 0.5 * (A + A.T)


def random_nplets(rng: np.random.Generator, N: int, B: int, k_lo: int, k_hi: int) -> np.ndarray:
    idx = -np.ones((B, k_hi), dtype=np.int32)
    ks = rng.integers(k_lo, k_hi + 1, size=B)
    for b in range(B):
        idx[b, : ks[b]] = np.sort(rng.choice(N, size=int(ks[b]), replace=False))
    return idx


# --------------------------------------------------------------------------- search inputs
def sa_initial(seed: int, kappa: int, N: int, k_lo: int, k_hi: int) -> np.ndarray:
    """kappa random n-plets as boolean masks [kappa][N]: order ~ U{k_lo..k_hi}, members uniform
    without replacement."""
    rng = np.random.default_rng(seed)
    masks = np.zeros((kappa, N), dtype=bool)
    for j in range(kappa):
        k = int(rng.integers(k_lo, k_hi + 1))
        masks[j, rng.choice(N, size=k, replace=False)] = True
    return masks


def sa_draws(seed: int, iters: int, kappa: int) -> dict:
    """Uniform [0, 1) draws consumed by the annealing searches: per (iteration, chain) one for the
    move type, one to pick a member, one to pick an outsider and one for acceptance."""
    rng = np.random.default_rng(seed)
    u = rng.random((4, iters, kappa))
    return {"move": u[0], "a": u[1], "b": u[2], "accept": u[3]}


def condition_pairs(P: int, seed: int = 7, N: int = 12, T: int = 1500, planted=(2, 5, 9)) -> np.ndarray:
    """P subjects x 2 conditions, stacked [2P][T][N] (condition A for rows 0..P-1, B for P..2P-1,
    subject p in rows p and P + p).  Every dataset is 2-factor data with subject-specific loadings
    U(-1, 1) and unit noise; in condition A the planted triplet (i, j, k) has x_k = x_i + x_j +
    0.5 eps (synergy), in condition B x_k is replaced by independent noise of the same variance."""
    rng = np.random.default_rng(seed)
    i, j, k = planted
    out = np.empty((2 * P, T, N))
    for p in range(P):
        L = rng.uniform(-1.0, 1.0, (N, 2))
        for c in range(2):
            X = rng.standard_normal((T, 2)) @ L.T + rng.standard_normal((T, N))
            syn = X[:, i] + X[:, j] + 0.5 * rng.standard_normal(T)
            X[:, k] = syn if c == 0 else rng.standard_normal(T) * syn.std()
            out[c * P + p] = X
    return out
