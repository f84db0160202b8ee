"""Seeded generators for meshes, coefficients and vectors (no method arithmetic).

Every generator draws from its own numpy stream ``rng_for(seed, tag)`` so that
changing one quantity never shifts the random numbers of another.

Mesh family (Section 3, the meshes M_N): the unit square split into N x N
squares with two triangles each, or the unit cube split into N^3 cubes with six
Kuhn tetrahedra each.  Vertex (i, j[, l]) has id i + (N+1)(j + (N+1) l).  The
paper calls its meshes irregular without giving the perturbation; ``jitter``
moves interior vertices by U[-jitter, jitter]/N per coordinate (jitter <= 0.15
keeps every simplex valid: the smallest altitude of these simplices is h/sqrt(2)).
"""

from __future__ import annotations

import concurrent.futures
import itertools
import os

import numpy as np

__all__ = [
    "rng_for",
    "unit_mesh",
    "cell_centroids",
    "coef_uniform",
    "coef_aniso_2d",
    "coef_aniso_3d",
    "gaussian_field_rff",
    "coef_lognormal",
    "theta_normal",
    "random_vector",
    "batch_spec",
    "WORKLOADS",
]

_TAGS = {
    "jitter": 1,
    "coef": 2,
    "aniso": 3,
    "rff": 4,
    "theta": 5,
    "vector": 6,
    "batch": 7,
    "noise": 8,
}


def rng_for(seed: int, tag: str, sub: int = 0) -> np.random.Generator:
    """Independent numpy stream for (seed, quantity, sub-index)."""
    return np.random.default_rng(np.random.SeedSequence([int(seed), _TAGS[tag], int(sub)]))


def unit_mesh(dim: int, n: int, jitter: float = 0.0, seed: int = 0):
    """Structured simplex mesh of the unit square (dim=2) or cube (dim=3).

    Returns (coords float64 [nv, dim], cells int32 [nc, dim+1]).
    2D: square (i, j) gives triangles (v00, v10, v11) and (v00, v11, v01).
    3D: cube (i, j, l) gives one tetrahedron per axis permutation p, walking
    v000 -> +e_p0 -> +e_p1 -> +e_p2 = v111 (Kuhn subdivision).
    Cells are ordered by cell index i + n(j + n l), then by the sub-simplex.
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    axes = [np.arange(m, dtype=np.float64) / n] * dim
    grid = np.meshgrid(*axes, indexing="ij")
    # vertex id = i + m*j (+ m*m*l): i is the fastest index
    coords = np.stack([g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grid], axis=1)
    coords = np.ascontiguousarray(coords)

    idx = np.arange(n)
    if dim == 2:
        J, I = np.meshgrid(idx, idx, indexing="ij")
        I = I.reshape(-1)
        J = J.reshape(-1)

        def vid(di, dj):
            return (I + di) + m * (J + dj)

        v00, v10, v11, v01 = vid(0, 0), vid(1, 0), vid(1, 1), vid(0, 1)
        cells = np.stack(
            [np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)], axis=1
        ).reshape(-1, 3)
    else:
        L, J, I = np.meshgrid(idx, idx, idx, indexing="ij")
        I = I.reshape(-1)
        J = J.reshape(-1)
        L = L.reshape(-1)

        def vid(o):
            return (I + o[0]) + m * ((J + o[1]) + m * (L + o[2]))

        tets = []
        for p in itertools.permutations((0, 1, 2)):
            o = [0, 0, 0]
            path = [vid(o)]
            for ax in p:
                o = list(o)
                o[ax] += 1
                path.append(vid(o))
            tets.append(np.stack(path, 1))
        cells = np.stack(tets, axis=1).reshape(-1, 4)
    cells = np.ascontiguousarray(cells, dtype=np.int32)

    if jitter:
        if not (0.0 <= jitter <= 0.15):
            raise ValueError("jitter must lie in [0, 0.15]")
        rng = rng_for(seed, "jitter", dim * 100000 + n)
        disp = rng.uniform(-jitter, jitter, size=coords.shape) / n
        interior = np.all((coords > 0.5 / n) & (coords < 1.0 - 0.5 / n), axis=1)
        coords = coords + disp * interior[:, None]
    return coords, cells


def cell_centroids(coords: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """Mean of the vertices of every cell, float64 [nc, dim]."""
    return coords[cells].mean(axis=1)


def coef_uniform(nel: int, lo: float, hi: float, seed: int, sub: int = 0) -> np.ndarray:
    """Piecewise-constant scalar coefficient ~ U[lo, hi] per element."""
    return rng_for(seed, "coef", sub).uniform(lo, hi, size=nel)


def coef_aniso_2d(nel: int, seed: int, lam_lo: float = 1.0, lam_hi: float = 100.0) -> np.ndarray:
    """Per-element SPD 2x2 tensor Q(phi) diag(l1, l2) Q(phi)^T, phi ~ U[0, pi), l ~ U[lo, hi].

    Returned packed as the upper triangle row by row: [M00, M01, M11], shape [nel, 3].
    """
    rng = rng_for(seed, "aniso", 2)
    phi = rng.uniform(0.0, np.pi, size=nel)
    lam = rng.uniform(lam_lo, lam_hi, size=(nel, 2))
    c, s = np.cos(phi), np.sin(phi)
    m00 = c * c * lam[:, 0] + s * s * lam[:, 1]
    m11 = s * s * lam[:, 0] + c * c * lam[:, 1]
    m01 = c * s * (lam[:, 0] - lam[:, 1])
    return np.stack([m00, m01, m11], axis=1)


def coef_aniso_3d(nel: int, seed: int, lam_lo: float = 1.0, lam_hi: float = 100.0) -> np.ndarray:
    """Per-element SPD 3x3 tensor Q diag(l) Q^T with Q a random rotation, l ~ U[lo, hi].

    Packed upper triangle row by row: [M00, M01, M02, M11, M12, M22], shape [nel, 6].
    """
    rng = rng_for(seed, "aniso", 3)
    g = rng.standard_normal(size=(nel, 3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    lam = rng.uniform(lam_lo, lam_hi, size=(nel, 3))
    m = np.einsum("eij,ej,ekj->eik", q, lam, q)
    iu = np.triu_indices(3)
    return np.ascontiguousarray(m[:, iu[0], iu[1]])


def gaussian_field_rff(points: np.ndarray, seed: int, ell: float = 0.1, std: float = 1.0,
                       n_features: int = 1024, chunk: int = 65536) -> np.ndarray:
    """Zero-mean Gaussian random field with squared-exponential covariance.

    Random Fourier features: g(x) = std sqrt(2/K) sum_k cos(w_k . x + b_k), with
    w_k ~ N(0, ell^-2 I) and b_k ~ U[0, 2 pi).  Covariance -> std^2 exp(-|x-y|^2 / (2 ell^2)).
    """
    dim = points.shape[1]
    rng = rng_for(seed, "rff", dim)
    w = rng.standard_normal(size=(n_features, dim)) / ell
    b = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
    out = np.empty(points.shape[0])
    scale = std * np.sqrt(2.0 / n_features)

    def one(s):
        p = points[s:s + chunk]
        out[s:s + chunk] = scale * np.cos(p @ w.T + b).sum(axis=1)

    # chunks on host threads (numpy releases the GIL): every chunk is computed the same
    # way as on one thread, so the field is the same bit for bit
    starts = range(0, points.shape[0], chunk)
    workers = min(16, os.cpu_count() or 1, len(starts))
    if workers <= 1:
        for s in starts:
            one(s)
    else:
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            list(ex.map(one, starts))
    return out


def coef_lognormal(coords: np.ndarray, cells: np.ndarray, seed: int, ell: float = 0.1,
                   std: float = 1.0) -> np.ndarray:
    """a_T = exp(g(centroid_T)) with g the Gaussian field above."""
    return np.exp(gaussian_field_rff(cell_centroids(coords, cells), seed, ell=ell, std=std))


def theta_normal(nel: int, seed: int, sigma: float = 0.5, sub: int = 0) -> np.ndarray:
    """Per-element log-coefficient theta ~ N(0, sigma^2)."""
    return rng_for(seed, "theta", sub).normal(0.0, sigma, size=nel)


def random_vector(n: int, seed: int, sub: int = 0) -> np.ndarray:
    """Trial vector with entries ~ U[-1, 1]."""
    return rng_for(seed, "vector", sub).uniform(-1.0, 1.0, size=n)


def batch_spec(count: int, seed: int, n_lo: int = 32, n_hi: int = 256, k_lo: int = 1, k_hi: int = 4):
    """Uneven batch of 2D problems: N ~ round(logU[n_lo, n_hi]), k ~ U{k_lo..k_hi}.

    Returns a list of (n, k, coefficient_seed_sub) tuples.
    """
    rng = rng_for(seed, "batch")
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(int)
    ks = rng.integers(k_lo, k_hi + 1, size=count)
    return [(int(n), int(k), i) for i, (n, k) in enumerate(zip(ns, ks))]


# Named workloads: the synthetic stand-ins for the experiments the hot path is measured on.
WORKLOADS = {
    "c1_2d16_p2_se": dict(dim=2, n=16, k=2, kind="se", coef="uniform", lo=1.0, hi=10.0, bc="dirichlet"),
    "c2_2d512_wp": dict(dim=2, n=512, ks=(1, 2, 3, 4, 5), kind="wp", coef="uniform", lo=1.0, hi=100.0, bc="none"),
    "c2_2d512_se": dict(dim=2, n=512, ks=(1, 2, 3, 4, 5), kind="se", coef="aniso", bc="dirichlet"),
    "c3_3d64_se": dict(dim=3, n=64, ks=(2, 3), kind="se", coef="lognormal", bc="dirichlet"),
    "c4_2d256_p3_inverse": dict(dim=2, n=256, k=3, kind="se", coef="theta", sigma=0.5, bc="dirichlet"),
    "c5_batch256": dict(dim=2, count=256, n_lo=32, n_hi=256, k_lo=1, k_hi=4, kind="se", coef="uniform",
                        lo=1.0, hi=10.0, bc="dirichlet"),
}
