"""Test helpers shared by the parity tests (no method arithmetic)."""

from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def match_dofs(product_xyz: np.ndarray, oracle_xyz: np.ndarray, tol: float = 1e-9) -> np.ndarray:
    """perm with product dof i located at oracle dof perm[i] (matched by coordinates)."""
    assert product_xyz.shape == oracle_xyz.shape
    dist, idx = cKDTree(oracle_xyz).query(product_xyz)
    assert dist.max() <= tol, f"unmatched dof, distance {dist.max()}"
    assert len(np.unique(idx)) == len(idx), "dof matching is not one to one"
    return idx


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def header_functions(path: str) -> list[str]:
    """Names of the functions declared in a C header."""
    import re

    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dogip_[a-z0-9_]+)\s*\(", txt)))
