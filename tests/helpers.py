"""Test helpers: layout conversion between the oracle (row-major cells) and the library (Morton)."""
import numpy as np


def morton_of_cells(level: int) -> np.ndarray:
    """For oracle cell c = x + s y + s^2 z, the library's Morton index (x bit lowest)."""
    s = 1 << level
    c = np.arange(s ** 3)
    x, y, z = c % s, (c // s) % s, c // (s * s)
    m = np.zeros_like(c)
    for b in range(level):
        m |= ((x >> b) & 1) << (3 * b)
        m |= ((y >> b) & 1) << (3 * b + 1)
        m |= ((z >> b) & 1) << (3 * b + 2)
    return m


def oracle_to_morton(a: np.ndarray, level: int) -> np.ndarray:
    out = np.empty_like(a)
    out[morton_of_cells(level)] = a
    return out


def morton_to_oracle(a: np.ndarray, level: int) -> np.ndarray:
    return a[morton_of_cells(level)]


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2)) / (den if den > 0 else 1.0))
