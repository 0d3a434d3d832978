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
    """||a - b||_2 / ||b||_2 over all entries (complex entries by their modulus). Real and complex
    arrays are not mixed: comparing a complex result with a real reference (or the reverse)
    raises, so that no imaginary part is dropped silently."""
    a = np.asarray(a)
    b = np.asarray(b)
    if np.iscomplexobj(a) != np.iscomplexobj(b):
        raise TypeError("rel(): one argument is complex and the other is real")
    dt = np.complex128 if np.iscomplexobj(a) else np.float64
    a = a.astype(dt)
    b = b.astype(dt)
    den = np.sqrt(np.sum(np.abs(b) ** 2))
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2)) / (den if den > 0 else 1.0))
