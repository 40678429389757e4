"""Morton (Z-order) ordering of 2-D locations — oracle (test infrastructure only).

Section VI assumes "an appropriate ordering" of the locations so that strong
correlations sit near the diagonal.  The reading used throughout: each
coordinate is quantised to 16 bits, q = min(floor(c * 2^16), 2^16 - 1), with
c clamped to [0, 1]; the key interleaves the bits of q_x into the even bit
positions (bit 0 = the least significant bit of q_x) and those of q_y into
the odd positions, giving a 32-bit key.  Points are sorted by ascending key;
equal keys keep their input order (stable sort).  For (longitude, latitude)
locations in degrees (great-circle distance), the key is that of
((lon + 180) / 360, (lat + 90) / 180).
"""
from __future__ import annotations

import numpy as np


def _quantise(c: float) -> int:
    c = min(max(float(c), 0.0), 1.0)
    return min(int(np.floor(c * 65536.0)), 65535)


def morton_key(x: float, y: float) -> int:
    """The 32-bit Z-order key of one point, bit by bit."""
    qx, qy = _quantise(x), _quantise(y)
    key = 0
    for bit in range(16):
        key |= ((qx >> bit) & 1) << (2 * bit)
        key |= ((qy >> bit) & 1) << (2 * bit + 1)
    return key


def morton_keys(locs: np.ndarray, metric: str = "euclidean") -> np.ndarray:
    """Keys of all points (uint32), computed one point at a time."""
    pts = np.asarray(locs, dtype=np.float64)
    if metric == "gcd":
        pts = np.stack([(pts[:, 0] + 180.0) / 360.0, (pts[:, 1] + 90.0) / 180.0], axis=1)
    return np.array([morton_key(x, y) for x, y in pts], dtype=np.uint32)


def morton_order(locs: np.ndarray, metric: str = "euclidean") -> np.ndarray:
    """Permutation perm (int64) with locs[perm] in ascending key order, ties by index."""
    return np.argsort(morton_keys(locs, metric), kind="stable").astype(np.int64)
