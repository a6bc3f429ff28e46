"""Interval estimates used by the distributional GPU tests (plain formulas,
pinned by tests/test_stats_cpu.py to published worked examples)."""
import numpy as np

Z95 = 1.959963984540054


def wilson(k, n, z=Z95):
    """Wilson score interval of a proportion k/n (no continuity correction)."""
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return c - h, c + h


def newcombe_diff(k1, n1, k2, n2):
    """95% interval of p1 - p2 from the two Wilson intervals (Newcombe 1998,
    the hybrid score method)."""
    p1, p2 = k1 / n1, k2 / n2
    l1, u1 = wilson(k1, n1)
    l2, u2 = wilson(k2, n2)
    d = p1 - p2
    return d - np.sqrt((p1 - l1) ** 2 + (u2 - p2) ** 2), d + np.sqrt((u1 - p1) ** 2 + (p2 - l2) ** 2)
