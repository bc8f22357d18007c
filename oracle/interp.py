"""Lagrange interpolation weights in product form (oracle side).

For nodes x_0..x_{M-1} and an evaluation point x the degree-(M-1)
interpolant is sum_j w_j(x) f_j with
    w_j(x) = prod_{k != j} (x - x_k) / (x_j - x_k).
This is the textbook definition; it is used for every polynomial
interpolation step of Secs. 3.2 and 3.4.  Works for float64 and
numpy.longdouble (the dtype of ``nodes`` decides).
"""
import numpy as np


def lagrange_weights(nodes, x):
    """nodes: [..., M]; x: [...] -> weights [..., M] in the dtype of ``nodes``."""
    nodes = np.asarray(nodes)
    x = np.asarray(x, dtype=nodes.dtype)[..., None]
    M = nodes.shape[-1]
    w = np.ones(np.broadcast_shapes(nodes.shape, x.shape), dtype=nodes.dtype)
    for j in range(M):
        for k in range(M):
            if k == j:
                continue
            w[..., j] *= (x[..., 0] - nodes[..., k]) / (nodes[..., j] - nodes[..., k])
    return w
