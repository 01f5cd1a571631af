"""CPU replay of the request loop's results -- TEST INFRASTRUCTURE ONLY
(tests, smoke and the benchmark's CPU leg).

Each client's state starts as the identity; its j-th product (j counting all
products the client has received, over its requests in arrival order)
replaces the state S by F_j S, F_j = philox.factor(seed, client, j, n,
sqrt(3 / n)), computed by the binary64 oracle (alpha 1, beta 0).  The final
states therefore depend only on each client's total number of products, not
on timing or on how clients were batched together.

Parity status: pinned in tests/test_serve_host.py (identity start, first
factor exact, two-factor chain against numpy's matmul).
"""
from __future__ import annotations

import math

import numpy as np

import oracle
from oracle import philox


def scale(n: int) -> float:
    return math.sqrt(3.0 / n)


def final_state(seed: int, client: int, n: int, products: int) -> np.ndarray:
    """State of a client of size n after `products` products (ordinary
    n x n array)."""
    S = np.eye(n)
    for j in range(products):
        F = philox.factor(seed, client, j, n, scale(n))
        # column-major storage (cols, ld) of F, S and the result
        C = np.zeros((n, n))
        oracle.gemm("N", "N", n, n, n, 1.0, np.ascontiguousarray(F.T), n,
                    np.ascontiguousarray(S.T), n, 0.0, C, n)
        S = C.T.copy()
    return S


def products_per_client(num_clients: int, clients, lengths) -> np.ndarray:
    tot = np.zeros(num_clients, dtype=np.int64)
    np.add.at(tot, np.asarray(clients), np.asarray(lengths))
    return tot
