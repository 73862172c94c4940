"""Batches of independent CSR matrices of uneven sizes as one block-diagonal
matrix, so every op of the library runs once over the whole batch (one
launch per kernel instead of one per block).

Rows of different blocks never interact: each row (or column, or level) is
processed by exactly the same arithmetic as in a solo run, so batched
results equal per-block results bit for bit, and the level sets of the
batch are the union of the blocks' level sets (a row keeps its level).
"""
from __future__ import annotations

import numpy as np
import torch

from . import gen
from . import sparse as sp


class Batch:
    def __init__(self, blocks, dtype=torch.float32, device="cuda"):
        """blocks: list of square host Csr matrices."""
        big, brp = gen.block_diag(blocks)
        self.host = big
        self.block_rowptr = brp.astype(np.int64)
        self.A = sp.CsrTensor.from_host(big, dtype=dtype, device=device)
        self.nblocks = len(blocks)

    @property
    def pattern(self):
        return self.A.pattern

    def split(self, v):
        """Per-block views of a vector (or rows of a matrix) over the batch."""
        return [v[int(a):int(b)] for a, b in zip(self.block_rowptr[:-1], self.block_rowptr[1:])]

    def concat(self, parts):
        return torch.cat(list(parts), dim=0)


def geometric_batch(nblocks, n_range=(1024, 65536), k_range=(6, 14), first=0):
    """Host blocks of the batched workload: random geometric-graph
    Laplacians + 1e-2 I (gen.geometric_graph_laplacian), blocks first ..
    first + nblocks - 1."""
    return [gen.geometric_graph_laplacian(b, n_range=n_range, k_range=k_range)
            for b in range(first, first + nblocks)]
