"""Input preparation on the GPU (outside the merge path).

Sub-index graphs and recall ground truth need exact k-NN lists. They are
inputs of the merge, not steps of it: the k-NN here uses a float32 matrix
product (exact for the integer-valued workloads: every product and partial
sum is an integer below 2**24) and a top-k on int64 keys distance * n + id,
which orders ties by id exactly like the (distance, id) order of the method.
The graph itself is then built by librnsm (rnsm_build_graph).
"""
from __future__ import annotations

import torch


@torch.no_grad()
def knn_l2_exact(base: torch.Tensor, queries: torch.Tensor | None, K: int,
                 exclude_self: bool = False, block: int = 4096) -> torch.Tensor:
    """Top-K ids (int32, [nq, K]) of every query row by (squared L2, id).

    base, queries: float32 CUDA tensors holding integers (|x| small enough
    that squared norms stay below 2**24). With exclude_self the queries are
    the base rows themselves and each row's own id is skipped.
    """
    assert base.dtype == torch.float32 and base.is_cuda
    q_all = base if queries is None else queries
    n = base.shape[0]
    assert n < (1 << 31) // 1 and float(base.abs().max()) < 4096
    sq = (base * base).sum(1)
    assert float(sq.max()) < 2 ** 24, "squared norms must stay exact in float32"
    out = torch.empty((q_all.shape[0], K), dtype=torch.int32, device=base.device)
    ids = torch.arange(n, device=base.device, dtype=torch.int64)
    kk = K + 1 if exclude_self else K
    prev = torch.backends.cuda.matmul.allow_tf32
    torch.backends.cuda.matmul.allow_tf32 = False
    try:
        for s in range(0, q_all.shape[0], block):
            q = q_all[s:s + block]
            qs = (q * q).sum(1)
            d = torch.addmm(qs[:, None] + sq[None, :], q, base.t(), beta=1.0, alpha=-2.0)
            key = d.to(torch.int64).clamp_(min=0) * n + ids[None, :]
            del d
            if exclude_self:
                r = torch.arange(s, s + q.shape[0], device=base.device)
                key[torch.arange(q.shape[0], device=base.device), r] = torch.iinfo(torch.int64).max
            top = torch.topk(key, kk, dim=1, largest=False, sorted=True).values
            del key
            out[s:s + q.shape[0]] = (top[:, :K] % n).to(torch.int32)
    finally:
        torch.backends.cuda.matmul.allow_tf32 = prev
    return out


@torch.no_grad()
def knn_float_exact(base: torch.Tensor, queries: torch.Tensor | None, K: int, metric: int = 0,
                    exclude_self: bool = False, block: int = 4096) -> torch.Tensor:
    """Top-K ids (int32, [nq, K]) of every query row by float32 distance:
    squared L2 (metric 0) or 1 - <q, x> (metric 1), brute force. For
    real-valued data, where equal distances practically never occur; the
    order among exactly equal distances is topk's, not by id."""
    assert base.dtype == torch.float32 and base.is_cuda and metric in (0, 1)
    q_all = base if queries is None else queries
    n = base.shape[0]
    sq = (base * base).sum(1) if metric == 0 else None
    out = torch.empty((q_all.shape[0], K), dtype=torch.int32, device=base.device)
    kk = K + 1 if exclude_self else K
    prev = torch.backends.cuda.matmul.allow_tf32
    torch.backends.cuda.matmul.allow_tf32 = False
    try:
        for s in range(0, q_all.shape[0], block):
            q = q_all[s:s + block]
            if metric == 0:
                d = torch.addmm((q * q).sum(1)[:, None] + sq[None, :], q, base.t(), beta=1.0,
                                alpha=-2.0)
            else:
                d = torch.addmm(torch.ones((), device=base.device), q, base.t(), beta=1.0,
                                alpha=-1.0)
            if exclude_self:
                r = torch.arange(s, s + q.shape[0], device=base.device)
                d[torch.arange(q.shape[0], device=base.device), r] = float("inf")
            top = torch.topk(d, kk, dim=1, largest=False, sorted=True).indices
            del d
            out[s:s + q.shape[0]] = top[:, :K].to(torch.int32)
    finally:
        torch.backends.cuda.matmul.allow_tf32 = prev
    return out
