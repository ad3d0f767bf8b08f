"""Shared helpers of the GPU parity tests (the HIP path through the C ABI)."""
from __future__ import annotations

import sys

import numpy as np

import oracle

TOL = {"fp32": 1e-5, "fp64": 1e-10}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_plan(prob, precision="fp32", **kw):
    from paper_2101_08072_amd import Options, Plan
    return Plan.from_problem(prob, options=Options(precision=precision, **kw))


def to_dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda").to(dtype).contiguous()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return oracle.rel_l2(a, b)
