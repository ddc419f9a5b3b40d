"""Batched form: many independent control problems of uneven size, one
gradient iteration for all of them per call (Section 3.2.1's optimisation
loop, instance by instance), with the forward and adjoint passes as single
persistent launches, the iteration captured in a HIP graph and the launch
shape chosen by the library's autotuner.  This module only marshals data in
and out of libmrt.so.
"""
from __future__ import annotations

from typing import List

import numpy as np
import torch

from . import abi
from .solver import make_problem_struct

FIELDS = {"u0": abi.MRT_FIELD_U0, "v0": abi.MRT_FIELD_V0,
          "control": abi.MRT_FIELD_CONTROL, "target": abi.MRT_FIELD_TARGET,
          "uN": abi.MRT_FIELD_UN, "vN": abi.MRT_FIELD_VN, "grad": abi.MRT_FIELD_GRAD}


class Batch:
    def __init__(self, problems: List, dtype=torch.float32, ckpt_every: int = 0,
                 mem_budget: int = 0, device="cuda:0"):
        self.problems = problems
        self.dtype = dtype
        self.device = torch.device(device)
        code = abi.MRT_F64 if dtype == torch.float64 else abi.MRT_F32
        self.structs = [make_problem_struct(p, code, int(p.nx), None) for p in problems]
        with torch.cuda.device(self.device):
            self.handle = abi.mrt_batch_create(self.structs, ckpt_every, mem_budget)
        for k, p in enumerate(problems):
            for name, arr in (("u0", p.u0), ("v0", p.v0), ("control", p.control),
                              ("target", p.u_target)):
                self.set(k, name, arr)
        torch.cuda.synchronize(self.device)

    @property
    def count(self) -> int:
        return len(self.problems)

    def set(self, k: int, name: str, arr) -> None:
        t = torch.as_tensor(np.ascontiguousarray(arr)).to(self.device, self.dtype).contiguous()
        abi.mrt_batch_copy(self.handle, k, FIELDS[name], True, t)
        torch.cuda.current_stream(self.device).synchronize()

    def get(self, k: int, name: str) -> torch.Tensor:
        L = int(self.problems[k].nx)
        t = torch.empty((L, L), dtype=self.dtype, device=self.device)
        abi.mrt_batch_copy(self.handle, k, FIELDS[name], False, t)
        return t

    def tune(self, steps: int = 20) -> dict:
        return abi.mrt_batch_tune(self.handle, steps)

    def set_tiles(self, tile_w: int, blocks_per_cu: int) -> None:
        abi.mrt_batch_set_tiles(self.handle, tile_w, blocks_per_cu)

    def tiles(self) -> dict:
        return abi.mrt_batch_get_tiles(self.handle)

    def set_timeout(self, seconds: float) -> None:
        abi.mrt_batch_set_timeout(self.handle, seconds)

    def iterate(self, zeta: float = 0.0, use_graph: bool = True) -> None:
        abi.mrt_batch_iteration(self.handle, zeta, use_graph)

    def forward(self) -> None:
        """Forward solves only (a batch created with ckpt_every < 0):
        writes uN and vN of every instance; raises on a barrier time-out."""
        abi.mrt_batch_forward(self.handle)

    def scalars(self):
        return abi.mrt_batch_scalars(self.handle, self.count)

    def close(self) -> None:
        if getattr(self, "handle", None):
            abi.mrt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
