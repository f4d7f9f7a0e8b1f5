"""Pack seeded synthetic potentials into a batch's device input buffer (torch).

Plumbing only: the fine-mesh potential of an item is the linear combination
sum_t c_t U_t of the unit-coefficient term matrices from ``configs``; the
combination is formed on the device so that thousands of items can be staged
without host traffic.  Nothing of the wave-packet method happens here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import configs


def pack_host_matrices(u_elems: int, u_off, mats, dtype, device="cuda") -> torch.Tensor:
    u = torch.empty(int(u_elems), dtype=dtype, device=device)
    for off, m in zip(u_off, mats):
        flat = torch.from_numpy(np.ascontiguousarray(m, dtype=np.float64).ravel())
        u[int(off):int(off) + flat.numel()].copy_(flat.to(dtype))
    return u


def pack_coupled_yukawa(u_elems: int, u_off, nodes: np.ndarray, coeffs: np.ndarray, dtype, device="cuda",
                        J: int = 1, chunk: int = 64, terms=None) -> torch.Tensor:
    """Items i = 0..len(coeffs)-1 of equal size with contiguous offsets.

    ``terms`` may pass precomputed ``configs.coupled_yukawa_terms(nodes, J)``.
    """
    if terms is None:
        terms = configs.coupled_yukawa_terms(nodes, J)
    t = torch.from_numpy(np.stack([x.ravel() for x in terms])).to(device)
    per = t.shape[1]
    u_off = np.asarray(u_off)
    if not np.array_equal(u_off, np.arange(len(coeffs)) * per):
        raise ValueError("pack_coupled_yukawa needs equal, contiguous items")
    c = torch.as_tensor(np.asarray(coeffs), dtype=torch.float64, device=device)
    u = torch.empty(int(u_elems), dtype=dtype, device=device)
    for s in range(0, len(coeffs), chunk):
        e = min(len(coeffs), s + chunk)
        u[s * per:e * per].view(e - s, per).copy_((c[s:e] @ t).to(dtype))
    return u
