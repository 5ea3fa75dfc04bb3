"""Helpers shared by the GPU parity tests (host side only)."""

from __future__ import annotations

import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def rand_state(rng: np.random.Generator, N: int) -> np.ndarray:
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return v / np.linalg.norm(v)


def f_rel_err(f: float, f_ref: float, psi_ref: np.ndarray | None, q: np.ndarray) -> float:
    """|f - f_ref| / sum_j |psi_j|^2 |q_j| (equals |f_ref| when q >= 0)."""
    if psi_ref is not None:
        scale = float(np.sum(np.abs(psi_ref) ** 2 * np.abs(q)))
    else:
        scale = abs(f_ref)
    return abs(f - f_ref) / max(scale, 1e-300)


def state_err(psi: np.ndarray, psi_ref: np.ndarray) -> float:
    """2-norm of the difference of two (unit-norm) states."""
    return float(np.linalg.norm(psi - psi_ref))
