"""Helpers shared by the GPU tests: device vectors from the seeded inputs and
oracle objects (the oracle runs on the CPU; nothing here computes the method)."""
import sys

import numpy as np
import torch

DEV = "cuda:0"


def dvec(a: np.ndarray) -> torch.Tensor:
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def announce(*what):
    print("CASE", *what, flush=True)
    sys.stdout.flush()
