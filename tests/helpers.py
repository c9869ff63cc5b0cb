"""Small test helpers (no ADMM arithmetic)."""
import numpy as np


def slot_z(problem) -> np.ndarray:
    """z index of every edge slot in user slot order."""
    off = problem.var_offsets()
    out = []
    for g in problem.groups:
        for row in g.var_ids:
            for v in row:
                out.extend(range(off[v], off[v + 1]))
    return np.asarray(out, dtype=np.int64)


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def have_gpu() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
