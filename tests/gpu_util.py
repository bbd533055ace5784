"""Helpers of the GPU tests: device transfers and the problems they use."""
import numpy as np
import torch

import workloads as W


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel_err(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


# Small problems spanning several tiles and ragged edges (the grids are
# not multiples of any block shape), in 2-D and 3-D, both modes.
def step_problems():
    return {
        "bubble2d_200x136": W.bubble_problem("b2", 2, (200, 136), [(0.45, 0.35)], [0.2],
                                             W.P0, 10 * W.P0, div_amp=1e-6, div_seed=3),
        "bubble3d_40x24x56": W.bubble_problem("b3", 3, (40, 24, 56), [(0.5, 0.3, 0.6)], [0.3],
                                              100 * W.P0, 0.01 * W.P0, div_amp=1e-7, div_seed=5),
        "explicit_64": W.explicit_const(64, 64),
        "twobubble2d_96x80": W.bubble_problem("b4", 2, (96, 80), [(0.3, 0.4), (0.7, 0.4)],
                                              [0.15, 0.12], W.P0, W.P0, div_amp=1e-6, div_seed=9),
    }
