"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the eigensolver or of the finite-element
discretisation.  It only draws random numbers and evaluates the synthetic
potential at coordinates that the caller supplies (each side computes its own
node coordinates).

Workloads (Hartree atomic units: energies in Ha, lengths in bohr):

* ``"small"``   -- cube L=10, 4^3 cells, GLL degree 4 (3,375 interior DoFs),
  4 Gaussian wells of depth 2 Ha and width 1 bohr, 16 states, filter degree 20.
* ``"large_p6"`` -- cube L=40, 24^3 cells, degree 6 (2,924,207 DoFs), 64 wells,
  512 states, filter degree 30, filter block 128.
* ``"large_p5"`` -- the same 64 wells on 32^3 cells, degree 5 (4,019,679 DoFs),
  1024 states, filter degree 30, filter block 128.
* ``"batch"``   -- 64 independent problems drawn by :func:`batch_problems`.

Random-number conventions: ``numpy.random.Generator(PCG64(seed))``; wells draw
centres (well-major, x,y,z), then depths, then widths; the start block X0 is
standard normal, DoF-major (row = DoF, column = state), from seed ``seed+100``.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Wells:
    centres: np.ndarray  # [n, 3]
    depths: np.ndarray   # [n] (positive; the well value is -depth at its centre)
    widths: np.ndarray   # [n] standard deviation of the Gaussian, bohr


@dataclasses.dataclass(frozen=True)
class Problem:
    name: str
    L: float
    n_el: int
    p: int
    nstates: int
    degree: int
    block_width: int
    well_seed: int
    x0_seed: int
    n_wells: int
    depth_range: tuple  # (lo, hi); lo == hi means fixed
    width_range: tuple

    @property
    def n_dof(self) -> int:
        return (self.n_el * self.p - 1) ** 3

    @property
    def nblock(self) -> int:
        return block_size(self.nstates)


def block_size(nstates: int) -> int:
    """States plus guard states: N + max(4, ceil(0.1 N)), rounded up to 8."""
    nb = nstates + max(4, -(-nstates // 10))
    return -(-nb // 8) * 8


PROBLEMS = {
    "small": Problem("small", 10.0, 4, 4, 16, 20, 24, 1, 101, 4, (2.0, 2.0), (1.0, 1.0)),
    "large_p6": Problem("large_p6", 40.0, 24, 6, 512, 30, 128, 2, 102, 64, (1.0, 3.0), (0.5, 1.5)),
    "large_p5": Problem("large_p5", 40.0, 32, 5, 1024, 30, 128, 2, 103, 64, (1.0, 3.0), (0.5, 1.5)),
}


def draw_wells(n: int, L: float, seed: int, depth_range=(1.0, 3.0), width_range=(0.5, 1.5)) -> Wells:
    """Draw n Gaussian wells inside [3 w_max, L - 3 w_max]^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    wmax = float(width_range[1])
    lo, hi = 3.0 * wmax, L - 3.0 * wmax
    centres = rng.uniform(lo, hi, size=(n, 3))
    if depth_range[0] == depth_range[1]:
        depths = np.full(n, float(depth_range[0]))
    else:
        depths = rng.uniform(depth_range[0], depth_range[1], size=n)
    if width_range[0] == width_range[1]:
        widths = np.full(n, float(width_range[0]))
    else:
        widths = rng.uniform(width_range[0], width_range[1], size=n)
    return Wells(centres, depths, widths)


def problem_wells(prob: Problem) -> Wells:
    return draw_wells(prob.n_wells, prob.L, prob.well_seed, prob.depth_range, prob.width_range)


def eval_wells(w: Wells, xyz: np.ndarray, chunk: int = 1 << 20) -> np.ndarray:
    """V(x) = -sum_k d_k exp(-|x - c_k|^2 / (2 w_k^2)) at points xyz [n, 3]."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    out = np.empty(xyz.shape[0], dtype=np.float64)
    inv2w2 = 1.0 / (2.0 * w.widths ** 2)
    for s in range(0, xyz.shape[0], chunk):
        pts = xyz[s:s + chunk]
        acc = np.zeros(pts.shape[0])
        for k in range(w.centres.shape[0]):
            d = pts - w.centres[k]
            acc -= w.depths[k] * np.exp(-(d * d).sum(axis=1) * inv2w2[k])
        out[s:s + chunk] = acc
    return out


def harmonic(xyz: np.ndarray, omega: float, centre) -> np.ndarray:
    """V(x) = 1/2 omega^2 |x - centre|^2 (a separable test potential)."""
    d = np.asarray(xyz, dtype=np.float64).reshape(-1, 3) - np.asarray(centre, dtype=np.float64)
    return 0.5 * omega * omega * (d * d).sum(axis=1)


def start_block(n_dof: int, ncols: int, seed: int, ld: int | None = None) -> np.ndarray:
    """Seeded N(0,1) start block, DoF-major [n_dof, ld] (columns >= ncols are zero)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((n_dof, ncols))
    if ld is None or ld == ncols:
        return x
    out = np.zeros((n_dof, ld))
    out[:, :ncols] = x
    return out


def perturbed(v: np.ndarray, seed: tuple, rel: float = 0.01) -> np.ndarray:
    """V * (1 + rel * xi), xi ~ N(0,1) per node, seeded by a tuple (stream, request, solve)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    return v * (1.0 + rel * rng.standard_normal(v.shape[0]))


def batch_problems(count: int = 64, seed: int = 4):
    """Problem list of the batched workload: n_el in {4..12}, p in {4..7},
    L = 2.5 n_el, N in {16..256}, max(4, round(L^3/1000)) wells; problem i
    uses well seed 4000 + i and start-block seed 4100 + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    probs = []
    for i in range(count):
        n_el = int(rng.integers(4, 13))
        p = int(rng.integers(4, 8))
        nst = int(rng.integers(16, 257))
        L = 2.5 * n_el
        nw = max(4, int(round(L ** 3 / 1000.0)))
        nd = (n_el * p - 1) ** 3
        nst = min(nst, max(16, nd // 8))
        probs.append(Problem(f"batch{i}", L, n_el, p, nst, 20, 0, 4000 + i, 4100 + i,
                             nw, (1.0, 3.0), (0.5, 1.5)))
    return probs


def fmt_problem(prob: Problem) -> str:
    return (f"{prob.name}: L={prob.L:g} n_el={prob.n_el} p={prob.p} n_dof={prob.n_dof} "
            f"N={prob.nstates} N_b={prob.nblock} m={prob.degree}")


__all__ = ["Wells", "Problem", "PROBLEMS", "block_size", "draw_wells", "problem_wells",
           "eval_wells", "harmonic", "start_block", "perturbed", "batch_problems", "fmt_problem"]


def start_block_device(n_dof: int, ncols: int, seed: int, device="cuda:0", ld: int | None = None):
    """Seeded N(0,1) start block generated on the GPU (torch's Philox generator),
    DoF-major [n_dof, ld]; used where a host-generated block would be too slow."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    ld = ncols if ld is None else ld
    x = torch.zeros((n_dof, ld), dtype=torch.float64, device=device)
    x[:, :ncols] = torch.randn((n_dof, ncols), generator=g, dtype=torch.float64, device=device)
    return x[:, :ncols] if ld != ncols else x
