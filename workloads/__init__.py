"""Seeded synthetic inputs for the Allen-Cahn CTD solver.

This module only draws numbers: problem parameters and the nodal values of
initial cosine modes.  It holds none of the method's arithmetic (no shape
functions, no quadrature, no solves), so both the GPU path and the CPU oracle
may import it.

Initial condition recipe: each initial mode is a rank-one product of
cos(k*pi*(x-lo)/(hi-lo)) per axis (these satisfy the homogeneous Neumann
condition of the weak form), with integer k drawn uniformly from [1, kmax]
per axis and mode.  Amplitudes are drawn uniformly in [-1, 1] and rescaled
so that the sum of their absolute values is 0.9; since |cos| <= 1 this puts
u0 inside [-0.9, 0.9] everywhere (equality at the origin when all amplitudes
share a sign).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

# Named workloads.  Keys are descriptive, values are the raw problem statement.
# Fields not fixed by the workload description inherit: s=2, p=2 (patch size 2,
# quadratic reproduction), a=12 (dilation, natural element units), 5 Gauss
# points per element, fixed-point tolerance 1e-2 with at most 20 sweeps,
# enrichment tolerance 1e-8.
CONFIGS = {
    "ac2d_n128": dict(dim=2, nodes=128, eps=0.02, S=2.0, dt=1e-3, steps=50,
                      m0=4, kmax=8, enrich_tol=1e-8, max_modes=64),
    "ac3d_n256": dict(dim=3, nodes=256, eps=0.01, S=2.0, dt=5e-4, steps=100,
                      m0=8, kmax=16, enrich_tol=1e-8, max_modes=64),
    "ac3d_n1024": dict(dim=3, nodes=1024, eps=0.005, S=2.0, dt=2e-4, steps=200,
                       m0=8, kmax=16, enrich_tol=1e-8, max_modes=128),
    "batch2d_512": dict(dim=2, instances=512, nodes_range=(64, 2048),
                        eps_range=(0.005, 0.05), dt_range=(1e-4, 1e-3),
                        m0_range=(4, 16), kmax=8, S=2.0, steps=100,
                        enrich_tol=1e-8, max_modes=64),
    "serve_mix": dict(rate=200.0, requests=10000, p3d=0.2,
                      nodes2d_range=(64, 2048), nodes3d_range=(64, 512),
                      steps_range=(20, 500), eps_range=(0.005, 0.05),
                      dt_range=(1e-4, 1e-3), m0_range=(4, 16), kmax2d=8,
                      kmax3d=16, S=2.0, enrich_tol=1e-8, max_modes=64),
}

CONFIG_IDS = {name: i for i, name in enumerate(CONFIGS)}

DEFAULTS = dict(lo=0.0, hi=1.0, patch_s=2, poly_p=2, dilation_a=12.0,
                gauss_points=5, fp_tol=1e-2, fp_max_iter=20, seed=0)


@dataclass
class Instance:
    """One Allen-Cahn CTD problem: raw parameters plus initial modes."""
    dim: int
    nodes: tuple
    eps: float
    S: float
    dt: float
    steps: int
    amp: np.ndarray                      # (m0,)
    factors: list                        # dim arrays, nodes[d] x m0, column = mode
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    patch_s: int = 2
    poly_p: int = 2
    dilation_a: float = 12.0
    gauss_points: int = 5
    fp_tol: float = 1e-2
    fp_max_iter: int = 20
    enrich_tol: float = 1e-8
    max_modes: int = 64
    seed: int = 0
    extra: dict = field(default_factory=dict)

    def params(self) -> dict:
        d = asdict(self)
        d.pop("amp"); d.pop("factors")
        return d


def _rng(seed):
    return np.random.default_rng(np.random.SeedSequence(seed))


def cosine_modes(rng, dim, nodes, m0, kmax, lo=(0.0,) * 3, hi=(1.0,) * 3):
    """Nodal values of m0 seeded rank-one cosine products and their amplitudes."""
    k = rng.integers(1, kmax + 1, size=(m0, dim))
    amp = rng.uniform(-1.0, 1.0, size=m0)
    amp *= 0.9 / np.abs(amp).sum()
    factors = []
    for d in range(dim):
        n = nodes[d]
        t = np.arange(n, dtype=np.float64) / (n - 1)        # (x - lo)/(hi - lo)
        factors.append(np.ascontiguousarray(
            np.cos(np.pi * t[:, None] * k[:, d][None, :].astype(np.float64))))
    return amp.astype(np.float64), factors


def make_instance(name: str, seed: int | None = None, **overrides) -> Instance:
    """Single-instance workload by name (ac2d_n128, ac3d_n256, ac3d_n1024)."""
    cfg = dict(DEFAULTS)
    cfg.update(CONFIGS[name])
    cfg.update(overrides)
    if seed is None:
        seed = CONFIG_IDS.get(name, 0)
    rng = _rng(seed)
    dim = cfg["dim"]
    n = cfg["nodes"]
    nodes = tuple(n if isinstance(n, int) else n[d] for d in range(dim))
    amp, factors = cosine_modes(rng, dim, nodes, cfg["m0"], cfg["kmax"])
    return Instance(dim=dim, nodes=nodes, eps=cfg["eps"], S=cfg["S"],
                    dt=cfg["dt"], steps=cfg["steps"], amp=amp, factors=factors,
                    patch_s=cfg["patch_s"], poly_p=cfg["poly_p"],
                    dilation_a=cfg["dilation_a"],
                    gauss_points=cfg["gauss_points"], fp_tol=cfg["fp_tol"],
                    fp_max_iter=cfg["fp_max_iter"],
                    enrich_tol=cfg["enrich_tol"], max_modes=cfg["max_modes"],
                    seed=seed)


def _log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def make_batch(name: str = "batch2d_512", seed: int | None = None,
               count: int | None = None, **overrides) -> list:
    """Uneven 2D instances: nodes log-uniform, eps and dt uniform, 4..16 modes."""
    cfg = dict(DEFAULTS)
    cfg.update(CONFIGS[name])
    cfg.update(overrides)
    if seed is None:
        seed = CONFIG_IDS[name]
    root = np.random.SeedSequence(seed)
    total = cfg["instances"]
    out = []
    for i, child in enumerate(root.spawn(total)):
        if count is not None and i >= count:
            break
        rng = np.random.default_rng(child)
        n = _log_uniform_int(rng, *cfg["nodes_range"])
        eps = rng.uniform(*cfg["eps_range"])
        dt = rng.uniform(*cfg["dt_range"])
        m0 = int(rng.integers(cfg["m0_range"][0], cfg["m0_range"][1] + 1))
        amp, factors = cosine_modes(rng, 2, (n, n), m0, cfg["kmax"])
        out.append(Instance(dim=2, nodes=(n, n), eps=eps, S=cfg["S"], dt=dt,
                            steps=cfg["steps"], amp=amp, factors=factors,
                            patch_s=cfg["patch_s"], poly_p=cfg["poly_p"],
                            dilation_a=cfg["dilation_a"],
                            gauss_points=cfg["gauss_points"],
                            fp_tol=cfg["fp_tol"], fp_max_iter=cfg["fp_max_iter"],
                            enrich_tol=cfg["enrich_tol"],
                            max_modes=cfg["max_modes"], seed=seed * 100003 + i))
    return out


def make_requests(name: str = "serve_mix", seed: int | None = None,
                  count: int | None = None, **overrides) -> list:
    """Poisson request stream: (arrival_time_s, Instance) pairs."""
    cfg = dict(DEFAULTS)
    cfg.update(CONFIGS[name])
    cfg.update(overrides)
    if seed is None:
        seed = CONFIG_IDS[name]
    root = np.random.SeedSequence(seed)
    total = cfg["requests"] if count is None else count
    arr_rng = np.random.default_rng(root.spawn(1)[0])
    gaps = arr_rng.exponential(1.0 / cfg["rate"], size=total)
    t = np.cumsum(gaps)
    out = []
    for i, child in enumerate(root.spawn(total)):
        rng = np.random.default_rng(child)
        is3d = rng.uniform() < cfg["p3d"]
        dim = 3 if is3d else 2
        n = _log_uniform_int(rng, *(cfg["nodes3d_range"] if is3d
                                    else cfg["nodes2d_range"]))
        eps = rng.uniform(*cfg["eps_range"])
        dt = rng.uniform(*cfg["dt_range"])
        steps = int(rng.integers(cfg["steps_range"][0], cfg["steps_range"][1] + 1))
        m0 = int(rng.integers(cfg["m0_range"][0], cfg["m0_range"][1] + 1))
        kmax = cfg["kmax3d"] if is3d else cfg["kmax2d"]
        amp, factors = cosine_modes(rng, dim, (n,) * dim, m0, kmax)
        inst = Instance(dim=dim, nodes=(n,) * dim, eps=eps, S=cfg["S"], dt=dt,
                        steps=steps, amp=amp, factors=factors,
                        patch_s=cfg["patch_s"], poly_p=cfg["poly_p"],
                        dilation_a=cfg["dilation_a"],
                        gauss_points=cfg["gauss_points"], fp_tol=cfg["fp_tol"],
                        fp_max_iter=cfg["fp_max_iter"],
                        enrich_tol=cfg["enrich_tol"],
                        max_modes=cfg["max_modes"], seed=seed * 100003 + i)
        out.append((float(t[i]), inst))
    return out


def small_instance(dim=2, n=24, m0=3, kmax=4, seed=7, **kw) -> Instance:
    """Tiny seeded instance for parity tests (several tiles plus a ragged tail)."""
    rng = _rng(seed)
    nodes = (n,) * dim if isinstance(n, int) else tuple(n)
    amp, factors = cosine_modes(rng, dim, nodes, m0, kmax)
    base = dict(eps=0.05, S=2.0, dt=1e-3, steps=3, enrich_tol=1e-8, max_modes=32)
    base.update(kw)
    return Instance(dim=dim, nodes=nodes, amp=amp, factors=factors, seed=seed,
                    **base)
