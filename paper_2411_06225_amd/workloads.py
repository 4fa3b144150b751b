"""Seeded synthetic workloads: problem sizes, parameters, initial conditions and
random-network weights.

This module holds no arithmetic of the method.  It only describes the
workloads (grid, physical parameters, slices, propagators, network size) and
draws their seeded inputs, so that the GPU library and the CPU oracle are fed
identical arrays.  It imports neither of them.

The synthetic workloads stand in for the paper's experiments (Sec. 5 and
App. E/G): no dataset is involved, every initial condition is drawn from a
seeded numpy generator with the shape and value distribution stated below.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BURGERS1D, DIFFREACT2D, BRUSS2D, SWE2D, BRUSS3D = 0, 1, 2, 3, 4
NSPECIES = {BURGERS1D: 1, DIFFREACT2D: 2, BRUSS2D: 2, SWE2D: 3, BRUSS3D: 2}
TANH, RELU = 0, 1
RK1, RK4, RK8 = 1, 4, 8


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    kind: int
    nx: int
    ny: int
    domain: tuple          # (x0, x1, y0, y1)
    params: tuple          # see the kind
    N: int                 # slices
    t0: float
    tN: float
    F: tuple               # (method, steps per slice)
    G: tuple
    M: int                 # hidden neurons
    act: int
    lam: float
    eps: float
    ic: str                # initial-condition recipe name
    seed: int
    precision: str = "fp64"  # "fp64" (plain) or "mixed"
    nz: int = 1              # cells along z (3D Brusselator)

    @property
    def d(self) -> int:
        return NSPECIES[self.kind] * self.nx * self.ny * self.nz

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# -- the five workload families ------------------------------------------------
# 1: viscous Burgers, periodic [-1, 1], nu = 0.01, 128 points, N = 16, t in [0, 5],
#    F = RK4 x 2000, G = RK1 x 4 (forward Euler at this step is unstable for this
#    grid; the stabilised variant uses 40 steps), 100 tanh neurons.
BURGERS_D128 = Workload("burgers_d128", BURGERS1D, 128, 1, (-1.0, 1.0, -1.0, 1.0), (0.01,),
                        16, 0.0, 5.0, (RK4, 2000), (RK1, 4), 100, TANH, 1e-6, 1e-6,
                        "burgers_sines", 1)
BURGERS_D128_STABLE = BURGERS_D128.replace(name="burgers_d128_g40", G=(RK1, 40))

# 2: FitzHugh-Nagumo diffusion-reaction, (-1, 1)^2, 64 x 64 cells, Neumann walls,
#    Du = 1e-3, Dv = 5e-3, c = 5e-3, N = 64, t in [0, 20], F = RK4 x 4000,
#    G = RK1 x 10, 200 neurons (ReLU, the paper's activation), u, v ~ N(0, 1).
DIFFREACT_64 = Workload("diffreact_64x64", DIFFREACT2D, 64, 64, (-1.0, 1.0, -1.0, 1.0),
                        (1e-3, 5e-3, 5e-3), 64, 0.0, 20.0, (RK4, 4000), (RK1, 10), 200, RELU,
                        1e-6, 1e-6, "normal_fields", 2)

# 3: Brusselator, periodic (-1, 1)^2, 128 x 128, A = 1, B = 3, Du = 0.02, Dv = 0.01,
#    N = 128, t in [0, 30], F = RK4 x 10000, G = RK1 x 100, 100 neurons,
#    IC (A, B/A) + 0.1 U(-1, 1).
BRUSS_128 = Workload("bruss_128x128", BRUSS2D, 128, 128, (-1.0, 1.0, -1.0, 1.0),
                     (1.0, 3.0, 0.02, 0.01), 128, 0.0, 30.0, (RK4, 10000), (RK1, 100), 100, RELU,
                     1e-6, 1e-6, "bruss_perturbed", 3, "mixed")

# 5: shallow water, [0, 1]^2, 192 x 192, g = 9.81, reflective walls, N = 256,
#    t in [0, 1], F = RK4 x 1000, G = RK1 x 8, 300 neurons,
#    h = 1 + 4 Gaussian bumps (amplitude 0.1, width 0.05), zero velocity.
SWE_192 = Workload("swe_192x192", SWE2D, 192, 192, (0.0, 1.0, 0.0, 1.0), (9.81,), 256, 0.0, 1.0,
                   (RK4, 1000), (RK1, 8), 300, RELU, 1e-6, 1e-6, "gauss_bumps", 5, "mixed")

# App. E: Brusselator in three dimensions, periodic (-1, 1)^3, 20^3 cells
#    (d = 16000), A = 1, B = 3, Du = 0.1, Dv = 0.01, t in [0, 35], N = 512,
#    u = A, v ~ N(0, 1); F = the eighth-order method x 20 steps per slice,
#    G = RK1 x 8 (both inside their stability regions: the setup table's
#    coarse step 0.052 lies outside forward Euler's for this Laplacian),
#    100 ReLU neurons.
BRUSS3D_20 = Workload("bruss3d_20", BRUSS3D, 20, 20, (-1.0, 1.0, -1.0, 1.0), (1.0, 3.0, 0.1, 0.01), 512, 0.0, 35.0,
                      (RK8, 20), (RK1, 8), 100, RELU, 1e-6, 1e-6, "bruss3d_normal", 6, "fp64", nz=20)

WORKLOADS = {w.name: w for w in (BURGERS_D128, BURGERS_D128_STABLE, DIFFREACT_64, BRUSS_128, SWE_192, BRUSS3D_20)}


def cell_centres(n: int, a: float, b: float) -> np.ndarray:
    h = (b - a) / n
    return a + (np.arange(n) + 0.5) * h


def initial_condition(w: Workload, seed: int | None = None) -> np.ndarray:
    """Seeded initial state u0 (length d, float64) of workload w."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    x0, x1, y0, y1 = w.domain
    if w.ic == "burgers_sines":
        # u0(x) = sum_{k=1..4} a_k sin(k pi x), a_k ~ N(0, variance 0.25)
        x = x0 + np.arange(w.nx) * (x1 - x0) / w.nx
        a = rng.normal(0.0, 0.5, 4)
        return sum(a[k - 1] * np.sin(k * np.pi * x) for k in range(1, 5)).astype(np.float64)
    if w.ic == "normal_fields":
        u = rng.standard_normal((w.ny, w.nx))
        v = rng.standard_normal((w.ny, w.nx))
        return np.concatenate([u.ravel(), v.ravel()]).astype(np.float64)
    if w.ic == "bruss_perturbed":
        A, B = w.params[0], w.params[1]
        u = A + 0.1 * rng.uniform(-1.0, 1.0, (w.ny, w.nx))
        v = B / A + 0.1 * rng.uniform(-1.0, 1.0, (w.ny, w.nx))
        return np.concatenate([u.ravel(), v.ravel()]).astype(np.float64)
    if w.ic == "bruss3d_normal":
        # App. E: u = A everywhere, v normally distributed over the grid
        u = np.full((w.nz, w.ny, w.nx), w.params[0])
        v = rng.standard_normal((w.nz, w.ny, w.nx))
        return np.concatenate([u.ravel(), v.ravel()]).astype(np.float64)
    if w.ic == "gauss_bumps":
        xc = cell_centres(w.nx, x0, x1)
        yc = cell_centres(w.ny, y0, y1)
        X, Y = np.meshgrid(xc, yc)
        h = np.ones((w.ny, w.nx))
        centres = rng.uniform(0.15, 0.85, (4, 2))
        for cx, cy in centres:
            h += 0.1 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * 0.05 ** 2))
        z = np.zeros_like(h)
        return np.concatenate([h.ravel(), z.ravel(), z.ravel()]).astype(np.float64)
    raise ValueError(w.ic)


def random_weights(w: Workload, seed: int | None = None, d: int | None = None):
    """A (M x d) and zeta (M) with i.i.d. U(-1, 1) entries (Algorithm
    "RandNets training procedure", weight sampling), drawn from numpy."""
    rng = np.random.default_rng(100 + (w.seed if seed is None else seed))
    d = w.d if d is None else d
    A = rng.uniform(-1.0, 1.0, (w.M, d))
    zeta = rng.uniform(-1.0, 1.0, w.M)
    return A, zeta


def small(w: Workload, **kw) -> Workload:
    """A reduced copy of a workload for tests (same physics and recipe)."""
    return w.replace(name=w.name + "_small", **kw)


# -- batched workload (many Burgers instances of uneven size) -------------------
@dataclasses.dataclass(frozen=True)
class BatchWorkload:
    name: str
    instances: tuple       # tuple of Workload
    seed: int


def burgers_batch(n_inst: int = 64, sizes=(256, 512, 1024, 2048, 4096), N: int = 32,
                  tN: float = 5.0, M: int = 100, seed: int = 4) -> BatchWorkload:
    """n_inst periodic Burgers problems on [-1, 1] with d drawn from sizes and nu
    log-uniform in [1e-3, 1e-1].  Steps per slice are chosen so that both
    explicit solvers are inside their stability regions for u_max = 2:
    RK4 needs dt * rho <= 2.5, forward Euler dt <= 0.9 dx^2 / (2 nu) and
    dt <= 0.9 * 2 nu / u_max^2, with rho = 4 nu / dx^2 + u_max / dx."""
    rng = np.random.default_rng(seed)
    ds = rng.choice(np.asarray(sizes), n_inst)
    nus = 10.0 ** rng.uniform(-3.0, -1.0, n_inst)
    insts = []
    Ts = tN / N
    for b in range(n_inst):
        d, nu = int(ds[b]), float(nus[b])
        dx = 2.0 / d
        umax = 2.0
        rho = 4 * nu / dx ** 2 + umax / dx
        nf = max(2000, math.ceil(Ts * rho / 2.5))
        dtg = min(0.9 * dx ** 2 / (2 * nu), 0.9 * 2 * nu / umax ** 2)
        ng = max(4, math.ceil(Ts / dtg))
        insts.append(Workload(f"burgers_b{b}", BURGERS1D, d, 1, (-1.0, 1.0, -1.0, 1.0), (nu,), N,
                              0.0, tN, (RK4, nf), (RK1, ng), M, TANH, 1e-6, 1e-6, "burgers_sines",
                              1000 + b, "mixed"))
    return BatchWorkload(f"burgers_batch{n_inst}", tuple(insts), seed)
