"""Boundary conditions, loads and run presets for the synthetic workloads.

Conventions (both sides follow them; neither shares code with the other):

* A grid has ``nx * ny * nz`` unit hexahedral elements; node coordinates are
  integers ``(i, j, k)`` with ``0 <= i <= nx`` etc.  Axis x is the beam's
  length, y its width and z points up.
* A fixed degree of freedom is ``(i, j, k, c)`` with component ``c`` in
  {0: x, 1: y, 2: z}.  A point load is ``(i, j, k, c, value)``.

The geometries follow the paper's numerical examples: the cantilever clamped
at one end (Section 4.2.3 and the 2D cantilever of Section 4.1.1 lifted to
3D) and the simply supported beam whose four bottom corners are fixed with a
load at the bottom centre (Section 4.2.2).  Load layouts that exist only in
the paper's figures are replaced by the simple layouts below.
"""

from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

Fixed = Tuple[int, int, int, int]
Load = Tuple[int, int, int, int, float]


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    fixed: List[Fixed]
    loads: List[List[Load]]  # one list of point loads per load case
    name: str = ""

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_node(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def n_case(self) -> int:
        return len(self.loads)


def _trapezoid(n: int) -> np.ndarray:
    """Tributary lengths of the ``n + 1`` nodes of a unit-spaced segment."""
    w = np.ones(n + 1)
    if n == 0:
        return np.ones(1)
    w[0] = w[-1] = 0.5
    return w / n


def cantilever(nx: int, ny: int, nz: int) -> Problem:
    """Clamped x=0 face; unit downward force spread over the bottom edge of
    the x=nx face with trapezoid (tributary-length) weights summing to 1."""
    fixed = [(0, j, k, c) for k in range(nz + 1) for j in range(ny + 1) for c in range(3)]
    w = _trapezoid(ny)
    loads = [[(nx, j, 0, 2, -float(w[j])) for j in range(ny + 1)]]
    return Problem(nx, ny, nz, fixed, loads, f"cantilever{nx}x{ny}x{nz}")


def bridge(nx: int, ny: int, nz: int) -> Problem:
    """Simply supported beam: the four bottom-corner nodes fully fixed and a
    unit downward point load at the bottom-centre node (nx, ny even)."""
    corners = [(0, 0), (nx, 0), (0, ny), (nx, ny)]
    fixed = [(i, j, 0, c) for (i, j) in corners for c in range(3)]
    loads = [[(nx // 2, ny // 2, 0, 2, -1.0)]]
    return Problem(nx, ny, nz, fixed, loads, f"bridge{nx}x{ny}x{nz}")


def patch_test(nx: int, ny: int, nz: int, sigma: float = 1.0) -> Problem:
    """Symmetry-plane rollers (u_x=0 on x=0, u_y=0 on y=0, u_z=0 on z=0) and
    a uniform traction ``sigma`` in +x on the x=nx face, lumped to the face
    nodes by tributary area (the consistent load of a bilinear face)."""
    fixed = []
    for k in range(nz + 1):
        for j in range(ny + 1):
            fixed.append((0, j, k, 0))
    for k in range(nz + 1):
        for i in range(nx + 1):
            fixed.append((i, 0, k, 1))
    for j in range(ny + 1):
        for i in range(nx + 1):
            fixed.append((i, j, 0, 2))
    wy = _trapezoid(ny) * ny
    wz = _trapezoid(nz) * nz
    loads = [[(nx, j, k, 0, float(sigma * wy[j] * wz[k]))
              for k in range(nz + 1) for j in range(ny + 1)]]
    return Problem(nx, ny, nz, fixed, loads, f"patch{nx}x{ny}x{nz}")


def point_loads_on_face(nx: int, ny: int, nz: int, n_case: int, seed: int) -> Problem:
    """Clamped x=0 face; ``n_case`` load cases, each a unit downward point
    load at a seeded node of the x=nx face."""
    rng = np.random.default_rng(seed)
    fixed = [(0, j, k, c) for k in range(nz + 1) for j in range(ny + 1) for c in range(3)]
    loads = []
    for _ in range(n_case):
        j = int(rng.integers(0, ny + 1))
        k = int(rng.integers(0, nz + 1))
        loads.append([(nx, j, k, 2, -1.0)])
    return Problem(nx, ny, nz, fixed, loads, f"pointloads{nx}x{ny}x{nz}")


@dataclasses.dataclass
class Problem2D:
    """A plane-stress problem on an nx x ny grid of unit squares: nodes (i, j),
    fixed DOFs (i, j, c), point loads (i, j, c, value) per load case, and
    linear springs (i, j, c, stiffness) on single DOFs."""
    nx: int
    ny: int
    fixed: List[Tuple[int, int, int]]
    loads: List[List[Tuple[int, int, int, float]]]
    name: str = ""
    springs: List[Tuple[int, int, int, float]] = dataclasses.field(default_factory=list)

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny

    @property
    def n_node(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    @property
    def n_case(self) -> int:
        return len(self.loads)


def cantilever2d(nx: int, ny: int) -> Problem2D:
    """Section 4.1.1: the whole left side fully restrained, a unit downward
    point load at the midpoint of the right end (ny even)."""
    fixed = [(0, j, c) for j in range(ny + 1) for c in range(2)]
    return Problem2D(nx, ny, fixed, [[(nx, ny // 2, 1, -1.0)]], f"cantilever2d{nx}x{ny}")


def half_wheel(nx: int, ny: int) -> Problem2D:
    """Section 4.2.1: the lower-left corner fully constrained, the load-direction
    DOF of the lower-right corner constrained, a unit downward point load at
    the midpoint of the bottom edge (nx even)."""
    fixed = [(0, 0, 0), (0, 0, 1), (nx, 0, 1)]
    return Problem2D(nx, ny, fixed, [[(nx // 2, 0, 1, -1.0)]], f"halfwheel{nx}x{ny}")


def inverter2d(nx: int, ny: int, k_in: float = 1.0, k_out: float = 0.1) -> Problem2D:
    """Section 4.3's displacement inverter on the half domain below its axis of
    symmetry, taken as the bottom edge j = 0: the y DOFs of that edge fixed
    (symmetry), both DOFs of the two top nodes of the left side fixed
    (support), input point A = (0, 0) and output point B = (nx, 0) on the
    axis.  Load case 0 is the unit input force +x at A; load case 1 the unit
    dummy load +x at B, whose solution gives the output displacement's
    sensitivity.  Springs k_in at A and k_out at B, both in x."""
    fixed = [(i, 0, 1) for i in range(nx + 1)]
    fixed += [(0, ny, 0), (0, ny, 1), (0, ny - 1, 0), (0, ny - 1, 1)]
    loads = [[(0, 0, 0, 1.0)], [(nx, 0, 0, 1.0)]]
    springs = [(0, 0, 0, k_in), (nx, 0, 0, k_out)]
    return Problem2D(nx, ny, fixed, loads, f"inverter{nx}x{ny}", springs)


def batch_sizes(n: int, seed0: int = 4000, choices=(16, 24, 32, 40, 48, 56, 64),
                max_ratio: float = 2.0) -> List[Tuple[int, int, int]]:
    """Grid sizes of a batch of ``n`` cube-ish instances: instance i draws each
    axis i.i.d. from ``choices`` with generator seed ``seed0 + i``, redrawing
    until max/min <= ``max_ratio``."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        while True:
            d = [int(x) for x in rng.choice(choices, size=3)]
            if max(d) <= max_ratio * min(d):
                break
        out.append((d[0], d[1], d[2]))
    return out


def serve_trace(n: int, qps: float, seed: int = 5,
                sizes=((32, 32, 32), (48, 48, 48), (64, 64, 64), (96, 48, 48), (128, 128, 128)),
                repeat_frac: float = 0.5, w_max: float = 0.05, max_case: int = 8,
                sigma: float = 4.0) -> List[dict]:
    """A seeded stream of ``n`` analysis requests with Poisson arrivals at rate
    ``qps`` (exponential gaps from a generator of their own, so the requests
    are the same at every rate; ``qps`` <= 0: all at t = 0).

    A new design draws its grid uniformly from ``sizes``, 1..``max_case``
    load cases (clamped x=0, unit -z point loads at seeded x=nx face nodes)
    and a smoothed random density (correlation ``sigma`` voxels, [1e-3, 1]).
    With probability ``repeat_frac`` a request instead repeats an earlier
    design (its family: same grid and loads), perturbed by smoothed noise
    (correlation 2 voxels, like a filtered design update) of mean absolute
    density change w drawn uniformly from (0, ``w_max``] (the change measure
    of eq. 30).  Each request is a dict: rid, arrival [s], family, grid,
    n_case, load_seed, rho (float64, (nz, ny, nx))."""
    from .fields import smooth_perturb, smoothed_field

    rng = np.random.default_rng(seed)
    arr = np.random.default_rng([seed, 1])  # arrivals apart: same requests at any rate
    t = 0.0
    reqs: List[dict] = []
    families: List[dict] = []
    for rid in range(n):
        if qps > 0:
            t += float(arr.exponential(1.0 / qps))
        if families and rng.random() < repeat_frac:
            fam = families[int(rng.integers(0, len(families)))]
            w = float(rng.uniform(0.0, w_max)) or w_max
            rho = smooth_perturb(fam["rho"], w, seed=int(rng.integers(0, 2 ** 31)))
            fam["rho"] = rho
        else:
            nx, ny, nz = sizes[int(rng.integers(0, len(sizes)))]
            fam = dict(family=len(families), grid=(nx, ny, nz),
                       n_case=int(rng.integers(1, max_case + 1)),
                       load_seed=int(rng.integers(0, 2 ** 31)))
            fam["rho"] = smoothed_field(nx, ny, nz, sigma, 1e-3, 1.0,
                                        seed=int(rng.integers(0, 2 ** 31)))
            families.append(fam)
            rho = fam["rho"]
        reqs.append(dict(rid=rid, arrival=t, family=fam["family"], grid=fam["grid"],
                         n_case=fam["n_case"], load_seed=fam["load_seed"], rho=rho))
    return reqs


# Run presets of the synthetic workloads.  Material and method parameters are
# the paper's (E0=1, Emin=1e-9, nu=0.3, p=3; Section 4); grid sizes, radii,
# tolerances and level counts are the workload definitions.
PRESETS = {
    "cantilever24": dict(nx=24, ny=12, nz=12, rmin=1.5, levels=3, seed=1,
                         density="uniform", lo=0.3, hi=1.0),
    "cantilever96": dict(nx=96, ny=48, nz=48, rmin=2.0, levels=4, volfrac=0.3,
                         cycles=50, Nm=6, Ns=2, N_on=20, ca_tol=1e-3),
    "cantilever256": dict(nx=256, ny=128, nz=128, levels=6, seed=3,
                          density="smoothed", sigma=8.0, lo=1e-3, hi=1.0),
}
