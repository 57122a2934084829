"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds *problem definitions only*: periodic split-Cartesian meshes
(element vertex ids and physical vertex coordinates), smooth mesh warps, and
initial states in primitive variables.  It contains none of the method's
arithmetic (no quadrature, operators, geometry, projection or fluxes); the
oracle and the library each compute those on their own from these inputs.

Workloads follow the paper's numerical experiments (periodic boxes, 2 triangles
per square / 6 tetrahedra per cube, smooth sinusoidal warps, Euler states of
density-wave, vortex and Taylor-Green type), with the sizes of the benchmark
configurations used in this project.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

GAMMA = 1.4


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
@dataclass
class Mesh:
    """Conforming simplicial mesh of a periodic box.

    elem_vertex_ids    int64 [n_elements, dim+1]   global vertex ids; periodic
                       images of a vertex share one id.
    elem_vertex_coords float64 [n_elements, dim+1, dim] physical coordinates of
                       each element's vertices (unwrapped: an element lies
                       inside its own cell of the Cartesian grid).
    box                float64 [dim] periodic lengths.
    """

    dim: int
    elem_vertex_ids: np.ndarray
    elem_vertex_coords: np.ndarray
    box: np.ndarray
    M: int = 0

    @property
    def n_elements(self) -> int:
        return int(self.elem_vertex_ids.shape[0])


def split_box_mesh(dim: int, M: int, L: float, origin: float = 0.0) -> Mesh:
    """Cartesian grid of M cells per direction on [origin, origin+L]^dim,
    each square split into 2 triangles along its (0,0)-(1,1) diagonal, each
    cube into the 6 Kuhn tetrahedra 0 -> e_a -> e_a+e_b -> (1,1,1)."""
    h = L / M
    if dim == 2:
        local = [((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1))]
    elif dim == 3:
        local = []
        for perm in itertools.permutations(range(3)):
            p0 = (0, 0, 0)
            p1 = [0, 0, 0]
            p1[perm[0]] = 1
            p2 = list(p1)
            p2[perm[1]] = 1
            local.append((p0, tuple(p1), tuple(p2), (1, 1, 1)))
    else:
        raise ValueError("dim must be 2 or 3")
    ids = []
    coords = []
    for cell in itertools.product(range(M), repeat=dim):
        cell = cell[::-1]  # x fastest
        for simplex in local:
            vid = []
            vx = []
            for corner in simplex:
                g = [cell[k] + corner[k] for k in range(dim)]
                gid = 0
                for k in reversed(range(dim)):
                    gid = gid * M + (g[k] % M)
                vid.append(gid)
                vx.append([origin + h * g[k] for k in range(dim)])
            ids.append(vid)
            coords.append(vx)
    return Mesh(dim, np.asarray(ids, dtype=np.int64),
                np.asarray(coords, dtype=np.float64),
                np.full(dim, L, dtype=np.float64), M)


# --------------------------------------------------------------------------
# warps (problem geometry; applied to the physical positions of mapping nodes)
# --------------------------------------------------------------------------
def warp_none(x: np.ndarray) -> np.ndarray:
    return np.array(x, dtype=np.float64, copy=True)


def make_warp_sinprod(L: float, amp: float) -> Callable[[np.ndarray], np.ndarray]:
    """x_i <- x_i + amp * prod_k sin(2 pi x_k / L), every coordinate evaluated
    at the unwarped point.  Vanishes on the periodic boundary, so the warped
    mesh stays periodic and conforming."""

    def warp(x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        s = np.prod(np.sin(2.0 * math.pi * x / L), axis=-1, keepdims=True)
        return x + amp * s

    return warp


# --------------------------------------------------------------------------
# states (primitive variables rho, v, p  ->  conservative u)
# --------------------------------------------------------------------------
def prim_to_cons(rho, v, p, gamma=GAMMA):
    rho = np.asarray(rho, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    mom = rho[..., None] * v
    E = p / (gamma - 1.0) + 0.5 * rho * np.sum(v * v, axis=-1)
    return np.concatenate([rho[..., None], mom, E[..., None]], axis=-1)


def density_wave(x, L=2.0, gamma=GAMMA):
    """rho = 1 + 0.2 sin(2 pi/L sum x), v = 1, p = 1 (periodic)."""
    x = np.asarray(x, dtype=np.float64)
    d = x.shape[-1]
    rho = 1.0 + 0.2 * np.sin(2.0 * math.pi / L * np.sum(x, axis=-1))
    v = np.ones(x.shape[:-1] + (d,))
    p = np.ones(x.shape[:-1])
    return prim_to_cons(rho, v, p, gamma)


def isentropic_vortex(x, beta=5.0, center=(5.0, 5.0), vinf=(1.0, 1.0), t=0.0, gamma=GAMMA):
    x = np.asarray(x, dtype=np.float64)
    X = x[..., 0] - center[0] - vinf[0] * t
    Y = x[..., 1] - center[1] - vinf[1] * t
    r2 = X * X + Y * Y
    f = np.exp(0.5 * (1.0 - r2))
    du = -beta / (2.0 * math.pi) * f * Y
    dv = beta / (2.0 * math.pi) * f * X
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    v = np.stack([vinf[0] + du, vinf[1] + dv], axis=-1)
    return prim_to_cons(rho, v, p, gamma)


def taylor_green(x, Ma=0.1, gamma=GAMMA):
    """rho=1, v=(sin x cos y cos z, -cos x sin y cos z, 0),
    p = 1/(gamma Ma^2) + (cos2x + cos2y)(cos2z + 2)/16."""
    x = np.asarray(x, dtype=np.float64)
    a, b, c = x[..., 0], x[..., 1], x[..., 2]
    rho = np.ones_like(a)
    v = np.stack([np.sin(a) * np.cos(b) * np.cos(c),
                  -np.cos(a) * np.sin(b) * np.cos(c),
                  np.zeros_like(a)], axis=-1)
    p = 1.0 / (gamma * Ma * Ma) + (np.cos(2 * a) + np.cos(2 * b)) * (np.cos(2 * c) + 2.0) / 16.0
    return prim_to_cons(rho, v, p, gamma)


@dataclass
class RandomSmooth:
    """q = c + a * Phi(x), Phi a random trigonometric polynomial with modes
    |k|_inf <= kmax on the box, coefficients N(0,1) normalised by their
    absolute sum so that |Phi| <= 1.  One Phi per primitive variable."""

    dim: int
    L: float
    seed: int
    kmax: int = 2
    _coef: list = field(default_factory=list, init=False, repr=False)

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        modes = np.array(list(itertools.product(range(-self.kmax, self.kmax + 1), repeat=self.dim)),
                         dtype=np.float64)
        self._modes = modes
        for _ in range(self.dim + 2):
            cs = rng.standard_normal((modes.shape[0], 2))
            cs /= np.sum(np.abs(cs))
            self._coef.append(cs)

    def _phis(self, x, chunk=1 << 18):
        """All dim + 2 polynomials at the points x [n][dim]: a cos(k.x) +
        b sin(k.x) = Re((a - i b) exp(i k.x)), exp(i k.x) the product of the
        per-direction factors (no transcendental per mode), in chunks of points."""
        ks = np.arange(-self.kmax, self.kmax + 1, dtype=np.float64)
        nk = ks.size
        C = np.stack([cs[:, 0] - 1j * cs[:, 1] for cs in self._coef], axis=1)   # [mode][polynomial]
        out = np.empty((x.shape[0], len(self._coef)))
        w = 2.0 * math.pi / self.L
        for s in range(0, x.shape[0], chunk):
            xc = x[s:s + chunk]
            e = [np.exp(1j * w * np.multiply.outer(xc[:, d], ks)) for d in range(self.dim)]
            E = e[0]
            for d in range(1, self.dim):   # modes in the order of itertools.product
                E = (E[:, :, None] * e[d][:, None, :]).reshape(xc.shape[0], -1)
            assert E.shape[1] == nk ** self.dim
            out[s:s + chunk] = (E @ C).real
        return out

    def __call__(self, x, gamma=GAMMA):
        x = np.asarray(x, dtype=np.float64)
        shp = x.shape[:-1]
        xf = x.reshape(-1, self.dim)
        ph = self._phis(xf)
        rho = 1.0 + 0.2 * ph[:, 0]
        v = np.stack([0.299 / math.sqrt(3.0) * ph[:, 1 + k] for k in range(self.dim)], axis=-1)
        p = 1.0 + 0.2 * ph[:, self.dim + 1]
        return prim_to_cons(rho, v, p, gamma).reshape(shp + (self.dim + 2,))


# --------------------------------------------------------------------------
# benchmark configurations
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    dim: int
    M: int
    L: float
    degree: int
    warp: Callable[[np.ndarray], np.ndarray]
    state: Callable[[np.ndarray], np.ndarray]
    ecflux: int          # 0 Ranocha, 1 Chandrashekar
    dissipation: int     # 0 entropy-conservative interface, 1 local Lax-Friedrichs (Davis)
    gamma: float = GAMMA

    def mesh(self) -> Mesh:
        return split_box_mesh(self.dim, self.M, self.L)


def density_wave_tri(M=8, degree=2, ecflux=1, dissipation=0) -> Workload:
    """128 affine triangles on [0,2]^2, p=2, density wave."""
    return Workload(f"density_wave_tri_M{M}_p{degree}", 2, M, 2.0, degree, warp_none,
                    lambda x: density_wave(x, 2.0), ecflux, dissipation)


def vortex_tri(M=64, degree=4) -> Workload:
    """2*64^2 curved triangles on [0,10]^2, isentropic vortex, LF dissipation."""
    return Workload(f"vortex_tri_M{M}_p{degree}", 2, M, 10.0, degree,
                    make_warp_sinprod(10.0, 0.05), isentropic_vortex, 0, 1)


def tgv_tet(M=16, degree=4, dissipation=0) -> Workload:
    """6*M^3 curved tetrahedra on [0,2pi]^3, Taylor-Green flow at Ma 0.1."""
    L = 2.0 * math.pi
    return Workload(f"tgv_tet_M{M}_p{degree}", 3, M, L, degree,
                    make_warp_sinprod(L, 0.05), taylor_green, 0, dissipation)


def random_tet(M=4, degree=3, seed=20231213, dissipation=1) -> Workload:
    L = 2.0 * math.pi
    return Workload(f"random_tet_M{M}_p{degree}_s{seed}", 3, M, L, degree,
                    make_warp_sinprod(L, 0.05), RandomSmooth(3, L, seed), 0, dissipation)


def random_tri(M=4, degree=3, seed=7, dissipation=1, L=2.0) -> Workload:
    return Workload(f"random_tri_M{M}_p{degree}_s{seed}", 2, M, L, degree,
                    make_warp_sinprod(L, 0.05 * L / (2 * math.pi)), RandomSmooth(2, L, seed), 0, dissipation)


def mixed_degrees(n_elements: int, seed: int, lo: int = 2, hi: int = 10) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=n_elements).astype(np.int32)


@dataclass
class Batch:
    """Several independent meshes with per-element degrees."""
    name: str
    dim: int
    meshes: list          # [Mesh]
    degrees: list         # [np.ndarray int32 per mesh]
    L: float
    warp: Callable
    state: Callable
    ecflux: int = 0
    dissipation: int = 1
    gamma: float = GAMMA


def batched_tets(Ms=(8, 10, 12, 14), lo=2, hi=10, seed=20231213) -> Batch:
    """Periodic [0,2pi]^3 meshes of 6 M^3 curved tetrahedra, element degrees
    uniform on {lo..hi} from one seeded generator, random smooth Euler state
    (rho, p in [0.8, 1.2], |v| < 0.3), Ranocha flux with LF dissipation."""
    L = 2.0 * math.pi
    rng = np.random.default_rng(seed)
    meshes = [split_box_mesh(3, M, L) for M in Ms]
    degs = [rng.integers(lo, hi + 1, size=m.n_elements).astype(np.int32) for m in meshes]
    name = f"batched_tets_M{'-'.join(str(M) for M in Ms)}_p{lo}-{hi}"
    return Batch(name, 3, meshes, degs, L, make_warp_sinprod(L, 0.05), RandomSmooth(3, L, seed))


def kelvin_helmholtz(x, gamma=GAMMA):
    """Kelvin-Helmholtz instability on (0,2)^2 (Sec. 7.5): B = tanh(15(y-1/2)) -
    tanh(15(y-3/2)), rho = 1/2 + 3B/4, v = (B-1)/2, sin(2 pi x)/10, p = 1."""
    x = np.asarray(x, dtype=np.float64)
    B = np.tanh(15.0 * (x[..., 1] - 0.5)) - np.tanh(15.0 * (x[..., 1] - 1.5))
    rho = 0.5 + 0.75 * B
    v = np.stack([0.5 * (B - 1.0), 0.1 * np.sin(2.0 * math.pi * x[..., 0])], axis=-1)
    return prim_to_cons(rho, v, np.ones_like(rho), gamma)


def khi_tri(M=16, degree=4, dissipation=1) -> Workload:
    """2 M^2 curved triangles on [0,2]^2, Kelvin-Helmholtz instability."""
    return Workload(f"khi_tri_M{M}_p{degree}", 2, M, 2.0, degree, make_warp_sinprod(2.0, 0.05),
                    kelvin_helmholtz, 0, dissipation)


def tgv_tet_mach(M=4, degree=4, Ma=0.1, dissipation=1) -> Workload:
    """6 M^3 curved tetrahedra on [0,2pi]^3, Taylor-Green flow at Mach Ma."""
    L = 2.0 * math.pi
    return Workload(f"tgv_tet_M{M}_p{degree}_Ma{Ma}", 3, M, L, degree, make_warp_sinprod(L, 0.05),
                    lambda x, gamma=GAMMA: taylor_green(x, Ma, gamma), 0, dissipation)


def named(name: str):
    """The benchmark workload of a given name: vortex_tri_M{M}_p{p},
    tgv_tet_M{M}_p{p}, batched_tets_M{M1-M2-...}_p{lo}-{hi}."""
    import re
    m = re.fullmatch(r"vortex_tri_M(\d+)_p(\d+)", name)
    if m:
        return vortex_tri(M=int(m.group(1)), degree=int(m.group(2)))
    m = re.fullmatch(r"tgv_tet_M(\d+)_p(\d+)", name)
    if m:
        return tgv_tet(M=int(m.group(1)), degree=int(m.group(2)))
    m = re.fullmatch(r"batched_tets_M([\d-]+)_p(\d+)-(\d+)", name)
    if m:
        return batched_tets(Ms=tuple(int(x) for x in m.group(1).split("-")), lo=int(m.group(2)), hi=int(m.group(3)))
    raise KeyError(name)
