"""Seeded scene descriptors for the five benchmark workloads.

Each builder returns a :class:`SceneSpec`: the mesh, material constants,
collider geometry, time-step settings, initial state and the seeded loss
direction.  Everything here is an *input*; nothing computes the method.

Shapes and sizes follow the published workload list (tet meshes of boxes on a
ground plane, Neo-Hookean material, smoothed Fischer-Burmeister contact).  The
values that the list leaves open are fixed here (cell sizes, the push law on
the beam, the slab's sphere path, the batched-scene recipe).
"""

from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

from .mesh import VoxelMesh, box_mesh, quadruped_mesh

GRAVITY = np.array([0.0, 0.0, -9.81])


@dataclasses.dataclass
class SceneSpec:
    name: str
    mesh: VoxelMesh
    density: float
    E: float
    nu: float
    mu: float
    h: float
    eps: float  # smoothing parameter of phi_eps: sqrt(x^2 + y^2 + 2 eps^2)
    steps: int
    gravity: np.ndarray
    planes: np.ndarray  # (n_planes, 4): unit normal n and offset d, gap = n.x - d
    contact_margin: float
    q0: np.ndarray  # (n_verts, 3)
    v0: np.ndarray  # (n_verts, 3)
    loss_dir: np.ndarray  # (n_verts, 3): loss = sum(loss_dir * q_T)
    seed: int
    # sphere colliders: list of (radius, centre(t) callable returning (3,) array)
    spheres: list = dataclasses.field(default_factory=list)
    # external force on vertices at step t (without gravity), (n_verts, 3)
    f_ext: Optional[Callable[[int], np.ndarray]] = None
    # material model of the local projection: "nh", "arap" or "corot"
    material: str = "nh"

    @property
    def n_verts(self) -> int:
        return self.mesh.n_verts

    @property
    def n_tets(self) -> int:
        return self.mesh.n_tets

    def force(self, t: int) -> np.ndarray:
        if self.f_ext is None:
            return np.zeros((self.n_verts, 3))
        return self.f_ext(t)

    def sphere_array(self, t: int) -> np.ndarray:
        """(n_spheres, 4) rows (cx, cy, cz, r) at time index t."""
        if not self.spheres:
            return np.zeros((0, 4))
        return np.array([[*np.asarray(c(t), dtype=np.float64), r] for r, c in self.spheres])


def loss_vector(rng: np.random.Generator, n_verts: int) -> np.ndarray:
    return rng.standard_normal((n_verts, 3))


GROUND = np.array([[0.0, 0.0, 1.0, 0.0]])


def tiny_scene(variant: str = "impact", seed: int = 0) -> SceneSpec:
    """4x4x4 cells (384 tets, 125 verts), side 0.1 m, 5 mm above the ground.

    ``literal``: dropped at rest (free fall of 20 steps never reaches the
    ground).  ``impact``: same, plus a downward initial speed of 0.5 m/s so
    that the cube lands after about 9 ms and slides.
    """
    rng = np.random.default_rng(seed)
    mesh = box_mesh(4, 4, 4, 0.025, origin=(0.0, 0.0, 0.005))
    v0 = np.zeros((mesh.n_verts, 3))
    v0[:, :2] = rng.uniform(-0.1, 0.1, size=(mesh.n_verts, 2))
    if variant == "impact":
        v0[:, 2] = -0.5
    elif variant != "literal":
        raise ValueError(variant)
    loss = loss_vector(rng, mesh.n_verts)
    return SceneSpec(
        name=f"tiny-{variant}", mesh=mesh, density=1000.0, E=1e5, nu=0.4, mu=0.5,
        h=1e-3, eps=1e-6, steps=20, gravity=GRAVITY.copy(), planes=GROUND.copy(),
        contact_margin=2e-3, q0=mesh.rest.copy(), v0=v0, loss_dir=loss, seed=seed,
    )


def beam_push_force(mesh: VoxelMesh, rng: np.random.Generator, steps: int, total: float = 50.0):
    """Tangential push on the top face: magnitude ramps 0 -> ``total`` newtons
    linearly over the run, one seeded horizontal direction, spread over the
    top-face vertices with seeded U[0,1] weights normalised to sum 1."""
    top = np.nonzero(mesh.grid_index[:, 2] == mesh.grid_index[:, 2].max())[0]
    w = rng.uniform(0.0, 1.0, size=top.shape[0])
    w = w / w.sum()
    ang = rng.uniform(0.0, 2.0 * np.pi)
    direction = np.array([np.cos(ang), np.sin(ang), 0.0])

    def f(t: int) -> np.ndarray:
        out = np.zeros((mesh.n_verts, 3))
        mag = total * (t + 1) / steps
        out[top] = (mag * w)[:, None] * direction[None, :]
        return out

    return f


def beam_scene(mu: float = 0.4, seed: int = 1, steps: int = 100,
               nx: int = 32, ny: int = 8, nz: int = 8) -> SceneSpec:
    """32x8x8-cell beam (12,288 tets, 2,673 verts), cell 0.0175 m, resting on
    the ground, pushed sideways on its top face (0 -> 50 N)."""
    rng = np.random.default_rng(seed)
    mesh = box_mesh(nx, ny, nz, 0.0175, origin=(0.0, 0.0, 0.0))
    push = beam_push_force(mesh, rng, steps)
    loss = loss_vector(rng, mesh.n_verts)
    return SceneSpec(
        name=f"beam-mu{mu}", mesh=mesh, density=1000.0, E=1e6, nu=0.45, mu=mu,
        h=1e-3, eps=np.sqrt(0.5e-12), steps=steps, gravity=GRAVITY.copy(),
        planes=GROUND.copy(), contact_margin=2e-3, q0=mesh.rest.copy(),
        v0=np.zeros((mesh.n_verts, 3)), loss_dir=loss, seed=seed, f_ext=push,
    )


def slab_scene(seed: int = 2, steps: int = 50, nx: int = 64, ny: int = 32, nz: int = 32,
               cell: float = 0.01) -> SceneSpec:
    """64x32x32-cell slab (393,216 tets, 70,785 verts), cell 0.01 m, pressed
    into the ground by a kinematic sphere of radius 0.3 x the slab width
    descending at constant speed to an indentation of 0.093 m x (width /
    0.64 m) at the last step.  Smaller nx, ny, nz give the same set-up at a
    reduced size."""
    rng = np.random.default_rng(seed)
    mesh = box_mesh(nx, ny, nz, cell, origin=(0.0, 0.0, 0.0))
    width = nx * cell
    R = 0.3 * width
    top = nz * cell
    depth = 0.093 * width / 0.64
    cx, cy = 0.5 * nx * cell, 0.5 * ny * cell

    def centre(t: int) -> np.ndarray:
        return np.array([cx, cy, top + R - depth * t / steps])

    loss = loss_vector(rng, mesh.n_verts)
    return SceneSpec(
        name="slab" if (nx, ny, nz) == (64, 32, 32) else f"slab{nx}x{ny}x{nz}", mesh=mesh, density=1000.0,
        E=5e5, nu=0.45, mu=0.5, h=1e-3, eps=np.sqrt(0.5e-12), steps=steps, gravity=GRAVITY.copy(),
        planes=GROUND.copy(), contact_margin=2e-3, q0=mesh.rest.copy(), v0=np.zeros((mesh.n_verts, 3)),
        loss_dir=loss, seed=seed, spheres=[(R, centre)],
    )


def quadruped_scene(seed: int = 4, steps: int = 1000) -> SceneSpec:
    """Torso 32x16x8 cells on four 4x4x16-cell legs (30,720 tets), cell
    0.01 m, standing on the ground, mu = 0.8."""
    rng = np.random.default_rng(seed)
    mesh = quadruped_mesh(0.01, origin=(0.0, 0.0, 0.0))
    loss = np.zeros((mesh.n_verts, 3))
    loss[:, 0] = -1.0 / mesh.n_verts  # placeholder direction; the rollout loss is the COM shift
    return SceneSpec(
        name="quadruped", mesh=mesh, density=1000.0, E=1e5, nu=0.4, mu=0.8, h=1e-3,
        eps=np.sqrt(0.5e-12), steps=steps, gravity=GRAVITY.copy(), planes=GROUND.copy(),
        contact_margin=2e-3, q0=mesh.rest.copy(), v0=np.zeros((mesh.n_verts, 3)),
        loss_dir=loss, seed=seed,
    )


def batched_scenes(n_scenes: int = 256, seed: int = 3, tmax: float = 1e5):
    """Boxes with log-uniform tet counts in [2e3, tmax] (1e5 for the full
    workload), seeded aspect, E, nu, mu and tangential initial velocity; one
    in eight hovers 5 mm up."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scenes):
        T = np.exp(rng.uniform(np.log(2e3), np.log(tmax)))
        while True:
            a = rng.uniform(0.5, 2.0, size=3)
            cells = T / 6.0
            base = (cells / np.prod(a)) ** (1.0 / 3.0)
            nxyz = np.maximum(1, np.round(base * a).astype(int))
            if (nxyz[0] + 1) * (nxyz[1] + 1) <= 2000:
                break
        hover = (s % 8) == 7
        mesh = box_mesh(*map(int, nxyz), 0.01, origin=(0.0, 0.0, 0.005 if hover else 0.0))
        v0 = np.zeros((mesh.n_verts, 3))
        v0[:, :2] = rng.uniform(-0.1, 0.1, size=(mesh.n_verts, 2))
        E = float(np.exp(rng.uniform(np.log(1e4), np.log(1e7))))
        nu = float(rng.uniform(0.3, 0.48))
        mu = float(rng.uniform(0.1, 1.0))
        out.append(SceneSpec(
            name=f"batch{s}", mesh=mesh, density=1000.0, E=E, nu=nu, mu=mu, h=1e-3,
            eps=np.sqrt(0.5e-12), steps=10, gravity=GRAVITY.copy(), planes=GROUND.copy(),
            contact_margin=2e-3, q0=mesh.rest.copy(), v0=v0,
            loss_dir=loss_vector(rng, mesh.n_verts), seed=seed * 1000 + s,
        ))
    return out


SLOPE_DEG = 10.0
# the two friction coefficients straddle the slip threshold tan(slope) by
# +-4e-4 (a 1e-3-scale friction difference)
SLOPE_DMU = 4e-4


def slope_scene(side: str = "slip", two_eps2: float = 1e-12, seed: int = 5, h: float = 1e-2,
                duration: float = 30.0, E: float = 1e7) -> SceneSpec:
    """Stiff rubber-like cube (4x4x4 cells, 384 tets, side 0.1 m) resting on
    a 10-degree slope, for the smoothing sweep.  The slope is expressed by
    tilting gravity about the y axis (ground z = 0, down-slope direction +x),
    which is the same physics as a tilted plane under vertical gravity.
    ``side``: "slip" (mu = tan(slope) - 4e-4) or "stick" (mu = tan(slope) +
    4e-4).  ``two_eps2`` is the smoothing 2 eps^2."""
    if side not in ("slip", "stick"):
        raise ValueError(side)
    rng = np.random.default_rng(seed)
    th = np.deg2rad(SLOPE_DEG)
    mu = float(np.tan(th)) + (SLOPE_DMU if side == "stick" else -SLOPE_DMU)
    mesh = box_mesh(4, 4, 4, 0.025, origin=(0.0, 0.0, 0.0))
    g = 9.81 * np.array([np.sin(th), 0.0, -np.cos(th)])
    steps = int(round(duration / h))
    return SceneSpec(
        name=f"slope-{side}-{two_eps2:g}", mesh=mesh, density=1100.0, E=E, nu=0.45, mu=mu, h=h,
        eps=float(np.sqrt(0.5 * two_eps2)), steps=steps, gravity=g, planes=GROUND.copy(),
        contact_margin=2e-3, q0=mesh.rest.copy(), v0=np.zeros((mesh.n_verts, 3)),
        loss_dir=loss_vector(rng, mesh.n_verts), seed=seed,
    )


def perturbed_state(spec: SceneSpec, seed: int = 12, scale: float = 1e-5) -> np.ndarray:
    """Rest positions with a seeded N(0, scale^2) perturbation per coordinate
    (a deformed state at which an adjoint system can be set up)."""
    rng = np.random.default_rng(seed)
    return spec.mesh.rest + scale * rng.standard_normal(spec.mesh.rest.shape)


def slab_indented_state(spec: SceneSpec, t: int) -> np.ndarray:
    """The slab with its top face pressed onto the sphere's surface at the
    sphere's pose of step t: every vertex moves straight down by
    delta(x, y) z / H, where H is the slab height and delta the depth of the
    sphere's lower surface below the undeformed top face at (x, y) (zero
    outside the sphere's footprint).  Top-face vertices under the sphere lie
    on its surface, the bottom face stays on the ground, and every tet keeps
    det F = 1 - delta / H > 0 (a vertical displacement linear in z)."""
    R, centre = spec.spheres[0]
    c = np.asarray(centre(t), dtype=np.float64)
    q = spec.mesh.rest.copy()
    H = float(q[:, 2].max())
    r2 = (q[:, 0] - c[0]) ** 2 + (q[:, 1] - c[1]) ** 2
    inside = r2 < R * R
    zs = np.full(q.shape[0], np.inf)
    zs[inside] = c[2] - np.sqrt(R * R - r2[inside])
    depth = np.maximum(0.0, H - zs)
    q[:, 2] -= depth * q[:, 2] / H
    return q


def slab_last_step(spec: SceneSpec):
    """Inputs of the slab workload's measured step, its last one (the most
    contacts): positions at the start (qbar) and end (q) of the step with the
    top face on the sphere (slab_indented_state at the sphere's poses of
    steps T - 1 and T), and the seeded adjoint right-hand side g_q = the loss
    direction, g_v = 1e-3 N(0, 1).  Returns (qbar, q, g_q, g_v)."""
    T = spec.steps
    qbar = slab_indented_state(spec, T - 1)
    q = slab_indented_state(spec, T)
    gv = 1e-3 * np.random.default_rng(77).standard_normal(q.shape)
    return qbar, q, spec.loss_dir.copy(), gv


def contact_values(n: int, mu: float, seed: int = 13):
    """Seeded contact displacements and multipliers in frame coordinates for n
    sticking contacts: normal gaps U[1e-13, 1e-11] m, normal forces
    U[0.01, 1] N, tangential displacements of magnitude U[1e-13, 1e-11] m and
    tangential forces of magnitude U[0, 0.9] mu lambda_n pointing against
    them.  Returns (delta, lam), each (n, 3)."""
    rng = np.random.default_rng(seed)
    delta = np.zeros((n, 3))
    lam = np.zeros((n, 3))
    delta[:, 0] = rng.uniform(1e-13, 1e-11, n)
    lam[:, 0] = rng.uniform(0.01, 1.0, n)
    ang = rng.uniform(0.0, 2.0 * np.pi, n)
    dmag = rng.uniform(1e-13, 1e-11, n)
    fmag = rng.uniform(0.0, 0.9, n) * mu * lam[:, 0]
    delta[:, 1], delta[:, 2] = dmag * np.cos(ang), dmag * np.sin(ang)
    lam[:, 1], lam[:, 2] = -fmag * np.cos(ang), -fmag * np.sin(ang)
    return delta, lam


def actuation_groups(mesh: VoxelMesh, n_groups: int = 64, seed: int = 6):
    """Per-tet actuation group and fibre direction for an actuated mesh (the
    quadruped's 64 muscle groups): the tets are split by centroid x into 8
    slices of equal count, each slice by centroid z into 8 groups of equal
    count, and every group gets one seeded unit fibre direction.  Returns
    (group int32 [n_tets] in 0..n_groups-1, fibre [n_tets, 3])."""
    if n_groups != 64 or mesh.n_tets < 64:
        raise ValueError("the grouping is 8 x 8 equal-count bins")
    rng = np.random.default_rng(seed)
    c = mesh.rest[mesh.tets].mean(axis=1)
    group = np.zeros(mesh.n_tets, dtype=np.int32)
    for ix, sl in enumerate(np.array_split(np.lexsort((c[:, 2], c[:, 0])), 8)):
        for iz, part in enumerate(np.array_split(sl[np.lexsort((c[sl, 0], c[sl, 2]))], 8)):
            group[part] = 8 * ix + iz
    d = rng.standard_normal((n_groups, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return group, d[group]


def actuation_params(steps: int, n_groups: int = 64, h: float = 1e-3, amplitude: float = 1e4, seed: int = 7):
    """Seeded sinusoidal actuation parameters a[t, k] = A_k sin(2 pi f_k t h +
    phi_k) (active stress magnitudes, Pa), A_k ~ U[0.5, 1] amplitude, f_k ~
    U[1, 4] Hz, phi_k ~ U[0, 2 pi].  Returns (steps, n_groups)."""
    rng = np.random.default_rng(seed)
    A = amplitude * rng.uniform(0.5, 1.0, n_groups)
    f = rng.uniform(1.0, 4.0, n_groups)
    ph = rng.uniform(0.0, 2.0 * np.pi, n_groups)
    t = np.arange(steps)[:, None] * h
    return A[None, :] * np.sin(2.0 * np.pi * f[None, :] * t + ph[None, :])
