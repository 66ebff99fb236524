"""Named synthetic workloads (background grid, order, obstacles, boundary conditions, seeds).

The paper embeds public boundary meshes into a Cartesian background grid; those
meshes are not available, so these seeded analytic obstacles stand in for them
with the shapes the paper highlights (a narrow gap, a thin sheet of relative
thickness 1e-5, self-intersecting unions).  ``N`` may be overridden to get a
reduced-size instance of the same geometry.
"""
from dataclasses import dataclass, field
import numpy as np

from . import shapes


@dataclass
class Workload:
    name: str
    N: int
    k: int
    levels: int
    dirichlet_top: bool
    tol: float
    n_rhs: int
    field_kind: str
    field_seed: int
    description: str
    mesh_fn: object = field(repr=False, default=None)

    @property
    def h(self):
        return 1.0 / self.N

    def mesh(self):
        """Boundary triangle mesh (V, F) of the obstacles at this resolution."""
        return self.mesh_fn(self.N)

    def rhs_seeds(self):
        return [self.field_seed + s for s in range(self.n_rhs)]


# Curved obstacles are tessellated with edges no longer than two background
# cells, which puts one to two triangles in a typical cut cell.
def _c1_mesh(N):
    return shapes.icosphere((0.5, 0.5, 0.5), 0.3, max_edge=2.0 / N)


def _c2_mesh(N):
    s = shapes.icosphere((0.3, 0.5, 0.5), 0.2, max_edge=2.0 / N)
    b = shapes.box((0.7, 0.5, 0.5), (0.3, 0.1, 0.4), shapes.rot_z(30.0))
    return shapes.merge_meshes([s, b])


def _c3_mesh(N):
    return shapes.plate_pair(gap=0.3 / N)


def _c4_mesh(N):
    return shapes.thin_sheet(spacing=2.0 / N)


def ellipsoid_params(seed=0, count=64):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.1, 0.9, (count, 3))
    axes = rng.uniform(0.02, 0.1, (count, 3))
    quats = rng.standard_normal((count, 4))
    quats /= np.linalg.norm(quats, axis=1)[:, None]
    return centres, axes, quats


def _c5_mesh(N, count=64):
    c, a, q = ellipsoid_params(0, count)
    return shapes.merge_meshes([
        shapes.ellipsoid(c[i], a[i], shapes.quat_to_matrix(q[i]), max_edge=2.0 / N)
        for i in range(count)])


CONFIGS = {
    "c1": Workload("c1", 16, 1, 5, True, 1e-10, 1, "normal", 0,
                   "16^3, sphere r=0.3 at the centre, k=1, Dirichlet p=0 on z=1", _c1_mesh),
    "c2": Workload("c2", 64, 1, 5, False, 1e-8, 1, "normal", 0,
                   "64^3, sphere r=0.2 + box 0.3x0.1x0.4 rotated 30 deg about z, k=1", _c2_mesh),
    "c3": Workload("c3", 128, 2, 5, False, 1e-8, 16, "fourier", 0,
                   "128^3, two plates tilted 17 deg about x with a 0.3-cell gap, k=2", _c3_mesh),
    "c4": Workload("c4", 128, 2, 5, False, 1e-8, 1, "fourier", 0,
                   "128^3, curved thin sheet of thickness 1e-5, k=2", _c4_mesh),
    "c5": Workload("c5", 256, 2, 6, False, 1e-8, 1, "fourier", 0,
                   "256^3, union of 64 seeded ellipsoids, k=2", _c5_mesh),
}


def get_config(name, N=None, k=None, levels=None):
    """Return the named workload, optionally at a reduced background resolution."""
    base = CONFIGS[name]
    w = Workload(**{f: getattr(base, f) for f in base.__dataclass_fields__})
    if N is not None:
        w.N = int(N)
        w.name = f"{name}@{N}"
        w.description = w.description.replace(f"{base.N}^3", f"{w.N}^3", 1)
    if k is not None:
        w.k = int(k)
    if levels is not None:
        w.levels = int(levels)
    return w
