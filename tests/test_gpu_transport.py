"""The simulation-step transfers on the GPU against the oracle (Algorithm 1).

The library runs on the native builder's grid; the oracle on its own grid of
the same scene.  Cells are matched by centroid and vertices by position.
Checked: point location of seeded points, P2G at every vertex, and one whole
step (P2G, buoyancy, projection, G2P, advection) of eight particles per cell:
ghost flags, substep count, particle velocities and positions.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from conftest import oracle_problem
from oracle import transport as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [("c1", 8), ("c3", 8)]
_CACHE = {}


def _setup(name, N):
    if (name, N) in _CACHE:
        return _CACHE[(name, N)]
    import synth
    from paper_2607_17725_amd import fvem
    print(f"[gpu transport] building {name}@{N}", flush=True)
    w = synth.get_config(name, N=N)
    V, F = w.mesh()
    g = fvem.Grid(V, F, w.N, w.k, w.levels, w.dirichlet_top)
    h = fvem.Hierarchy(g)
    tr = fvem.Transport(g)
    pb = oracle_problem(name, N)
    loc = T.Locator(pb)
    cen = g.describe()["cell_geom"].reshape(-1, 5)[:, :3]
    d, cell_map = cKDTree(pb.meshes[0].cell_centroid).query(cen)
    assert d.max() < 1e-9
    d, vert_map = cKDTree(pb.vertices).query(g.vertices)
    assert d.max() < 1e-12
    _CACHE[(name, N)] = (w, g, h, tr, pb, loc, cell_map, vert_map)
    return _CACHE[(name, N)]


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("name,N", CASES)
def test_locate_matches_oracle(name, N):
    w, g, h, tr, pb, loc, cell_map, vert_map = _setup(name, N)
    rng = np.random.default_rng(5)
    pts = np.concatenate([rng.uniform(-0.05, 1.05, size=(3000, 3)), pb.meshes[0].cell_centroid])
    got = tr.locate(_dev(pts)).cpu().numpy()
    want = np.array([loc.cell_of(x) for x in pts])
    mapped = np.where(got >= 0, cell_map[np.maximum(got, 0)], -1)
    assert np.array_equal(mapped, want)
    print(f"[gpu transport] {name}@{N}: {np.count_nonzero(want >= 0)} of {len(pts)} points in the fluid", flush=True)


@pytest.mark.parametrize("name,N", CASES)
def test_p2g_matches_oracle(name, N):
    import synth
    w, g, h, tr, pb, loc, cell_map, vert_map = _setup(name, N)
    x, u, rho, temp = synth.seeded_particles(N, seed=1)
    f = np.column_stack([u, rho, temp])
    got = tr.p2g(_dev(x), _dev(f)).cpu().numpy()
    want = T.p2g(pb.vertices, x, f, 1.0 / N)[vert_map]
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # bitwise reproducible
    again = tr.p2g(_dev(x), _dev(f)).cpu().numpy()
    assert np.array_equal(got, again)


@pytest.mark.parametrize("name,N", CASES)
def test_smoke_step_matches_oracle(name, N):
    import synth
    from paper_2607_17725_amd import fvem
    w, g, h, tr, pb, loc, cell_map, vert_map = _setup(name, N)
    x, u, rho, temp = synth.seeded_particles(N, seed=2)
    ghost_o = np.array([loc.cell_of(p) < 0 for p in x])
    xd, ud = _dev(x), _dev(u)
    ghost = (tr.locate(xd) < 0).to(torch.uint8)
    assert np.array_equal(ghost.cpu().numpy().astype(bool), ghost_o)
    # ghosts carry zero velocity and no smoke
    u[ghost_o] = 0.0
    rho[ghost_o] = 0.0
    temp[ghost_o] = 0.0
    ud = _dev(u)
    dt, a_flip, alpha, beta = 0.25, 0.9, 0.5, 2.0   # two CFL substeps
    info = fvem.smoke_step(h, tr, xd, ud, _dev(rho), _dev(temp), ghost, dt, a_flip=a_flip, alpha=alpha, beta=beta,
                           tol=1e-12, precision=fvem.PREC_FP64)
    x2, u2, oi = T.step(pb, loc, x, u, rho, temp, ghost_o, dt, a_flip, alpha, beta)
    assert info["substeps"] == oi["substeps"]
    umax = np.abs(u2).max()
    du = np.abs(ud.cpu().numpy() - u2).max()
    dx = np.abs(xd.cpu().numpy() - x2).max()
    print(f"[gpu transport] {name}@{N}: substeps {info['substeps']}, max |du| {du:.2e} (|u| {umax:.2e}), "
          f"max |dx| {dx:.2e}", flush=True)
    assert du <= 1e-8 * umax
    assert dx <= 1e-10
    # non-ghost particles end in the fluid
    cells = tr.locate(xd).cpu().numpy()
    assert np.all(cells[~ghost_o] >= 0)
