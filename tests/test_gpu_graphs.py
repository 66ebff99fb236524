"""V-cycles replayed as HIP graphs against the same V-cycles launched kernel by kernel.

Two hierarchies are built from one native-grid description: one replays its
V-cycles as graphs (the default), one launches them eagerly.  Every replay,
interleaved with other eager work and host synchronisations, must equal the
eager result bitwise (the kernels are deterministic), in both precisions and
in both buffer states; so must whole solves, profiled or not.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pair():
    import synth
    from paper_2607_17725_amd import fvem
    w = synth.get_config("c3", N=16)
    V, F = w.mesh()
    print("[gpu graphs] building c3@16", flush=True)
    g = fvem.Grid(V, F, w.N, w.k, w.levels, w.dirichlet_top)
    desc = g.describe()
    return w, g, fvem.Hierarchy(desc), fvem.Hierarchy(desc, vcycle_graphs=-1)


def test_vcycle_replays_match_eager(pair):
    from paper_2607_17725_amd import fvem
    w, g, hg, he = pair
    rng = np.random.default_rng(21)
    for rep in range(6):
        r = torch.as_tensor(rng.standard_normal(hg.n_dof), device="cuda")
        r = hg.apply(fvem.OP_PROJECT, r)
        for op in (fvem.OP_VCYCLE32, fvem.OP_VCYCLE):
            zg = hg.apply(op, r).cpu().numpy()
            # eager work and a host synchronisation between the replays
            _ = hg.apply(fvem.OP_K, r)
            torch.cuda.synchronize()
            ze = he.apply(op, r).cpu().numpy()
            assert np.array_equal(zg, ze), f"replay {rep}, op {op}"
    print("[gpu graphs] 12 replays equal to the eager V-cycles", flush=True)


def test_solves_match_eager(pair):
    import synth
    from paper_2607_17725_amd import fvem
    w, g, hg, he = pair
    for seed in (0, 1):
        u = torch.as_tensor(synth.fourier_field(g.vertices, seed).ravel(), device="cuda")
        for prec in (fvem.PREC_MIXED, fvem.PREC_FP64):
            pe, se = he.solve(u, tol=1e-10, precision=prec)
            for profile in (0, 2, 1):
                pg, sg = hg.solve(u, tol=1e-10, precision=prec, profile=profile)
                assert sg["iterations"] == se["iterations"]
                assert torch.equal(pg, pe), f"seed {seed}, precision {prec}, profile {profile}"
                if profile:
                    assert sg["n_vcycle"] >= sg["iterations"] and sg["ms_vcycle"] > 0
    print("[gpu graphs] solves equal with and without graphs", flush=True)
