"""Velocity correction, loss and chained projections on the GPU, through the C ABI.

Against the oracle on identical inputs (its grid and element blocks):
* the cell-field operators Pi_1, grad Pi_k, mass and vertex average, their
  transposes and the accumulate mode, to 1e-12 relative;
* the projected velocity s = Pi_1 u - grad Pi_k p and its transpose, FP64
  and mixed, to 1e-7 relative after solving to 1e-10 (the pressure error
  is the conditioning times the tolerance; the thin sheet's FP64 residual
  floor sits near 1e-12);
* loss and gradient of the thin-sheet workload (its oracle-sized grid)
  through torch.autograd against the oracle's exact reverse mode (bar:
  1e-5 relative) and against central finite differences along seeded
  directions;
* a 3-step chain with checkpoints stored in FP64 and FP32 against the
  oracle's exact chain gradient.
On the native builder's 16^3 ellipsoid scene (the 64-ellipsoid workload at
a size the GPU finishes in seconds): the chained gradient against central
finite differences along two directions, and the FP32-storage gradient
against the FP64-storage one.
"""
import numpy as np
import pytest

from oracle_desc import describe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_H = {}


def hier_for(request, name):
    from paper_2607_17725_amd import fvem
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    if name not in _H:
        pb = request.getfixturevalue(name)
        print(f"[gpu velocity] building hierarchy for {name}", flush=True)
        _H[name] = (fvem.Hierarchy(describe(pb), lattice_min_fraction=1e-6), pb)
    return _H[name]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name", ["c1_small", "c3_small", "c4_small"])
def test_velocity_operators_match_oracle(name, request):
    from paper_2607_17725_amd import fvem
    from oracle import velocity as vel
    h, pb = hier_for(request, name)
    o = vel.operators(pb)
    rng = np.random.default_rng(21)
    nc, nv3, n = 12 * h.n_cells, 3 * h.n_vert, h.n_dof
    assert nc == o["Pi"].shape[0]
    cases = [(fvem.OP_PI1, o["Pi"], nv3), (fvem.OP_PI1T, o["Pi"].T, nc), (fvem.OP_G, o["G"], n),
             (fvem.OP_GT, o["G"].T, nc), (fvem.OP_MASS, o["M"], nc), (fvem.OP_AV, o["Av"], nc),
             (fvem.OP_AVT, o["Av"].T, nv3)]
    for op, A, nin in cases:
        x = rng.standard_normal(nin)
        y = _host(h.apply(op, _dev(x)))
        ref = A @ x
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max(), f"op {op}"
    # accumulate: y += Av x
    x = rng.standard_normal(nc)
    y0 = rng.standard_normal(nv3)
    y = _dev(y0)
    h.apply(fvem.OP_AV, _dev(x), out=y, accumulate=True)
    ref = y0 + o["Av"] @ x
    assert np.abs(_host(y) - ref).max() <= 1e-12 * np.abs(ref).max()
    with pytest.raises(fvem.FvemError):
        h.apply(fvem.OP_GT, _dev(x), out=torch.zeros(n, dtype=torch.float64, device="cuda"), accumulate=True)


@pytest.mark.parametrize("name", ["c3_small", "c4_small"])
@pytest.mark.parametrize("precision", [0, 1])
def test_project_velocity_matches_oracle(name, precision, request):
    import synth
    from oracle import velocity as vel
    h, pb = hier_for(request, name)
    u = synth.fourier_field(pb.vertices, 3).ravel()
    s_ref, p_ref = vel.project(pb, u)
    p = torch.empty(h.n_dof, dtype=torch.float64, device="cuda")
    s, st = h.project_velocity(_dev(u), p=p, tol=1e-10, precision=precision, maxit=1000)
    gs = np.random.default_rng(8).standard_normal(12 * h.n_cells)
    gu, _ = h.project_velocity_adjoint(_dev(gs), tol=1e-10, precision=precision, maxit=1000)
    gu_ref = vel.project_vjp(pb, gs)
    print(f"[gpu velocity] {name} precision={precision} iters={st['iterations']} "
          f"s err={_rel(_host(s), s_ref):.2e} p err={_rel(_host(p), p_ref):.2e} "
          f"adjoint err={_rel(_host(gu), gu_ref):.2e}")
    assert _rel(_host(s), s_ref) <= 1e-7
    assert _rel(_host(p), p_ref) <= 1e-7
    assert _rel(_host(gu), gu_ref) <= 1e-7


def _loss_grad_gpu(h, u, t, precision, tol):
    from paper_2607_17725_amd import fvem
    Vel, Loss = fvem.velocity_function(), fvem.loss_function()
    ut = _dev(u).requires_grad_(True)
    L = Loss.apply(Vel.apply(ut, h, tol, precision), _dev(t), h)
    L.backward()
    return float(L), _host(ut.grad)


def test_sheet_loss_gradient(request):
    """The thin-sheet workload's loss gradient: oracle exact gradient and finite differences."""
    import synth
    from oracle import velocity as vel
    h, pb = hier_for(request, "c4_small")
    o = vel.operators(pb)
    u = synth.fourier_field(pb.vertices, 0).ravel()
    t = o["Pi"] @ synth.fourier_field(pb.vertices, 1).ravel()
    L_ref, g_ref = vel.loss_and_gradient(pb, u, t)
    for precision in (0, 1):
        L, g = _loss_grad_gpu(h, u, t, precision, 1e-10)
        print(f"[gpu velocity] sheet loss precision={precision}: L rel err {abs(L - L_ref) / L_ref:.2e}, "
              f"grad rel err {_rel(g, g_ref):.2e}")
        assert abs(L - L_ref) <= 1e-8 * L_ref
        assert _rel(g, g_ref) <= 1e-5
    # central differences along seeded directions, mixed forward solves
    for seed in (100, 101, 102, 103):
        d = synth.normal_field(pb.vertices, seed).ravel()
        eps = 1e-2 * np.linalg.norm(u) / np.linalg.norm(d)
        Lp, _ = _loss_grad_gpu(h, u + eps * d, t, 1, 1e-10)
        Lm, _ = _loss_grad_gpu(h, u - eps * d, t, 1, 1e-10)
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), 1e-3 * L_ref), f"direction {seed}"


def test_chain_gradient_matches_oracle(request):
    import synth
    from paper_2607_17725_amd import fvem
    from oracle import velocity as vel
    h, pb = hier_for(request, "c3_small")
    o = vel.operators(pb)
    K = 3
    u0 = synth.fourier_field(pb.vertices, 0).ravel()
    rng = np.random.default_rng(1000)
    eps = [0.1 * rng.standard_normal(u0.shape) for _ in range(K - 1)]
    targets = [o["Pi"] @ synth.fourier_field(pb.vertices, 2000 + k).ravel() for k in range(K)]
    L_ref, g_ref = vel.chain(pb, u0, eps, targets)
    grads = {}
    for dt in (torch.float64, torch.float32):
        L, g, info = fvem.chain_loss_and_grad(h, _dev(u0), [_dev(e) for e in eps], [_dev(t) for t in targets],
                                             store_dtype=dt, tol=1e-12, precision=1)
        grads[dt] = _host(g)
        print(f"[gpu velocity] chain store={dt}: L rel err {abs(L - L_ref) / L_ref:.2e}, "
              f"grad rel err {_rel(grads[dt], g_ref):.2e}, checkpoints {info['checkpoint_bytes']} B")
    assert _rel(grads[torch.float64], g_ref) <= 1e-8
    # FP32 checkpoints perturb the recomputed fields by ~1e-7 relative
    assert _rel(grads[torch.float32], g_ref) <= 1e-5


def test_ellipsoid_chain_finite_differences():
    """64-ellipsoid scene at 16^3 on the native builder: chain gradient vs finite differences."""
    import synth
    from paper_2607_17725_amd import fvem
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    w = synth.get_config("c5", N=16)
    V, F = w.mesh()
    print(f"[gpu velocity] building the ellipsoid scene at N=16", flush=True)
    g = fvem.Grid(V, F, w.N, w.k, w.levels, w.dirichlet_top)
    h = fvem.Hierarchy(g)
    K = 4
    X = g.vertices
    u0 = _dev(synth.fourier_field(X, 0).ravel())
    eps = [_dev(0.1 * synth.normal_field(X, 1000 + k).ravel()) for k in range(K - 1)]
    targets = [h.apply(fvem.OP_PI1, _dev(synth.fourier_field(X, 2000 + k).ravel())) for k in range(K)]
    out = {}
    for dt in (torch.float64, torch.float32):
        out[dt] = fvem.chain_loss_and_grad(h, u0, eps, targets, store_dtype=dt, tol=1e-11, precision=1)
    L, g64, _ = out[torch.float64]
    g32 = out[torch.float32][1]
    diff = float(torch.linalg.norm(g32 - g64) / torch.linalg.norm(g64))
    print(f"[gpu velocity] ellipsoid chain: L={L:.6e}, |g32-g64|/|g64| = {diff:.2e}")
    assert diff <= 1e-5
    for seed in (100, 101):
        d = _dev(synth.normal_field(X, seed).ravel())
        step = 1e-2 * float(torch.linalg.norm(u0) / torch.linalg.norm(d))
        Lp = fvem.chain_loss_and_grad(h, u0 + step * d, eps, targets, tol=1e-11, precision=1, with_grad=False)[0]
        Lm = fvem.chain_loss_and_grad(h, u0 - step * d, eps, targets, tol=1e-11, precision=1, with_grad=False)[0]
        fd = (Lp - Lm) / (2 * step)
        gd = float(torch.dot(g64, d))
        assert abs(fd - gd) <= 1e-6 * max(abs(fd), 1e-3 * L), f"direction {seed}: {fd} vs {gd}"
