"""Storage branches and error paths of the library on the GPU.

* Column storage: the same problem with 16-bit column codes (the default)
  and with int32 columns everywhere applies the same K and V-cycle and
  solves to the same pressure; the slice statistics show that coded, plain,
  value-template and stored-value slices all took part.
* NOT_SPD: a description whose element stiffness blocks are negated makes
  the coarsest factorisation meet negative pivots.
* BUSY: a second call on a handle while a solve runs on it is refused.
"""
import threading
import time

import numpy as np
import pytest

from conftest import oracle_problem
from oracle_desc import describe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("name", ["c3", "c1"])
def test_plain_and_coded_columns_agree(name):
    import synth
    from paper_2607_17725_amd import fvem
    pb = oracle_problem(name, 8)
    desc = describe(pb)
    print(f"[gpu paths] {name}: coded vs plain columns", flush=True)
    coded = fvem.Hierarchy(desc, lattice_min_fraction=1e-6)
    plain = fvem.Hierarchy(desc, lattice_min_fraction=1e-6, column_codes=-1)
    sc = [coded.level_slices(l) for l in range(coded.n_levels)]
    sp_ = [plain.level_slices(l) for l in range(plain.n_levels)]
    print(f"[gpu paths] slices coded {sc}\n[gpu paths] slices plain {sp_}", flush=True)
    assert sum(s["plain"] for s in sp_) > 0 and sum(s["coded"] for s in sp_) == 0
    assert sum(s["coded"] for s in sc) > 0
    assert sum(s["stored"] for s in sc) > 0
    if name == "c3":   # at 8^3 only the plates repeat rows often enough for value templates
        assert sum(s["templated"] for s in sc) > 0
    assert plain.level_bytes(1) > coded.level_bytes(1)
    x = np.random.default_rng(2).standard_normal(coded.n_dof)
    for op, tol in ((fvem.OP_K, 1e-15), (fvem.OP_VCYCLE32, 1e-6)):
        a = coded.apply(op, _dev(x)).cpu().numpy()
        b = plain.apply(op, _dev(x)).cpu().numpy()
        # identical storage order and arithmetic: only the column encoding differs
        assert np.linalg.norm(a - b) <= tol * np.linalg.norm(a)
    u = (synth.normal_field(pb.vertices, 0) if name == "c1" else synth.fourier_field(pb.vertices, 0)).ravel()
    ref = pb.solve_direct(u)
    for h in (coded, plain):
        p, _ = h.solve(_dev(u), tol=1e-10, precision=fvem.PREC_MIXED)
        assert np.linalg.norm(p.cpu().numpy() - ref) <= 1e-6 * np.linalg.norm(ref)


def test_not_spd_is_reported():
    from paper_2607_17725_amd import fvem
    desc = describe(oracle_problem("c3", 8))
    desc["ke_val"] = -desc["ke_val"]
    with pytest.raises(fvem.FvemError) as e:
        fvem.Hierarchy(desc)
    assert e.value.code == 4, str(e.value)   # FVEM_ERR_NOT_SPD


def test_busy_handle_is_refused():
    from paper_2607_17725_amd import fvem
    pb = oracle_problem("c3", 8)
    h = fvem.Hierarchy(describe(pb))
    u = _dev(np.random.default_rng(3).standard_normal(3 * pb.n_vertices))
    p = torch.empty(h.n_dof, dtype=torch.float64, device="cuda")
    done = {}

    def long_solve():
        # an unreachable tolerance keeps the handle busy for maxit iterations
        _, st = h.solve(u, out=p, tol=1e-300, maxit=3000, raise_not_converged=False)
        done["it"] = st["iterations"]

    t = threading.Thread(target=long_solve)
    t.start()
    time.sleep(0.5)
    busy = None
    try:
        h.apply(fvem.OP_K, p)
    except fvem.FvemError as e:
        busy = e.code
    t.join()
    assert done.get("it") == 3000
    assert busy == 7     # FVEM_ERR_BUSY
    h.apply(fvem.OP_K, p)   # free again afterwards
