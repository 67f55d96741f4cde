"""CPU-side checks of the C ABI library: it loads without a GPU, exports every
function include/dg.h declares, its host generators agree with the oracle's
independent ones, and argument errors are reported synchronously."""
import ctypes
import os
import re

import numpy as np
import pytest

import dgtest
from oracle import elements as oel
from oracle import refmat
from workload import cube_mesh, random_materials, seed_for

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd import _lib as L
    if not os.path.exists(dg.library_path()):
        pytest.fail("HIP library not built: run python -c 'import __graft_entry__ as g; g.build()'")
    return L._load()


def test_exports_every_declared_symbol():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "dg.h")).read()
    names = set(re.findall(r"^\s*(?:int|int64_t|const char \*)\s*\*?\s*(dg_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 16
    for n in sorted(names):
        assert hasattr(lib, n), n


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_reference_matrices_match_oracle(N):
    import paper_1903_11521_amd as dg
    _lib()
    M = dg.reference_matrices(N)
    rm = refmat.refmats(N)
    for key, ref in (("Khat", rm.Khat), ("Ktilde", rm.Ktilde), ("R", rm.R), ("Rhat", rm.Rhat), ("f", rm.f),
                     ("mass", rm.mass), ("face_mass", rm.face_mass)):
        a = M[key]
        assert np.array_equal(a != 0, ref != 0), key
        assert np.max(np.abs(a - ref)) <= 2e-14 * np.max(np.abs(ref)), key


def test_element_data_matches_oracle():
    import paper_1903_11521_amd as dg
    _lib()
    mesh = cube_mesh(4, seed_for(0), relabel=True)
    mats = random_materials(mesh.E, seed_for(0))
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
    for a, b in ((star, ostar), (Ap, oAp), (Am, oAm)):
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    # boundary faces: no neighbour -> zero A-, A+ from the element's own material
    nb = mesh.neigh.copy()
    nb[0, 2] = -1
    _, Ap2, Am2 = dg.element_data(mesh.X, mats, nb)
    assert np.all(Am2[0, 2] == 0)
    ap_self, _ = oel.flux_matrices(mesh.X[:1], mats[:1], None, neighbour_materials=np.tile(mats[:1], (1, 4, 1)).reshape(1, 4, 3))
    assert np.allclose(Ap2[0, 2], ap_self[0, 2], rtol=1e-12, atol=1e-12 * np.abs(ap_self).max())


def test_plan_argument_errors():
    import paper_1903_11521_amd as dg
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.dg_plan_create(7, 0, ctypes.byref(h)) == -2
    assert lib.dg_plan_create(1, 0, ctypes.byref(h)) == -2
    assert lib.dg_plan_create(3, 9, ctypes.byref(h)) == -2
    assert b"degree" in lib.dg_last_error() or b"precision" in lib.dg_last_error()
    assert lib.dg_plan_create(3, 0, ctypes.byref(h)) == 0
    assert lib.dg_volume(h, -1, None, None, None, None) == -1
    assert lib.dg_volume(h, 5, None, None, None, None) == -1
    assert b"null pointer" in lib.dg_last_error()
    assert lib.dg_volume(h, 0, None, None, None, None) == 0  # empty input is a no-op
    assert lib.dg_step(h, 5, 0.1, -1, *([None] * 10)) == -1
    assert lib.dg_step_fused(h, 5, 0.1, *([None] * 10)) == -1
    assert b"null pointer" in lib.dg_last_error()
    assert lib.dg_plan_fuses_steps(h) == 1          # degree 3: fused launch
    assert lib.dg_plan_fuses_steps(None) == -1
    assert lib.dg_plan_tune(None, 1000, None) == -1
    assert lib.dg_plan_tune(h, 10, None) == -1      # tuning size out of range, rejected before any allocation
    assert b"tuning size" in lib.dg_last_error()
    mis = ctypes.c_void_p(8)   # never dereferenced: rejected before any launch
    assert lib.dg_volume(h, 5, mis, mis, mis, None) == -1
    assert b"aligned" in lib.dg_last_error()
    assert lib.dg_plan_destroy(h) == 0
    B, Bf = ctypes.c_int(), ctypes.c_int()
    p = dg.Plan(5)
    assert (p.B, p.Bf) == (56, 21)
    del B, Bf


def test_flop_and_byte_models():
    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd import perfmodel as pm
    _lib()
    f = dg.flop_model(5)
    # the paper's SeisSol kernels at order 6 need about 253.5k non-zero flops per
    # element-update (appendix tables); this algorithm computes the face traces
    # once per element, so it needs somewhat fewer
    assert 150e3 < f["step"] < 300e3
    # method bytes per element at degree 5, FP64: Q 4032 B, packed star 648 B,
    # A+ and A- 2592 B each, tables 20 B
    b = pm.method_bytes(5)
    assert b["step_correct"] == 4032 * 3 + 648 + 2 * 2592 + 20
    assert b["step_predict"] == 4032 * 2 + 648
    assert b["step"] == 4032 * 4 + 648 + 2 * 2592 + 20
    assert b["predictor"] == 4032 + 648 + 72 * (56 + 35 + 20 + 10 + 4 + 1)
    # the layout's own bytes add the face traces (6048 B per element)
    lb = pm.layout_bytes(5)
    assert lb["step_correct"] - b["step_correct"] == 2 * 6048
    # step rooflines: 310 M/s at degree 5 and 155 M/s at degree 6 (FP64)
    assert abs(pm.step_roofline_rate(5) / 310.06e6 - 1) < 1e-3
    assert abs(pm.step_roofline_rate(6) / 155.34e6 - 1) < 1e-3
    r = pm.kernel_roofline(135e3 * 1000, 17948 * 1000, 17948 * 1000 / 4e12)
    assert r["bound"] == "hbm" and abs(r["frac"] - 0.5) < 1e-12


def test_lts_argument_errors():
    """dg_lts_create rejects bad schedules before it touches the device."""
    import numpy as np
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.dg_plan_create(3, 0, ctypes.byref(h)) == 0
    ip = ctypes.POINTER(ctypes.c_int32)
    out = ctypes.c_void_p()
    neigh = np.array([[1, -1, -1, -1], [0, 2, -1, -1], [1, -1, -1, -1]], dtype=np.int32)

    def create(cl, nb=neigh, dt0=1e-3, plan=h):
        cl = np.ascontiguousarray(cl, dtype=np.int32)
        return lib.dg_lts_create(plan, len(cl), cl.ctypes.data_as(ip), nb.ctypes.data_as(ip),
                                 ctypes.c_double(dt0), ctypes.byref(out))
    assert create([1, 0, 0]) == -1 and b"cluster by cluster" in lib.dg_last_error()
    assert create([0, 0, 2], np.array([[1, -1, -1, -1], [0, 2, -1, -1], [1, -1, -1, -1]], np.int32)) == -1
    assert b"more than one cluster" in lib.dg_last_error()
    assert create([0, 0, 16]) == -1 and b"outside" in lib.dg_last_error()
    assert create([0, 0, 1], dt0=0.0) == -1 and b"dt0" in lib.dg_last_error()
    bad = neigh.copy()
    bad[2, 3] = 3
    assert create([0, 0, 1], bad) == -1 and b"neighbour" in lib.dg_last_error()
    hb = ctypes.c_void_p()
    assert lib.dg_plan_create(3, 3, ctypes.byref(hb)) == 0
    assert create([0, 0, 1], plan=hb) == -2 and b"not available" in lib.dg_last_error()
    assert lib.dg_lts_create(h, 0, None, None, ctypes.c_double(1e-3), ctypes.byref(out)) == 0
    n, u = ctypes.c_int(), ctypes.c_int64()
    assert lib.dg_lts_clusters(out, ctypes.byref(n), ctypes.byref(u)) == 0 and n.value == 0 and u.value == 0
    assert lib.dg_lts_advance(out, 3, *([None] * 7)) == 0      # empty mesh: nothing to do
    assert lib.dg_lts_destroy(out) == 0
    assert lib.dg_lts_advance(None, 1, *([None] * 7)) == -1
    lib.dg_plan_destroy(hb)
    lib.dg_plan_destroy(h)


@pytest.mark.parametrize("order", [2, 3, 5, 8, 12, 16])
def test_lina_coefficients_match_oracle(order):
    """The product's LinA blob (Newton-iterated Gauss-Lobatto points, the
    closed-form collocation derivative) against the oracle's (companion-
    matrix roots, barycentric derivative)."""
    import numpy as np
    import paper_1903_11521_amd as dg
    from oracle import lina
    rho0, K0, h = 1.2, 1.4e5, 0.25
    got = dg.lina_coefficients(order, rho0, K0, h)
    m = lina.matrices(order - 1)
    star, Ap, Am = lina.element_matrices(rho0, K0, h)
    for name, ref in (("w", m["w"]), ("Kt", m["Kt"]), ("Kh", m["Kh"]), ("star", star), ("Ap", Ap), ("Am", Am)):
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got[name] - ref)) <= 1e-12 * scale * order, name
    lib = _lib()
    assert lib.dg_lina_blob_size(1) == -1 and lib.dg_lina_blob_size(17) == -1
    out = np.zeros(lib.dg_lina_blob_size(4))
    assert lib.dg_lina_coefficients(4, -1.0, K0, h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == -1
    assert lib.dg_lina_step(0, 13, 8, 1, 1e-3, *([None] * 5)) == -2      # FP64 order above the limit
    assert lib.dg_lina_step(3, 4, 8, 1, 1e-3, *([None] * 5)) == -2       # split-BF16: not a LinA form
    assert lib.dg_lina_step(0, 4, 8, 1, 1e-3, *([None] * 5)) == -1       # null pointers
    assert lib.dg_lina_step(0, 4, 0, 1, 1e-3, *([None] * 5)) == 0        # empty grid


def test_visco_element_data_matches_oracle():
    """The product's viscoelastic star and flux rows (impedance form of the
    Godunov state) against the oracle's (eigenvector projector)."""
    import numpy as np
    import paper_1903_11521_amd as dg
    from oracle import viscoelastic as ve
    from workload import cube_mesh, random_materials, seed_for
    mesh = cube_mesh(3, seed_for(7), relabel=True)
    mats = random_materials(mesh.E, seed_for(7))
    omega = np.array([0.7, 3.0, 9.0])
    Ylam, Ymu = ve.memory_parameters(mats, omega, [0.02, 0.01, 0.04], [0.03, 0.015, 0.005])
    nb = mesh.neigh.copy()
    nb[0, 2] = -1
    star, Ap, Am = dg.visco_element_data(mesh.X, mats, omega, Ylam, Ymu, nb)
    ostar = ve.star_matrices(mesh.X, mats, omega, Ylam, Ymu)
    oAp, oAm = ve.flux_matrices(mesh.X, mats, omega, Ylam, Ymu, nb)
    assert np.all(ostar[..., 9:] == 0) and np.all(oAp[..., 9:] == 0) and np.all(oAm[..., 9:] == 0)
    for got, ref in ((star, ostar[..., :9]), (Ap, oAp[..., :9]), (Am, oAm[..., :9])):
        assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert np.all(Am[0, 2] == 0)


def test_batch_item_argument_errors():
    """Batch items are checked before anything touches the device: quantity
    counts other than 9 and 27, viscoelastic items outside an FP64 batch and
    bad relaxation frequencies."""
    import ctypes
    import paper_1903_11521_amd._lib as L
    lib = L._load()
    fake = 1 << 20                               # never dereferenced: the checks fail first

    def item(n_quant, omega=(1.0, 2.0, 3.0)):
        return L.BatchItem(3, 10, 1e-3, fake, fake, fake, fake, fake, fake, fake, fake, n_quant,
                           (ctypes.c_double * 3)(*omega))
    out = ctypes.c_void_p()
    arr = (L.BatchItem * 1)(item(12))
    assert lib.dg_batch_create(0, arr, 1, ctypes.byref(out)) == -1 and b"neither 9 nor 27" in lib.dg_last_error()
    arr = (L.BatchItem * 1)(item(27))
    assert lib.dg_batch_create(1, arr, 1, ctypes.byref(out)) == -2 and b"DG_FP64" in lib.dg_last_error()
    arr = (L.BatchItem * 1)(item(27, (1.0, -1.0, 2.0)))
    assert lib.dg_batch_create(0, arr, 1, ctypes.byref(out)) == -1 and b"relaxation" in lib.dg_last_error()
    arr = (L.BatchItem * 1)(item(27, (1.0, float("nan"), 2.0)))
    assert lib.dg_batch_create(0, arr, 1, ctypes.byref(out)) == -1 and b"relaxation" in lib.dg_last_error()
    assert not out.value


def test_visco_tune_argument_errors():
    """Rejected before anything touches the device."""
    import ctypes
    import paper_1903_11521_amd._lib as L
    lib = L._load()
    w, g = ctypes.c_int(), ctypes.c_int()
    assert lib.dg_visco_tune(7, 1000, None, ctypes.byref(w), ctypes.byref(g)) == -2
    assert b"degree" in lib.dg_last_error()
    assert lib.dg_visco_tune(5, 10, None, ctypes.byref(w), ctypes.byref(g)) == -1
    assert b"tuning size" in lib.dg_last_error()


def test_visco_shape_set_and_get():
    """Host-only launch-shape table of the viscoelastic kernels."""
    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd._lib import DGError
    old = dg.visco_shape(3)
    assert dg.visco_shape(3, (8, 2)) == (8, 2)
    assert dg.visco_shape(3, old) == old
    for bad in ((6, 0), (4, -1), (4, 65)):
        with pytest.raises(DGError):
            dg.visco_shape(3, bad)
    with pytest.raises(DGError):
        dg.visco_shape(7)
