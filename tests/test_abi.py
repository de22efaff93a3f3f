"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and the host-side validation rejects bad descriptors (no GPU call)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1501_04840_amd import otdyn
    if not os.path.exists(otdyn.LIB_PATH):
        from paper_1501_04840_amd import build
        build.build()
    return otdyn


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ot_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    import ctypes
    lib = ctypes.CDLL(L.LIB_PATH)
    names = [n for h in os.listdir(os.path.join(ROOT, "include")) for n in _declared(h)]
    assert "ot_dyn_create" in names and "ot_dyn_step" in names and "ot_dyn_solve" in names
    for n in names:
        assert hasattr(lib, n), n


def test_default_desc_and_workspace(L):
    d = L.ot_dyn_default_desc(256, 256, 3, 32)
    assert (d.X, d.Y, d.C, d.P) == (256, 256, 3, 32)
    assert list(d.bc) == [L.OT_BC_NEUMANN, L.OT_BC_NEUMANN, L.OT_BC_PERIODIC]
    assert d.tau * d.sigma < 1 and d.theta == 1.0 and d.batch == 1 and d.adapt == 0
    assert d.prox == L.OT_PROX_NEWTON
    n = L.ot_dyn_workspace_size(d)
    N = 256 * 256 * 3 * 32
    assert n >= 15 * N * 4          # b, b_bar, a (4 fields each), r, r' and Phi
    assert n < 16 * N * 4 + (1 << 24)
    d.batch = 3
    assert L.ot_dyn_workspace_size(d) > 3 * 15 * N * 4


@pytest.mark.parametrize("field,value,status", [
    ("P", 1, -2), ("X", 0, -2), ("C", 100, -2), ("tau", 20.0, -1), ("sigma", -1.0, -1),
    ("theta", 1.5, -1), ("check_every", 0, -1), ("refine", 4, -1), ("refine", -1, -1), ("batch", 0, -2),
    ("adapt", 2, -1), ("prox", 2, -1), ("prox", -1, -1),
])
def test_descriptor_validation(L, field, value, status):
    d = L.ot_dyn_default_desc(16, 16, 3, 8)
    setattr(d, field, value)
    with pytest.raises(L.OtDynError) as e:
        L.ot_dyn_workspace_size(d)
    assert e.value.status == status


def test_bad_bc_and_extent(L):
    d = L.ot_dyn_default_desc(16, 16, 3, 8)
    d.bc[2] = 7
    with pytest.raises(L.OtDynError):
        L.ot_dyn_workspace_size(d)
    d = L.ot_dyn_default_desc(16, 16, 3, 8)
    d.extent[0] = 0.0
    with pytest.raises(L.OtDynError):
        L.ot_dyn_workspace_size(d)


def test_create_rejects_small_or_misaligned_workspace(L):
    d = L.ot_dyn_default_desc(16, 16, 3, 8)
    n = L.ot_dyn_workspace_size(d)
    with pytest.raises(L.OtDynError) as e:
        L.ot_dyn_create(d, 0, 0, n)            # null workspace
    assert e.value.status == L.OT_ERR_SHAPE
    with pytest.raises(L.OtDynError) as e:
        L.ot_dyn_create(d, 0, 1 << 20, n - 1)  # too small: rejected before any HIP call
    assert e.value.status == L.OT_ERR_SHAPE
    with pytest.raises(L.OtDynError) as e:
        L.ot_dyn_create(d, 0, (1 << 20) + 8, n)  # misaligned
    assert e.value.status == L.OT_ERR_SHAPE


def test_status_strings(L):
    for s in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert L.ot_dyn_status_str(s)
    assert L.ot_dyn_status_str(-99) == "unknown status"


def test_prox_eval_rejects_bad_arguments(L):
    """Argument errors of ot_dyn_prox_eval come back before any device call."""
    import ctypes
    lib = L.lib()
    buf = (ctypes.c_float * 12)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.ot_dyn_prox_eval(0, 4, None, p, 1.0, p, p, None) == L.OT_ERR_PARAM
    assert lib.ot_dyn_prox_eval(3, 4, p, p, 1.0, p, p, None) == L.OT_ERR_PARAM     # unknown kind
    assert lib.ot_dyn_prox_eval(-1, 4, p, p, 1.0, p, p, None) == L.OT_ERR_PARAM
    assert lib.ot_dyn_prox_eval(0, -1, p, p, 1.0, p, p, None) == L.OT_ERR_PARAM    # n < 0
    assert lib.ot_dyn_prox_eval(1, 4, p, p, 0.0, p, p, None) == L.OT_ERR_PARAM     # sigma <= 0


def test_hue_renderer_rejects_bad_sizes(L):
    """Host-side checks of ot_hue_workspace_size / ot_hue_create and of the
    other hue entry points (they return before any HIP call)."""
    import ctypes
    from paper_1501_04840_amd import othue
    for npix, nbins, frames in [(0, 64, 1), (-5, 64, 1), (10, 1, 1), (10, 4097, 1),
                                ((1 << 30) + 1, 64, 1), (10, 64, 0), (10, 64, 65536)]:
        with pytest.raises(L.OtDynError) as e:
            othue.ot_hue_workspace_size(npix, nbins, frames)
        assert e.value.status == L.OT_ERR_SHAPE
    n = othue.ot_hue_workspace_size(3840 * 2160, 360, 33)
    assert 20 * 3840 * 2160 <= n < 21 * 3840 * 2160 + (1 << 20)
    lib = othue.lib()
    out = ctypes.c_void_p()
    assert lib.ot_hue_create(16, 8, 1, None, None, 0, None) == L.OT_ERR_PARAM
    n = othue.ot_hue_workspace_size(16, 8, 1)
    assert lib.ot_hue_create(16, 8, 1, None, None, n, ctypes.byref(out)) == L.OT_ERR_SHAPE
    assert lib.ot_hue_create(16, 8, 1, None, 1 << 20, n - 1, ctypes.byref(out)) == L.OT_ERR_SHAPE
    assert lib.ot_hue_create(16, 8, 1, None, (1 << 20) + 4, n, ctypes.byref(out)) == L.OT_ERR_SHAPE
    assert lib.ot_hue_set_source(None, None) == L.OT_ERR_PARAM
    assert lib.ot_hue_render(None, None, 1, None, None) == L.OT_ERR_PARAM
    assert lib.ot_hue_histogram(None, None, None) == L.OT_ERR_PARAM
    assert lib.ot_hue_plan_info(None, 0, None, None) == L.OT_ERR_PARAM
    assert lib.ot_hue_plan(None, None, 1) == L.OT_ERR_PARAM
    assert lib.ot_hue_apply(None, None, None) == L.OT_ERR_PARAM
    assert lib.ot_hue_rgb_to_hsv(None, 5, None, None) == L.OT_ERR_PARAM
    assert lib.ot_hue_hsv_to_rgb(None, -1, None, None) == L.OT_ERR_PARAM
    assert lib.ot_hue_rgb_to_hsv(None, 0, None, None) == L.OT_OK


def test_batch_grouping_and_workspace_on_the_host(L):
    """Batch grouping and workspace layout are host logic (no GPU call): the
    1024 hue problems of uneven sizes, RGB problems of several resolutions,
    and the argument checks of the batch entry points."""
    from synth import inputs
    base = L.ot_dyn_default_desc(1, 1, 1, 2)
    base.bc[0] = L.OT_BC_PERIODIC
    dims = [(n, 1, 1, T) for n, T, _, _ in inputs.cfg4_problems(1024)]
    total = L.ot_dyn_batch_workspace_size(base, dims)
    cells = sum(n * T for n, _, _, T in dims)
    assert total > 15 * 4 * cells
    per_shape = {}
    for dd in dims:
        per_shape[dd] = per_shape.get(dd, 0) + 1
    assert len(per_shape) <= 10
    rgb = [(16, 16, 3, 8), (24, 20, 3, 8), (16, 16, 3, 8), (64, 1, 1, 16), (30, 1, 1, 8)]
    assert L.ot_dyn_batch_workspace_size(L.ot_dyn_default_desc(1, 1, 3, 2), rgb) > 0
    for bad, status in [([(0, 1, 1, 8)], L.OT_ERR_SHAPE), ([(8, 1, 1, 1)], L.OT_ERR_SHAPE),
                        ([], L.OT_ERR_PARAM)]:
        with pytest.raises(L.OtDynError) as e:
            L.ot_dyn_batch_workspace_size(base, bad)
        assert e.value.status == status
    with pytest.raises(L.OtDynError) as e:
        L.ot_dyn_batch_create(base, rgb, 0, 0, 1 << 20)     # null workspace
    assert e.value.status == L.OT_ERR_SHAPE


@pytest.mark.parametrize("field,value", [("carry_refine", -1)])
def test_descriptor_validation_new_fields(L, field, value):
    d = L.ot_dyn_default_desc(16, 16, 3, 8)
    assert d.carry_refine == 64
    setattr(d, field, value)
    with pytest.raises(L.OtDynError) as e:
        L.ot_dyn_workspace_size(d)
    assert e.value.status == L.OT_ERR_PARAM
