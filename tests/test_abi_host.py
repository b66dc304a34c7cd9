"""Host-side checks of the C ABI: the library loads, exports every entry point that include/vpm.h
declares, validates parameters without a device, and reports a missing device cleanly."""
import ctypes as C
import os
import re

import pytest

from paper_1504_00636_amd import vpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vpm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = vpm.lib()
    names = _declared()
    assert "vpm_run" in names and "vpm_partition" in names and "vpm_merge" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(vpm.EXPORTS) == set(names)


def test_version_string():
    assert "gfx950" in vpm.vpm_version()


def _p(**kw):
    base = dict(tol_x=0.1, tol_p=0.05, n_min_cell=0, min_subset=4, cell_len=(1, 1, 1), mass=1.0)
    base.update(kw)
    return vpm.make_params(**base)


def test_check_params_accepts_valid():
    assert vpm.vpm_check_params(_p()) == vpm.VPM_OK
    assert vpm.vpm_check_params(_p(decide=vpm.VPM_DECIDE_FP64)) == vpm.VPM_OK
    assert vpm.vpm_check_params(_p(merge_mode=vpm.VPM_MERGE_CENTROID, min_subset=1)) == vpm.VPM_OK
    assert vpm.vpm_check_params(_p(mass=0.0)) == vpm.VPM_OK


@pytest.mark.parametrize("bad", [
    dict(tol_x=-0.1), dict(tol_p=float("nan")), dict(tol_x=128.0), dict(tol_p=1e9),
    dict(n_min_cell=-1), dict(min_subset=0), dict(min_subset=1), dict(min_subset=70000),
    dict(cell_len=(1, 0, 1)), dict(cell_len=(1, 1, float("inf"))), dict(mass=-1.0),
    dict(merge_mode=7), dict(decide=3), dict(dtype=5),
])
def test_check_params_rejects(bad):
    assert vpm.vpm_check_params(_p(**bad)) == vpm.VPM_ERR_INVALID_ARG


def test_fp64_mode_allows_large_tolerance():
    assert vpm.vpm_check_params(_p(decide=vpm.VPM_DECIDE_FP64, tol_x=1e6)) == vpm.VPM_OK


def test_axis_rule_field():
    assert vpm.vpm_check_params(_p(axis_rule=vpm.VPM_AXIS_NORMALISED)) == vpm.VPM_OK
    for bad in (2, -1):
        p = _p()
        p.axis_rule = bad
        assert vpm.vpm_check_params(p) == vpm.VPM_ERR_INVALID_ARG


def test_null_params_rejected():
    assert vpm.lib().vpm_check_params(None) == vpm.VPM_ERR_INVALID_ARG


def test_status_strings():
    for st in (0, -1, -2, -3, -4, -5):
        assert vpm.status_string(st)


def test_create_without_gpu_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert vpm.lib().vpm_create(C.byref(h), 0) == vpm.VPM_ERR_NO_DEVICE


def test_entry_points_reject_null_context():
    L = vpm.lib()
    p = _p()
    assert L.vpm_run(None, None, None, 0, 0, C.byref(p), None, None, None, None) == vpm.VPM_ERR_INVALID_ARG
    assert L.vpm_partition(None, None, None, 0, 0, C.byref(p), None, None, None, None) == vpm.VPM_ERR_INVALID_ARG
    assert L.vpm_reserve(None, 1, 1) == vpm.VPM_ERR_INVALID_ARG


@pytest.mark.parametrize("masses", [[1.0, 1.0, 0.0], [], [1.0] * 9, [1.0, -1.0], [float("nan")], [float("inf")]])
def test_run_species_rejects_without_device(masses):
    """Null context, or a bad species table (none, more than VPM_MAX_SPECIES, negative or non-finite
    masses): rejected on the host before anything is enqueued."""
    L = vpm.lib()
    p = _p()
    tab = (C.c_double * max(1, len(masses)))(*masses)
    assert L.vpm_run_species(None, None, None, 0, 0, C.byref(p), None, tab, len(masses), None, None, None,
                             None) == vpm.VPM_ERR_INVALID_ARG


def _declared_arity():
    src = open(os.path.join(ROOT, "include", "vpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(vpm_[a-z_]+)\s*\(([^;{]*?)\)\s*;", src, flags=re.S):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_argument_counts_match_header():
    L = vpm.lib()
    ar = _declared_arity()
    assert ar["vpm_merge"] == 13 and ar["vpm_run"] == 10
    for name, n in ar.items():
        at = getattr(L, name).argtypes
        if at is not None:
            assert len(at) == n, (name, len(at), n)


@pytest.mark.parametrize("t,ok", [
    ((16, 576, 2048, 4352), True), ((8, 1, 1, 1), True), ((32, 320, 1024, 2560), True),
    ((4, 576, 2048, 4352), False), ((12, 576, 2048, 4352), False), ((16, 0, 2048, 4352), False),
    ((16, 577, 2048, 4352), False), ((16, 576, 575, 4352), False), ((16, 576, 2289, 4352), False), ((16, 576, 2288, 4352), True),
    ((16, 576, 2048, 2047), False), ((16, 576, 2048, 4593), False), ((16, 576, 2048, 4592), True),
    ((16, 576, 2048, 4352, 1), True), ((16, 576, 2048, 4352, 2), True), ((16, 576, 2048, 4352, 3), False), ((16, 576, 2048, 4352, -1), False),
    ((16, 576, 2048, 4352, 0, 0), True), ((16, 576, 2048, 4352, 0, 256), True), ((16, 576, 2048, 4352, 0, 257), False),
    ((16, 576, 2048, 4352, 0, -1), False), ((16, 576, 2048, 4352, 0, 128, 1), True),
    ((16, 576, 2048, 4352, 0, 128, 2), False), ((16, 576, 2048, 4352, 0, 128, -1), False),
    ((16, 576, 2048, 4352, 0, 128, 0, 576), True), ((16, 576, 2048, 4352, 0, 128, 0, 1144), True),
    ((16, 576, 2048, 4352, 0, 128, 0, 575), False), ((16, 576, 2048, 4352, 0, 128, 0, 1145), False),
    ((16, 300, 800, 4352, 0, 128, 0, 900), False), ((16, 300, 800, 4352, 0, 128, 0, 800), True)])
def test_check_tuning(t, ok):
    st = vpm.vpm_check_tuning(vpm.make_tuning(*t))
    assert (st == vpm.VPM_OK) == ok, (t, st)


def _header_structs():
    """Field lists of the header's typedef'd structs: name -> [(c type, field, array length)]."""
    import re
    text = open(os.path.join(ROOT, "include", "vpm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.replace("const", " ").strip()
            if not decl:
                continue
            base, first = re.match(r"(\w+)\s+(.*)$", decl).groups()
            for item in first.split(","):               # "void *x, *y" declares several
                m = re.match(r"\s*(\*?)\s*(\w+)\s*(?:\[(\w+)\])?\s*$", item)
                assert m, decl
                fields.append((base + (" *" if m.group(1) else ""), m.group(2), m.group(3)))
        out[name] = fields
    return out


@pytest.mark.parametrize("cname,pyclass", [("vpm_params", "VpmParams"), ("vpm_tuning", "VpmTuning"),
                                           ("vpm_soa", "VpmSoa")])
def test_binding_structs_match_header(cname, pyclass):
    """The ctypes structures have the header's fields, in its order, with matching types and sizes."""
    hdr = _header_structs()[cname]
    py = getattr(vpm, pyclass)._fields_
    assert [f for _, f, _ in hdr] == [f for f, _ in py]
    ctype = {"int32_t": C.c_int32, "double": C.c_double, "void *": C.c_void_p, "void*": C.c_void_p}
    for (t, f, n), (pf, pt) in zip(hdr, py):
        want = ctype[t]
        if n is not None:
            assert issubclass(pt, C.Array) and pt._type_ is want and pt._length_ == int(n), f
        else:
            assert pt is want, f
