"""The C-ABI library loads, exports every entry point its header declares, and
rejects bad parameters with documented status codes (no GPU needed: nothing
here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vfmm.h")
LIB = os.path.join(ROOT, "paper_1106_5273_amd", "libvfmm.so")


@pytest.fixture(scope="module")
def lib():
    import importlib.util
    if not os.path.exists(LIB):
        spec = importlib.util.spec_from_file_location("vfmm_build", os.path.join(ROOT, "paper_1106_5273_amd", "build.py"))
        m = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(m)
        m.build()
    return ctypes.CDLL(LIB)


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fmm_build", "fmm_evaluate", "rk_step", "vfmm_create", "vfmm_destroy", "vfmm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_exports_match_header():
    import paper_1106_5273_amd as vf
    assert sorted(vf.EXPORTED) == declared_functions()


@pytest.mark.parametrize("kw,needle", [
    (dict(p=7), "p must be"),
    (dict(ncrit=0), "ncrit"),
    (dict(theta=1.5), "theta"),
    (dict(periodic=1, box_len=0.0), "box_len"),
    (dict(periodic=1, box_len=1.0, images=0), "images"),
    (dict(periodic=1, box_len=1.0, direct=1), "direct"),
    (dict(scheme=5), "scheme"),
])
def test_create_rejects_bad_parameters(kw, needle):
    import paper_1106_5273_amd as vf
    p = vf.default_params(**kw)
    h = ctypes.c_void_p()
    st = vf._lib.vfmm_create(ctypes.byref(p), None, ctypes.byref(h))
    assert st == -1  # VFMM_EINVAL
    assert needle in vf._lib.vfmm_last_error(None).decode()
    assert not h.value


def test_null_context_is_rejected():
    import paper_1106_5273_amd as vf
    assert vf._lib.fmm_build(None, 10, None, None, None, None) == -1
    assert vf._lib.fmm_evaluate(None, 0, *([None] * 13)) == -1
    assert vf._lib.rk_step(None, 0, 0.0, 0.0, *([None] * 7)) == -1
    vf._lib.vfmm_destroy(None)


def test_default_parameters():
    import paper_1106_5273_amd as vf
    p = vf.default_params()
    assert (p.p, p.ncrit, p.periodic, p.images, p.scheme, p.zero_mean, p.direct) == (10, 64, 0, 3, 0, 1, 0)
    assert abs(p.theta - 0.5) < 1e-7 and abs(p.sigma_gap - 5.0) < 1e-7
    assert (p.kahan, p.m2l_mode, p.use_graph, p.precision, p.overlap, p.m2l_form) == (0, 0, 0, 0, 2, 2)


def test_unknown_parameter_is_rejected():
    import paper_1106_5273_amd as vf
    with pytest.raises(TypeError):
        vf.default_params(thetta=0.4)


def test_header_documents_readers_as_const_and_depth_policy():
    """Timings and statistics take a const context; VFMM_EDEPTH is documented
    as never returned (an overfull leaf at the key depth limit stays a leaf
    and is counted in the statistics)."""
    txt = open(HEADER).read()
    assert re.search(r"vfmm_get_timings\(const vfmm_ctx \*ctx", txt)
    assert re.search(r"vfmm_get_stats\(const vfmm_ctx \*ctx", txt)
    assert re.search(r"VFMM_EDEPTH = -3,\s*/\* never returned", txt)
    assert "overfull_leaves" in txt and "stale" in txt
    import paper_1106_5273_amd as vf
    names = [f for f, _ in vf.Stats._fields_]
    assert names[-2:] == ["stale", "overfull_leaves"]
