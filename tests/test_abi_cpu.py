"""CPU checks of the C ABI: the library loads without a GPU and exports every
function include/ipt.h declares (no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ipt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ipt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (the HIP runtime libipt.so binds to)
    from paper_2012_14702_amd import ipt
    if not os.path.exists(ipt.library_path()):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(ipt.library_path())


def test_header_declares_entry_points():
    names = _declared()
    for want in ("ipt_create", "ipt_destroy", "ipt_solve_dense", "ipt_solve_csr", "ipt_solve_batched",
                 "ipt_status_string", "ipt_last_error", "ipt_opts_default"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    missing = [nm for nm in _declared() if not hasattr(lib, nm)]
    assert not missing, missing


def test_status_strings_and_defaults(lib):
    from paper_2012_14702_amd import ipt
    l = ipt.load_library()
    for code in range(6):
        assert l.ipt_status_string(code).startswith(b"IPT_")
    o = ipt.default_opts()
    assert o.tol == 1e-10 and o.max_iter == 100 and o.precision == 0 and o.div_growth == 8


def test_null_handle_is_rejected(lib):
    from paper_2012_14702_amd import ipt
    l = ipt.load_library()
    assert l.ipt_destroy(None) == ipt.IPT_EINVAL
    assert l.ipt_create(None, None) == ipt.IPT_EINVAL
    assert l.ipt_solve_dense(None, 4, None, None, 4, 4, None, None, 0, None, None, 4, None, None, None,
                             None) == ipt.IPT_EINVAL
    assert l.ipt_batched_get_tiles(None, None) == ipt.IPT_EINVAL
    assert l.ipt_batched_set_tiles(None, None) == ipt.IPT_EINVAL


def test_product_path_has_no_oracle_dependency():
    """The package never imports, links or calls the test oracle."""
    pkg = os.path.join(ROOT, "paper_2012_14702_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower().replace("oracle-free", ""), f
