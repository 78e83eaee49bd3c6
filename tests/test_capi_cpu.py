"""The C-ABI library loads and exports every function include/qtm.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

import paper_1810_03047_amd as qtm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qtm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(qtm_[a-z_]+)\s*\(", src, flags=re.M)))


def test_header_declarations_parsed():
    names = _declared()
    assert "qtm_create" in names and "qtm_run" in names and "qtm_expect" in names
    assert len(names) >= 15


@pytest.mark.skipif(not os.path.exists(qtm.LIB_PATH), reason="libqtm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(qtm.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert qtm.exported_names() == _declared()


@pytest.mark.skipif(not os.path.exists(qtm.LIB_PATH), reason="libqtm.so not built")
def test_binding_loads_and_defaults():
    qtm.load()
    o = qtm.Opts()._c()
    assert o.rtol == 1e-6 and o.atol == 1e-8 and o.precision == qtm.PREC_FP64
    assert qtm.last_error() == ""


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(qtm.QtmError):
        qtm.load(str(tmp_path / "nope.so"))


def test_mlp_constants_match_architecture():
    nf, nh, no = 16, 64, 3
    assert qtm.MLP_NPARAM == nh * nf + nh + nh * nh + nh + no * nh + no
    assert qtm.MLP_NTOTAL == qtm.MLP_NPARAM + 2 * nf
    hdr = open(os.path.join(ROOT, "include", "qtm.h")).read()
    assert f"#define QTM_MLP_NPARAM {qtm.MLP_NPARAM}" in hdr
    assert f"#define QTM_MLP_NTOTAL {qtm.MLP_NTOTAL}" in hdr


@pytest.mark.skipif(not os.path.exists(qtm.LIB_PATH), reason="libqtm.so not built")
def test_invalid_options_rejected_before_any_device_call():
    """Option checks come first in qtm_create, so they run without a GPU."""
    import workloads as w
    s = w.two_level()
    for bad in (dict(chunk_traj=-1), dict(team_waves=-1), dict(tile_cols=-2), dict(class_waves=(5, 0, 0)),
                dict(rtol=0.0), dict(precision=7), dict(integrator=9)):
        with pytest.raises(qtm.QtmError) as e:
            qtm.create_system(s, qtm.Opts(**bad))
        assert e.value.code == qtm.E_INVAL, bad
