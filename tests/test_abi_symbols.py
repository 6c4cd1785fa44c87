"""The C-ABI library loads (no GPU needed) and exports every entry point the
public header declares; no compute call is made here."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lvq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lvq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_2402_02044_amd", "liblvq.so")
    if not os.path.exists(lib_path):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "build_lib", os.path.join(ROOT, "paper_2402_02044_amd", "build_lib.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    lib = ctypes.CDLL(lib_path)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_the_header():
    import paper_2402_02044_amd as L
    assert sorted(L.EXPORTS) == _declared()
    for n in _declared():
        assert callable(getattr(L, n))
    # pure host call: the row format of the C2 store
    assert L.lvq_row_format(L.lvq_config(768, 4, 8, 1, 1, 32, 0, 0)) == (416, 768, 768)
    assert L.lvq_row_format(L.lvq_config(96, 8, 0, 0, 0, 32, 0, 0)) == (128, 0, 96)
    assert L.lvq_strerror(L.LVQ_ERR_CAPACITY) == "not enough free slots"
