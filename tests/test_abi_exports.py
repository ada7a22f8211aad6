"""The C-ABI library loads without a GPU and exports every declared symbol."""
import os
import re

from paper_2510_23446_amd import tcf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(tcf\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    L = tcf.lib()
    names = declared_functions()
    assert "tcf_create" in names and "tcf_step" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"
    assert set(tcf.EXPORTS) <= set(names)


def test_default_options_and_error_string():
    o = tcf.default_options()
    assert o.precision == tcf.TCF_FP64 and o.pcg_rtol == 1e-10
    assert isinstance(tcf.lib().tcf_last_error(None), bytes)
