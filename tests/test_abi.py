"""The C-ABI library loads and exports every symbol include/pfk.h declares (CPU only)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfk.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pfk_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_list():
    from paper_1511_07226_amd import EXPORTED
    assert _declared() == sorted(EXPORTED)


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_1511_07226_amd import lib_path
    if not os.path.exists(lib_path()):
        pytest.fail("libpfk.so is not built (run python -m paper_1511_07226_amd.build)")
    L = ctypes.CDLL(lib_path())
    missing = [s for s in _declared() if not hasattr(L, s)]
    assert not missing, missing


def test_default_opts_and_error_path_without_gpu():
    from paper_1511_07226_amd import binding
    o = binding.default_opts()
    assert o.graph_iters >= 1 and o.max_restarts == 10 and o.force_breakdown_at == -1
    assert o.shift_sigma != o.shift_sigma            # NaN: estimate
    # argument validation runs on the host before any device call
    import ctypes as C
    h = C.c_void_p()
    nn = (C.c_int64 * 3)(8, 9, 8)
    code = binding.lib().pfk_operator_create(3, nn, None, None, 0, C.byref(h))
    assert code == -1 and b"eta" in binding.lib().pfk_last_error()


def test_binding_never_imports_the_oracle():
    import ast
    pkg = os.path.join(ROOT, "paper_1511_07226_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(dirpath, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        names = [a.name for a in node.names]
                    elif isinstance(node, ast.ImportFrom):
                        names = [node.module or ""]
                    else:
                        continue
                    assert not any(n == "oracle" or n.startswith("oracle.") for n in names), (f, names)
