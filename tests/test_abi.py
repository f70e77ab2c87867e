"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(itm_[a-z0-9_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def libpath():
    import paper_1410_0925_amd as itm
    if not os.path.exists(itm.LIB_PATH):
        from paper_1410_0925_amd import build
        build.build()
    return itm.LIB_PATH


def test_header_declares_the_boundary():
    names = declared()
    for n in ("itm_scene_create", "itm_integrate", "itm_raycast", "itm_export_blocks"):
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = declared() - exported
    assert not missing, missing


def test_binding_loads_and_names_match(libpath):
    import paper_1410_0925_amd as itm
    L = itm.lib()
    for n in declared():
        assert hasattr(L, n)
        assert n in itm.EXPORTED
    assert itm.itm_last_error() == ""


def test_binding_refuses_host_tensors(libpath):
    import numpy as np
    import torch
    import paper_1410_0925_amd as itm
    with pytest.raises(TypeError):
        itm._dev(torch.zeros(4), "torch.float32", 4)
    with pytest.raises(TypeError):
        itm._dev(np.zeros(4, np.float32), "torch.float32", 4)
