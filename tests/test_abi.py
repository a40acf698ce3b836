"""CPU-side checks of the boundary: the built library loads and exports every
entry point that include/dg.h declares (no compute call: no GPU here), and the
Python binding names the same entry points."""
import ctypes
import os
import re

import pytest

from paper_1812_04789_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b((?:dg|pmg|fgmres)_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for must in ("dg_residual", "dg_jvp", "pmg_setup", "pmg_apply", "fgmres_step", "dg_create", "dg_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_the_abi():
    assert set(_declared()) == set(binding.SIGNATURES)


def test_null_arguments_rejected_without_gpu_work():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load()
    out = ctypes.c_void_p()
    assert lib.dg_create(None, None, 2, None, ctypes.byref(out)) == binding.DG_EINVAL
    assert lib.dg_destroy(None) == binding.DG_EINVAL
    assert lib.dg_ndof(None) == 0
    assert lib.dg_residual(None, None, None) == binding.DG_EINVAL
    assert lib.dg_batched_lu(None, None, None, 1, 4) == binding.DG_EINVAL


def test_enums_match_header():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    kinds = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"DG_K_([A-Z0-9_]+)\s*=\s*(\d+)", src))
    count = kinds.pop("COUNT")
    assert len(binding.KERNEL_KINDS) == count
    for name, i in kinds.items():
        assert binding.KERNEL_KINDS[i] == name.lower()
    prec = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"DG_(FP64|FP32|BF16)\s*=\s*(\d+)", src))
    assert prec == {"FP64": binding.DG_FP64, "FP32": binding.DG_FP32, "BF16": binding.DG_BF16}


@pytest.mark.parametrize("cname,pyname", [("pmg_opts", "PmgOpts"), ("fgmres_opts", "FgmresOpts"),
                                          ("fgmres_stats", "FgmresStats"), ("dg_step_stats", "StepStats")])
def test_option_structs_match_header(cname, pyname):
    """The ctypes mirrors list the header's struct members in order."""
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    m = re.search(r"typedef struct \{([^}]*)\}\s*" + cname + r"\s*;", src)
    assert m, cname
    names = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        first = decl.split(",")
        head = re.match(r"^(?:const\s+)?[A-Za-z_]\w*(?:\s*\*)*\s+(.*)$", first[0]).group(1)
        for part in [head] + first[1:]:
            names.append(re.sub(r"\[.*\]", "", part).strip().lstrip("*").strip())
    fields = [f[0] for f in getattr(binding, pyname)._fields_]
    assert fields == names
