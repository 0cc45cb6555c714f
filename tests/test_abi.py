"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function that include/pic.h declares, and rejects bad calls cleanly."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^PIC_API[^(;]*?\b(pic_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1612_03369_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1612_03369_amd import build as B
        B.build(force=False)
    return L.load()


def test_header_lists_every_entry_point():
    names = declared_functions()
    from paper_1612_03369_amd import _lib as L
    assert names == sorted(L.EXPORTS)
    assert len(names) >= 29


def test_library_exports_every_declared_symbol(lib):
    from paper_1612_03369_amd import _lib as L
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (pic_\w+)", out))
    assert set(declared_functions()) <= exported
    for n in declared_functions():
        getattr(lib, n)
    # nothing else leaks out under the pic_ prefix
    assert exported == set(declared_functions())


def test_null_and_bad_arguments_are_rejected(lib):
    from paper_1612_03369_amd import _lib as L
    n3 = (C.c_int32 * 3)(4, 4, 4)
    lo = (C.c_double * 3)(0, 0, 0)
    hi = (C.c_double * 3)(1, 1, 1)
    assert lib.pic_mesh_uniform(None, 3, n3, lo, hi) == L.PIC_EINVAL
    assert lib.pic_advance(None, 0.1, 1, L.PIC_RK2, L.PIC_F64) == L.PIC_EINVAL
    assert lib.pic_create(None, 0, None) == L.PIC_EINVAL
    assert lib.pic_last_error(None) == b"null context"
    assert lib.pic_batch_last_error(None) == b"null batch"
    lib.pic_destroy(None)
    lib.pic_batch_destroy(None)


def test_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1612_03369_amd import _lib as L
    h = C.c_void_p()
    assert lib.pic_create(C.byref(h), 0, None) == L.PIC_EDEVICE
    assert not h.value


def test_python_api_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1612_03369_amd.api import Problem
    with pytest.raises(RuntimeError):
        Problem(0)


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1612_03369_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".inc", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from\s+oracle|import\s+oracle)|liboracle|pic_oracle", txt, flags=re.M), f
