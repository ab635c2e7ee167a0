"""The C-ABI library loads without a GPU and exports every function include/rte.h declares.

No compute entry point is called here; only symbol lookup (and rte_strerror, which is host-only).
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rte.h")
LIB = os.path.join(ROOT, "paper_2402_10488_amd", "librte.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    names = re.findall(r"\b(rte_\w+)\s*\(", text)
    # typedef'd function-pointer or macro names would also match; keep real prototypes only
    protos = re.findall(r"(?:^|\n)\s*(?:const\s+)?\w+\s*\**\s*(rte_\w+)\s*\(", text)
    return sorted(set(protos) & set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2402_10488_amd import build
        build.build()
    # torch first, as the binding does: the library then binds to torch's HIP runtime, and a
    # later GPU test in this process does not find a second runtime loaded
    import torch  # noqa: F401
    return ctypes.CDLL(LIB)


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for required in ("rte_sweep", "rte_scalar_flux", "rte_dsa_correct", "rte_rom_correct",
                     "rte_sisa_solve", "rte_problem_create", "rte_rom_create",
                     "rte_workspace_size"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT\s+(rte_\w+)$", out, flags=re.M))
    assert set(names) <= exported, sorted(set(names) - exported)


def test_strerror_is_host_only_and_total(lib):
    lib.rte_strerror.restype = ctypes.c_char_p
    for code in range(0, 8):
        assert lib.rte_strerror(code)
    assert lib.rte_strerror(12345)


def test_binding_mirrors_the_abi():
    from paper_2402_10488_amd import rte
    names = declared_functions()
    assert set(rte.EXPORTED) <= set(names)


def test_binding_binds_the_library_to_one_hip_runtime():
    """torch carries its own libamdhip64 with the same soname as the system one the library links
    against.  Importing the binding (in a fresh process) must leave exactly one HIP runtime and one
    HSA runtime mapped: two would not share devices, memory or streams."""
    code = ("import re\n"
            "from paper_2402_10488_amd import rte\n"
            "maps = open('/proc/self/maps').read()\n"
            "libs = sorted(set(l.split()[-1] for l in maps.splitlines()\n"
            "                  if re.search(r'lib(amdhip64|hsa-runtime64)', l)))\n"
            "print('\\n'.join(libs))\n")
    out = subprocess.run(["python3", "-c", code], capture_output=True, text=True, check=True,
                         cwd=ROOT).stdout.split()
    assert sum("amdhip64" in l for l in out) == 1, out
    assert sum("hsa-runtime64" in l for l in out) == 1, out
