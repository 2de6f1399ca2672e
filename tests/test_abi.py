"""The C-ABI library loads and exports every symbol include/amc.h declares
(no compute call: these run on hosts without a GPU)."""
import ctypes
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2605_14743_amd import amc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "amc.h")).read()
    return sorted(set(re.findall(r"AMC_API\s+[^;(]*?\b(amc_\w+)\s*\(", text)))


def test_header_declares_the_binding_list():
    assert declared() == sorted(amc.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(amc.LIB_PATH):
        pytest.skip("libamc.so not built")
    lib = ctypes.CDLL(amc.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", amc.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert exported == set(declared()), exported ^ set(declared())


def test_strerror_and_version_without_gpu():
    if not os.path.exists(amc.LIB_PATH):
        pytest.skip("libamc.so not built")
    L = amc.lib()
    for rc in (amc.OK, amc.E_INVALID_ARG, amc.E_OOM, amc.E_HIP, amc.E_SIGMA_OVERFLOW, amc.E_SINGULAR,
               amc.E_ADMISSION, amc.E_NOT_READY, amc.E_UNSUPPORTED, -99):
        assert isinstance(L.amc_strerror(rc), bytes)
    assert L.amc_version() >= 100


def test_struct_layouts_match_header():
    """ctypes mirrors of the ABI structs have the sizes and field offsets a C compiler gives."""
    structs = {"amc_model": amc.Model, "amc_query": amc.Query, "amc_stats": amc.Stats, "amc_result": amc.Result,
               "amc_tune_result": amc.TuneResult, "amc_traj_query": amc.TrajQuery,
               "amc_traj_result": amc.TrajResult, "amc_robust_query": amc.RobustQuery,
               "amc_robust_result": amc.RobustResult, "amc_boot_query": amc.BootQuery,
               "amc_boot_result": amc.BootResult, "amc_stability_result": amc.StabilityResult,
               "amc_server_stats": amc.ServerStats}
    lines = []
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src = "#include <stdio.h>\n#include <stddef.h>\n#include \"amc.h\"\nint main(void) {\n" + "\n".join(lines) + \
        "\n  return 0;\n}\n"
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(ln.split() for ln in out if ln.strip())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, f"{cname}.{f}"
