"""The C ABI: libmcmi.so loads and exports every function include/mcmi.h declares
(no compute calls, so this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mcmi_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_the_three_calls():
    names = declared_functions()
    assert {"mcmi_build_cdf", "mcmi_spai", "mcmi_apply"} <= names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2409_03095_amd", "libmcmi.so"))
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2409_03095_amd import mcmi
    assert set(mcmi.EXPORTED) <= declared_functions()
    assert "gfx950" in mcmi.version()


def test_oracle_shares_no_code_with_the_library():
    """The oracle is plain C under oracle/ and includes nothing of the library."""
    src = open(os.path.join(ROOT, "oracle", "mcmi_oracle.c")).read()
    includes = re.findall(r"#include\s*(\S+)", src)
    assert includes and all(i.startswith("<") for i in includes), includes
    for fn in os.listdir(os.path.join(ROOT, "paper_2409_03095_amd", "csrc")):
        text = open(os.path.join(ROOT, "paper_2409_03095_amd", "csrc", fn)).read()
        assert "oracle" not in text.lower(), fn


STRUCTS = {"mcmi_csr_in": "CsrIn", "mcmi_csr_out": "CsrOut", "mcmi_params": "Params", "mcmi_stats": "Stats",
           "mcmi_cdf_opts": "CdfOpts", "mcmi_solve_stats": "SolveStats"}


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding passes has the header's size and field offsets, as
    a C compiler lays them out (gcc on the header, no library code)."""
    from paper_2409_03095_amd import mcmi
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mcmi.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(mcmi, pyname)
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, pyname in STRUCTS.items():
        cls = getattr(mcmi, pyname)
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_binding_shares_torchs_hip_runtime():
    """Imported before torch, the binding still maps a single HIP runtime, torch's:
    a second copy of the runtime in the process sees no device."""
    code = ("import sys; sys.path.insert(0, sys.argv[1])\n"
            "from paper_2409_03095_amd import learned\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print('\\n'.join(sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})))\n")
    out = subprocess.check_output(["python3", "-c", code, ROOT], text=True).split()
    assert len(out) == 1, out
