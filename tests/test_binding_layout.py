"""The ctypes binding against the C header it marshals for (no GPU): every
prototype's return and argument types, and every struct's size and field
offsets as a C compiler lays them out from the header."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2603_00292_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt.h")
HANDLES = {"rt_context", "rt_accel", "rt_batch_plan"}
STRUCTS = {"rt_ray": _capi.rt_ray, "rt_hit": _capi.rt_hit, "rt_srt": _capi.rt_srt,
           "rt_mesh_desc": _capi.rt_mesh_desc, "rt_build_options": _capi.rt_build_options,
           "rt_variant": _capi.rt_variant, "rt_query_options": _capi.rt_query_options,
           "rt_tune_entry": _capi.rt_tune_entry, "rt_accel_info": _capi.rt_accel_info}


def header_text():
    s = open(HEADER).read()
    s = re.sub(r"/\*.*?\*/", "", s, flags=re.S)
    return re.sub(r"//[^\n]*", "", s)


def prototypes():
    out = {}
    for m in re.finditer(r"([A-Za-z_][\w \t\*]*?)\b(rt_\w+)\s*\(([^;{)]*)\)\s*;", header_text()):
        params = [p.strip() for p in m.group(3).split(",")]
        out[m.group(2)] = (m.group(1).strip(), [] if params == ["void"] else params)
    return out


def ctype_of(decl):
    """The ctypes type a C parameter or return type is passed as."""
    t = decl.replace("const", " ")
    if "*" in t:
        return "ptr"
    words = t.split()
    base = words[0] if len(words) == 1 else words[-2]
    if base in HANDLES:
        return "ptr"
    return {"uint32_t": "u32", "int": "int", "rt_status": "int", "float": "float",
            "uint64_t": "u64", "double": "double"}[base]


KIND = {C.c_void_p: "ptr", C.c_char_p: "ptr", C.c_uint32: "u32", C.c_int: "int", C.c_float: "float",
        C.c_uint64: "u64", C.c_double: "double"}


def test_every_prototype_matches_the_binding():
    lib = _capi.load()
    protos = prototypes()
    assert set(protos) == set(_capi.EXPORTS)
    for name, (ret, params) in protos.items():
        f = getattr(lib, name)
        assert KIND[f.restype] == ctype_of(ret + " x"), name
        got = [KIND[a] for a in f.argtypes]
        want = [ctype_of(p) for p in params]
        assert got == want, (name, got, want)


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    """sizeof and offsetof of every struct field, printed by a C program
    compiled against the header."""
    d = tmp_path_factory.mktemp("layout")
    fields = {}
    for m in re.finditer(r"typedef struct (\w+)\s*\{(.*?)\}\s*(\w+);", header_text(), flags=re.S):
        names = []
        for decl in m.group(2).split(";"):
            decl = decl.strip()
            if not decl:
                continue
            head = re.match(r"((?:const\s+)?\w+\s*\**)\s*(.*)", decl)
            names += [n.strip().lstrip("*") for n in head.group(2).split(",")]
        fields[m.group(3)] = names
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rt.h"', "int main(void) {"]
    for s, names in fields.items():
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for n in names:
            lines.append(f'  printf("{s} {n} %zu\\n", offsetof({s}, {n}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True, capture_output=True, timeout=120)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout
    lay = {}
    for line in out.splitlines():
        s, key, val = line.split()
        lay.setdefault(s, {})[key] = int(val)
    return fields, lay


def test_every_struct_matches_the_header(c_layout):
    fields, lay = c_layout
    assert set(fields) == set(STRUCTS)
    for s, cls in STRUCTS.items():
        assert C.sizeof(cls) == lay[s]["size"], s
        assert [f[0] for f in cls._fields_] == fields[s], s
        for n in fields[s]:
            assert getattr(cls, n).offset == lay[s][n], (s, n)
