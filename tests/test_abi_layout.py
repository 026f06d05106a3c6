"""The C ABI (include/h2.h) against the Python binding
(paper_2502_02395_amd/h2.py), without a GPU.

Structs: the same members in the same order, at the same offsets, of the
same sizes, and the same struct sizes.  The header's member lists are read
from its text; the offsets and sizes come from a C program compiled against
the header.

Functions: every prototype against the binding's argtypes and restype, the
same number of arguments, each of the same class.

A member or argument added, removed, reordered or retyped on one side only
fails here."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_2502_02395_amd import h2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "h2.h")
STRUCTS = {"h2_kernel": h2.Kernel, "h2_params": h2.Params, "h2_stats_t": h2.Stats,
           "h2_allocator": h2.Allocator}


def _members(text, name):
    """Member names of `typedef struct { ... } name;`, in declaration order."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + re.escape(name) + r"\s*;", text)
    assert m, name
    body = m.group(1)
    out = []
    for decl in body.split(";"):
        decl = " ".join(decl.split())
        if not decl:
            continue
        fp = re.search(r"\(\s*\*\s*(\w+)\s*\)", decl)
        if fp:                       # function pointer
            out.append(fp.group(1))
            continue
        parts = [re.sub(r"\[.*?\]", "", p).strip() for p in decl.split(",")]
        out.append(re.findall(r"\w+", parts[0])[-1])
        out += [re.findall(r"\w+", p)[-1] for p in parts[1:]]
    return out


def test_member_lists_match():
    text = open(HEADER).read()
    for cname, cls in STRUCTS.items():
        assert _members(text, cname) == [f for f, _ in cls._fields_], cname


def test_offsets_and_sizes_match(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("needs a C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "h2.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} . %zu 0\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu %zu\\n", offsetof({cname}, {f}), '
                         f"sizeof((({cname}*)0)->{f}));")
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    r = subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", exe],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60, check=True).stdout
    seen = 0
    for line in out.splitlines():
        cname, f, a, b = line.split()
        cls = STRUCTS[cname]
        if f == ".":
            assert ctypes.sizeof(cls) == int(a), (cname, ctypes.sizeof(cls), a)
        else:
            fd = getattr(cls, f)
            assert (fd.offset, fd.size) == (int(a), int(b)), (cname, f, fd.offset, fd.size, a, b)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in STRUCTS.values())


def _cls_c(decl):
    """Argument class of a C parameter or return type."""
    d = " ".join(decl.split())
    if "*" in d or d.split()[0] == "h2_handle":
        return "ptr"
    base = d.replace("const ", "").split()[0]
    return {"int64_t": "i64", "int32_t": "i32", "int": "i32", "h2_status": "i32", "float": "f32",
            "double": "f64", "void": "void"}[base]


def _cls_ctypes(t):
    if t is None:
        return "void"
    if t in (ctypes.c_void_p, ctypes.c_char_p) or issubclass(t, ctypes._Pointer):
        return "ptr"
    if ctypes.sizeof(t) == 8 and t in (ctypes.c_int64, ctypes.c_long, ctypes.c_longlong):
        return "i64"
    if t in (ctypes.c_int32, ctypes.c_int):
        return "i32"
    return {ctypes.c_float: "f32", ctypes.c_double: "f64"}[t]


def test_function_signatures_match():
    """Every prototype of the header against the binding's argtypes and
    restype: the same number of arguments, each of the same class (pointer,
    32- or 64-bit integer, float, double)."""
    if not os.path.exists(h2.LIB_PATH):
        pytest.skip("libh2.so not built")
    L = h2.load()
    text = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)
    protos = re.findall(r"\b(h2_status|void|const char\s*\*)\s+(h2_\w+)\s*\(([^;{]*?)\)\s*;", text)
    assert len(protos) >= 18
    for ret, name, params in protos:
        fn = getattr(L, name)
        args = [p for p in (" ".join(params.split())).split(",") if p.strip()]
        want = [_cls_c(p.rsplit(" ", 1)[0] if not p.strip().endswith("*") else p) for p in args]
        got = [_cls_ctypes(t) for t in (fn.argtypes or [])]
        assert got == want, (name, got, want)
        rw = _cls_c(ret)
        rg = _cls_ctypes(fn.restype) if fn.restype is not ctypes.c_int else "i32"
        assert rg == rw or (rw == "ptr" and fn.restype is ctypes.c_char_p), (name, rg, rw)
