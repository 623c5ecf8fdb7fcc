"""The Python binding marshals the C ABI's structs with ctypes; a field that the
header and the binding place differently would pass wrong arguments without any
error.  This test compiles a small C program against include/mandel.h with gcc,
prints each struct's size and every field's offset, and compares them with the
ctypes classes field by field (names in order, offsets, total size)."""
import ctypes
import os
import subprocess

import pytest

from paper_2007_00745_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "mandel_window": native.Window,
    "mandel_window_dd": native.WindowDD,
    "mandel_sched": native.Sched,
    "mandel_view": native.ViewC,
    "mandel_tuning": native.Tuning,
    "mandel_launch": native.LaunchC,
}


def _c_layout(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mandel.h"',
             "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    return got


def test_ctypes_structs_match_header(tmp_path):
    got = _c_layout(tmp_path)
    for cname, cls in STRUCTS.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_header_has_no_fields_missing_from_binding(tmp_path):
    # every member the header declares appears in the binding: the last ctypes field
    # ends exactly where the C struct ends (up to the struct's own tail padding)
    got = _c_layout(tmp_path)
    for cname, cls in STRUCTS.items():
        last, ftype = cls._fields_[-1]
        end = getattr(cls, last).offset + ctypes.sizeof(ftype)
        size = got[(cname, "sizeof")]
        align = max(ctypes.alignment(t) for _, t in cls._fields_)
        assert size - end < align, (cname, size, end)


def test_binding_constants_match_header(tmp_path):
    # the policy numbers and the automatic row-parts value as the header defines them
    src = tmp_path / "consts.c"
    src.write_text('#include <stdio.h>\n#include "mandel.h"\nint main(void) {\n'
                   'printf("%d %d %d %d %d %d\\n", MANDEL_FCFS_TILES, MANDEL_STATIC_ROWS, '
                   'MANDEL_ALTERNATING_ROWS, MANDEL_ORDERED_TILES, MANDEL_GRID_TILES, '
                   'MANDEL_TILE_PARTS_AUTO);\nreturn 0;\n}\n')
    exe = tmp_path / "consts"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True, capture_output=True, text=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == [native.FCFS_TILES, native.STATIC_ROWS, native.ALTERNATING_ROWS,
                   native.ORDERED_TILES, native.GRID_TILES, native.TILE_PARTS_AUTO]


if __name__ == "__main__":
    pytest.main([__file__, "-q"])
