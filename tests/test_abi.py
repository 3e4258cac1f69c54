"""The C-ABI library: exported symbols and argument validation (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def isax():
    import paper_2009_01614_amd as isax
    if not os.path.exists(isax.LIB_PATH):
        from paper_2009_01614_amd import build
        build.build()
    isax.lib()
    return isax


def _declared():
    with open(os.path.join(ROOT, "include", "isax.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"\b(isax_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(isax):
    names = _declared()
    assert len(names) >= 20
    L = ctypes.CDLL(isax.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(isax.SIGNATURES), set(names) ^ set(isax.SIGNATURES)


def test_breakpoints_match_oracle_bit_for_bit(isax):
    from oracle import isax_ref
    for c in range(1, 9):
        assert np.array_equal(isax.breakpoints(c), isax_ref.breakpoints_f32(c))


def test_validation_before_device_work(isax):
    L = isax.lib()
    fake = ctypes.c_void_p(0x10000)
    cases = [((None, 10, 256, 16, 8), "NULL"), ((fake, 0, 256, 16, 8), "n must"),
             ((fake, 10, 250, 16, 8), "divide"), ((fake, 10, 256, 16, 9), "card_bits"),
             ((fake, 10, 8192, 16, 8), "len"), ((fake, 10, 256, 0, 8), "segments"),
             ((fake, 1 << 31, 256, 16, 8), "2^31")]
    for args, text in cases:
        assert not L.isax_build(*args)
        assert text in isax.last_error(), (args, isax.last_error())
    assert L.isax_breakpoints(0, (ctypes.c_float * 4)()) == isax.ISAX_EINVAL
    assert L.isax_query(None, fake, 1, 1, fake, fake) == isax.ISAX_EINVAL
    assert "index is NULL" in isax.last_error()
    assert L.isax_summarize(fake, 10, 30, 4, 8, fake, None, None) == isax.ISAX_EINVAL
    assert not L.isax_server_create(None, 0, None)
    L.isax_free(None)
    assert L.isax_clock() > 0


def test_struct_layouts_match_the_header(isax, tmp_path):
    # the ctypes mirrors of the option, statistics and result structs against
    # sizeof / offsetof of the same structs compiled from include/isax.h
    structs = {"isax_build_options": isax.BuildOptions, "isax_query_stats": isax.QueryStats,
               "isax_query_options": isax.QueryOptions, "isax_index_info": isax.IndexInfo,
               "isax_profile_entry": isax.ProfileEntry, "isax_server_options": isax.ServerOptions,
               "isax_result": isax.Result}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "isax.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)
