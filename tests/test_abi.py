"""CPU checks of the C-ABI boundary: the library exports every function that
include/dtsph.h declares, the binding's constants equal the header's, and its
ctypes structures have the header's layout (sizes and field offsets, from a
probe compiled against the header)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_1904_00861_amd import dtsph as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dtsph.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dtsph_\w+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(D.EXPORTS)


def test_option_and_status_codes_match_the_header():
    # every DTSPH_* integer constant the header defines has the same value in the
    # binding (options, precisions, status and stop codes)
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define DTSPH_(\w+)\s+\(?(-?\d+)\)?", txt)}
    assert "OPT_FILTER_LANES" in defs
    for name, value in defs.items():
        if hasattr(D, name):
            assert getattr(D, name) == value, name
    missing = [n for n in defs if n.startswith("OPT_") and not hasattr(D, n)]
    assert not missing, missing


def test_library_exports_every_declared_function():
    if not os.path.exists(D.LIB_PATH):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", D.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for f in declared_functions():
        assert f in syms, f
    L = D.lib()
    for f in declared_functions():
        assert hasattr(L, f)


STRUCTS = {"dtsph_sim_desc": D.SimDesc, "dtsph_state_view": D.StateView, "dtsph_cells_view": D.CellsView,
           "dtsph_iter_report": D.IterReport, "dtsph_timing": D.Timing, "dtsph_info": D.Info,
           "dtsph_tune_entry": D.TuneEntry, "dtsph_tune_report": D.TuneReport}


def test_struct_layouts_match_header():
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dtsph.h"', "int main(void){"]
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "probe.c"), os.path.join(d, "probe")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = dict(ln.rsplit(" ", 1) for ln in out.splitlines())
    for cname, py in STRUCTS.items():
        assert int(got[f"{cname} size"]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_create_rejects_bad_arguments_without_a_gpu():
    # argument checks run before any device call
    from paper_1904_00861_amd import inputs as I
    p = I.tgv2d(10)
    with pytest.raises(D.DtsphError) as e:
        D.dtsph_create([dict(p.params, dim=5)], [p.n], [0])
    assert e.value.status == D.EINVAL
    with pytest.raises(D.DtsphError) as e:
        D.dtsph_create([dict(p.params, h=0.4)], [p.n], [0])
    assert e.value.status == D.EINVAL and "half the period" in str(e.value)
