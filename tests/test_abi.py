"""The C-ABI library loads on the CPU and exports every symbol include/dgdcr.h
declares; host-side validation returns error codes (no device work)."""
import os
import re

import numpy as np
import pytest

from paper_1502_02941_amd import api
from paper_1502_02941_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dgdcr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = api.lib()
    names = declared_functions()
    assert len(names) >= 13
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(api.EXPORTS)


def test_default_penalty_table():
    assert api.default_penalty(api.NIPG, 3) == (1.0, 1.0)
    assert api.default_penalty(api.SIPG, 2) == (18.0, -1.0)
    assert api.default_penalty(api.IIPG, 3) == (36.0, 0.0)
    for bad, code in (((7, 1), -6), ((2, 0), -5), ((2, 9), -5)):
        with pytest.raises(api.DGError) as e:
            api.default_penalty(*bad)
        assert e.value.status == code


@pytest.mark.parametrize("what,code", [("clockwise", -2), ("missing_bc", -3), ("duplicate_bc", -3),
                                       ("interior_listed", -3), ("three_elems", -4), ("degree", -5),
                                       ("nan", -7), ("node_range", -1), ("no_elements", -1)])
def test_mesh_validation_errors(what, code):
    m = W.structured_mesh(3)
    nodes, el, d, nm, k = m.nodes.copy(), m.elems.copy(), m.dirichlet.copy(), m.neumann.copy(), 1
    if what == "clockwise":
        el[4] = el[4][::-1]
    elif what == "missing_bc":
        d = d[:-1]
    elif what == "duplicate_bc":
        nm = d[:1].copy()
    elif what == "interior_listed":
        d = np.concatenate([d, [[0, 5]]]).astype(np.int32)
    elif what == "three_elems":
        el = np.concatenate([el, [[0, 1, 5]]]).astype(np.int32)
    elif what == "degree":
        k = 5
    elif what == "nan":
        nodes[3, 0] = np.nan
    elif what == "node_range":
        el[0, 0] = 999
    elif what == "no_elements":
        el, d, nm = el[:0], d[:0], nm[:0]
    with pytest.raises(api.DGError) as e:
        api.Mesh(nodes, el, d, nm, k)
    assert e.value.status == code


def test_status_strings():
    assert api.status_str(0) == "DG_OK" and api.status_str(-9) == "DG_ERR_OOM"


def test_batch_rejects_bad_instances_on_host():
    m = W.structured_mesh(4)
    ok = api.Problem(api.SIPG, 1, 6.0, eps=0.01, bx=1.0, by=0.0, alpha=0.0, f=1.0)
    bad_deg = api.Problem(api.SIPG, 3, 36.0, eps=0.01, bx=1.0, by=0.0, alpha=0.0, f=1.0)
    with pytest.raises(api.DGError) as e:
        api.Batch([(m, ok), (m, bad_deg)])
    assert e.value.status == -5
    bad_field = api.Problem(api.SIPG, 1, 6.0, eps=api.Field.gauss_sum([(0.5, 0.5, 0.1, 1.0)]), bx=1.0, by=0.0,
                            alpha=0.0, f=1.0)
    with pytest.raises(api.DGError) as e:
        api.Batch([(m, bad_field)])
    assert e.value.status == -1
    bad_mesh = W.MeshArrays(m.nodes, m.elems[:, ::-1].copy(), m.dirichlet, m.neumann)
    with pytest.raises(api.DGError) as e:
        api.Batch([(bad_mesh, ok)])
    assert e.value.status == -2


STRUCTS = {"dg_field": "_Field", "dg_problem": "_Problem", "dg_mesh_info": "_MeshInfo",
           "dg_solver_opts": "_SolverOpts", "dg_kernel_stats": "_KStats", "dg_solve_report": "_Report",
           "dg_instance": "_Instance", "dg_batch_opts": "_BatchOpts", "dg_reaction": "_Reaction",
           "dg_newton_opts": "_NewtonOpts", "dg_newton_report": "_NewtonReport", "dg_euler_report": "_EulerReport"}


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes mirror has the size and field offsets a C compiler gives the header."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dgdcr.h"', "int main(void) {"]
    for cname, pname in STRUCTS.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in getattr(api, pname)._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, pname in STRUCTS.items():
        cls = getattr(api, pname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
    assert api.REPORT_DTYPE.itemsize == ctypes.sizeof(api._Report)
    for fname, (_, off) in api.REPORT_DTYPE.fields.items():
        assert off == getattr(api._Report, {"reorth": "reorth_passes"}.get(fname, fname)).offset


def test_mesh_create_rejects_unknown_basis():
    m = W.structured_mesh(3)
    for bad in (-1, 2, 7):
        with pytest.raises(api.DGError) as e:
            api.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann, 1, basis=bad)
        assert e.value.status == -1
