"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every call include/lasto.h declares, its structs have the layout the
binding assumes, and the host mesh helper agrees with the oracle."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_0806_1723_amd import inputs as I
from paper_0806_1723_amd import lasto as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lasto.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lasto_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_call():
    lib = L.load()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.check_output(["nm", "-D", "--defined-only", L.LIB_PATH]).decode()
    exported = set(re.findall(r" T (lasto_\w+)", out))
    assert set(names) <= exported
    assert set(L.SYMBOLS) == set(names)


def test_struct_layouts_match_the_header(tmp_path):
    prog = tmp_path / "sizes.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lasto.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lasto_atom), '
                    'sizeof(lasto_solve_opts), sizeof(lasto_solve_info), '
                    'offsetof(lasto_solve_info, smooth_ms), offsetof(lasto_atom, clm), '
                    'offsetof(lasto_solve_opts, atoms), offsetof(lasto_solve_opts, coarse_net_level), '
                    'offsetof(lasto_solve_info, ms_bc), offsetof(lasto_solve_info, alg_bytes), '
                    'offsetof(lasto_solve_opts, inner_rate), offsetof(lasto_solve_info, inner_rate), '
                    'offsetof(lasto_solve_info, rel_start), offsetof(lasto_solve_opts, graphs), '
                    'offsetof(lasto_solve_opts, nu_coarse), offsetof(lasto_solve_opts, fused_sweeps));return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(L.Atom), C.sizeof(L.SolveOpts), C.sizeof(L.SolveInfo),
            L.SolveInfo.smooth_ms.offset, L.Atom.clm.offset, L.SolveOpts.atoms.offset,
            L.SolveOpts.coarse_net_level.offset, L.SolveInfo.ms_bc.offset, L.SolveInfo.alg_bytes.offset,
            L.SolveOpts.inner_rate.offset, L.SolveInfo.inner_rate.offset, L.SolveInfo.rel_start.offset,
            L.SolveOpts.graphs.offset, L.SolveOpts.nu_coarse.offset, L.SolveOpts.fused_sweeps.offset]
    assert got == want


def test_status_strings_and_defaults():
    assert L.status_string(0) == "ok"
    assert L.status_string(4) == "not converged"
    o = L.default_opts()
    assert (o.rtol, o.max_iters, o.nu1, o.nu2, o.method, o.precision, o.bc, o.lmax_bc, o.guess) == \
        (1e-10, 100, 2, 2, 0, 0, 1, 4, 0)
    assert o.debug_nan_iter == -1 and o.profile == 0 and o.inner_rate == 0.0 and o.graphs == 0
    assert o.fused_sweeps == 0


@pytest.mark.parametrize("cid,sample", [(1, 0), (2, 0), (3, 0), (5, 0), (4, 0), (4, 17)])
def test_mesh_helper_matches_oracle(oracle_mod, cid, sample):
    w = I.config(cid, sample=sample)
    a = L.mesh_for(w.axes)
    b = oracle_mod.mesh_for(w.axes)
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.abs(x - y).max() <= 1e-13 * np.abs(y).max()


def test_mesh_helper_errors():
    with pytest.raises(L.LastoError) as e:
        L.mesh_graded_1d(0.0, 1.0, 2, [], 0.1, 0.2)
    assert e.value.status == L.ERR_ARG
    with pytest.raises(L.LastoError):
        L.mesh_graded_1d(-20, 20, 65, [0.0], 0.01, 0.6, 1.05)   # infeasible, no hmin steps
    x, g, hm = L.mesh_graded_1d(-20, 20, 65, [0.0], 0.01, 1.0, 1.05, 0.01)
    assert hm > 0.01 and g <= 1.05


def test_binding_refuses_host_tensors():
    import torch
    with pytest.raises(TypeError):
        L._dev_ptr(torch.zeros(3, dtype=torch.float64))


def test_noalloc_limit_matches_the_header():
    src = open(HEADER).read()
    m = re.search(r"#define LASTO_NOALLOC_MAX_POINTS (\d+)", src)
    assert m and int(m.group(1)) == L.NOALLOC_MAX_POINTS
