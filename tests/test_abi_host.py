"""Host-side checks of the C ABI that need no GPU: every function declared in
include/mpm.h is exported by libmpm.so, parameter validation, workspace sizing, and the
host sampler (the input stage) against the oracle's sampler."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import mpm_scenes as sc
from paper_2101_12408_amd import _lib as L
from paper_2101_12408_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|double|const char\*)\s+(mpm_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(L.EXPORTS), set(names) - set(L.EXPORTS)


def test_struct_sizes_match_header_layout():
    # 16 int32 then doubles, particles 8 + 9 pointers (x ... gradT, F)
    assert C.sizeof(L.MpmParticles) == 8 + 9 * 8
    assert C.sizeof(L.MpmSurface) == 8 + 3 * 8
    assert L.MpmParams.dx.offset == 64


def test_params_and_workspace_validation():
    lib = L.load()
    p = L.MpmParams()
    assert lib.mpm_params_default(C.byref(p), 4, 64) == L.MPM_EINVAL
    assert lib.mpm_params_default(C.byref(p), 3, 64) == L.MPM_OK
    nb = C.c_size_t(0)
    assert lib.mpm_workspace_bytes(C.byref(p), 1000, 100, C.byref(nb)) == L.MPM_OK
    small = nb.value
    assert lib.mpm_workspace_bytes(C.byref(p), 100000, 100, C.byref(nb)) == L.MPM_OK
    assert nb.value > small
    p.n = 60
    assert lib.mpm_workspace_bytes(C.byref(p), 1000, 100, C.byref(nb)) == L.MPM_EINVAL
    p.n = 64
    p.dx = 0.1
    assert lib.mpm_workspace_bytes(C.byref(p), 1000, 100, C.byref(nb)) == L.MPM_EINVAL
    p.dx = 1 / 64
    assert lib.mpm_workspace_bytes(C.byref(p), -1, 100, C.byref(nb)) == L.MPM_EINVAL
    out = C.c_void_p()
    assert lib.mpm_ctx_create(C.byref(p), None, 0, 10, 10, C.byref(out)) == L.MPM_EINVAL


def test_tiled_index_matches_header_formula():
    for dim, n in ((2, 16), (3, 16)):
        idx = api.tiled_index(dim, n)
        assert np.array_equal(np.sort(idx), np.arange(n ** dim))
        E = 4 if dim == 3 else 8
        i = np.array([5, 11, 2][:dim])
        nat = i[0] + n * i[1] + (n * n * i[2] if dim == 3 else 0)
        tile = i[0] // E + (n // E) * (i[1] // E + ((n // E) * (i[2] // E) if dim == 3 else 0))
        loc = i[0] % E + E * (i[1] % E + (E * (i[2] % E) if dim == 3 else 0))
        assert idx[nat] == tile * 64 + loc


@pytest.mark.parametrize("case", ["square2d", "droplet3d", "contact3d"])
def test_host_sampler_matches_oracle(case):
    from oracle import sampler
    if case == "square2d":
        S = sc.square2d(n=32)
    elif case == "droplet3d":
        S = sc.droplet3d(16, 3, 0.05, [10, 0, 0])
    else:
        S = sc.contact3d(n=64, radius=0.08)
    P, p = S["particles"], S["params"]
    ref = sampler.sample_surface(P["x"], p, step=3)
    got = api.sample_surface(P["x"], p, step=3)
    assert len(got["s"]) == len(ref["s"])
    assert np.allclose(got["s"], ref["s"], rtol=0, atol=1e-13)
    assert np.allclose(got["dA"], ref["dA"], rtol=0, atol=1e-15)
    assert np.array_equal(got["label"], ref["label"])
    if case == "contact3d":
        assert 0 < ref["label"].sum() < len(ref["label"])


def test_struct_layouts_match_c_compiler(tmp_path):
    """sizeof / offsetof of every ABI struct as the C compiler lays it out, against the
    ctypes declarations of the binding."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    structs = {"mpm_params": L.MpmParams, "mpm_particles": L.MpmParticles, "mpm_surface": L.MpmSurface,
               "mpm_stats": L.MpmStats, "mpm_request": L.MpmRequest, "mpm_completion": L.MpmCompletion,
               "mpm_server_info": L.MpmServerInfo, "mpm_tuning": L.MpmTuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpm.h"', 'int main(void) {']
    for cname, ct in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in ct._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, ct in structs.items():
        assert got[(cname, "size")] == C.sizeof(ct), cname
        for f, _ in ct._fields_:
            assert got[(cname, f)] == getattr(ct, f).offset, (cname, f)
