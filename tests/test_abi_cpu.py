"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/mesh_sdd.h declares, its struct layouts match the header, and its
host-only logic (descriptor validation, interface-node enumeration of
section 3.5) agrees exactly with the oracle.  No compute call is made
(there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mesh_sdd.h")


@pytest.fixture(scope="module")
def M():
    from paper_1504_00084_amd import mesh_sdd
    if not os.path.exists(mesh_sdd.LIB_PATH):
        from paper_1504_00084_amd import build
        build.build()
    mesh_sdd.load()
    return mesh_sdd


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mesh_sdd_\w+)\s*\(", text)))


def test_header_declarations_are_exported(M):
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(M.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", M.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mesh_sdd_\w+)", out))
    assert set(names) <= exported
    assert set(M.EXPORTS) == set(names)


def test_struct_layouts_match_header(M, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "mesh_sdd.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(mesh_sdd_desc), '
                   'sizeof(mesh_sdd_step), sizeof(mesh_sdd_result), sizeof(mesh_sdd_stats), sizeof(mesh_sdd_launch), '
                   'offsetof(mesh_sdd_desc, seed), offsetof(mesh_sdd_step, mesh_step), '
                   'offsetof(mesh_sdd_result, device_ms), sizeof(mesh_sdd_mp_opts), '
                   'offsetof(mesh_sdd_mp_opts, fe_cfl));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(M.Desc), ctypes.sizeof(M.Step), ctypes.sizeof(M.Result), ctypes.sizeof(M.Stats),
            ctypes.sizeof(M.Launch), M.Desc.seed.offset, M.Step.mesh_step.offset, M.Result.device_ms.offset,
            ctypes.sizeof(M.MpOpts), M.MpOpts.fe_cfl.offset]
    assert got == want


def test_version_and_empty_error(M):
    assert "gfx950" in M.mesh_sdd_version()


@pytest.mark.parametrize("kw,frag", [
    (dict(n_xi=3), "grid"), (dict(sub_xi=5), "sub"), (dict(sub_eta=0), "sub"), (dict(K=0), "K ="),
    (dict(tau=0.0), "tau"), (dict(tau=float("nan")), "tau"), (dict(Lx=-1.0), "Lx"), (dict(precision=2), "precision"),
    (dict(bridge=3), "bridge"), (dict(instance_id=70000), "instance_id"), (dict(periodic_xi=2), "periodic"),
])
def test_desc_validation(M, kw, frag):
    base = dict(n_xi=33, n_eta=33, sub_xi=2, sub_eta=1)
    base.update(kw)
    d = M.make_desc(**base)
    with pytest.raises(M.MeshSddError) as e:
        M.mesh_sdd_desc_check(d)
    assert e.value.code == M.E_INVAL
    assert frag in str(e.value)
    bad = M.make_desc(33, 33, 2, 1)
    bad.struct_size = 4
    with pytest.raises(M.MeshSddError):
        M.mesh_sdd_desc_check(bad)


@pytest.mark.parametrize("n_xi,n_eta,sx,sy,px,py", [
    (33, 33, 2, 1, 0, 0), (129, 129, 4, 4, 0, 0), (257, 257, 8, 8, 1, 0), (513, 513, 16, 16, 0, 0),
    (17, 9, 4, 2, 0, 1), (9, 17, 1, 1, 1, 1), (31, 13, 3, 4, 0, 0), (9, 9, 1, 1, 0, 0), (65, 33, 16, 2, 1, 1),
])
def test_interface_nodes_match_oracle(M, oracle_lib, n_xi, n_eta, sx, sy, px, py):
    d = M.make_desc(n_xi, n_eta, sx, sy, px, py)
    i, j = M.mesh_sdd_desc_interface_nodes(d)
    oi, oj = oracle_lib.interface_nodes(oracle_lib.Problem(n_xi=n_xi, n_eta=n_eta, sub_xi=sx, sub_eta=sy,
                                                           periodic_xi=px, periodic_eta=py))
    assert np.array_equal(i, oi) and np.array_equal(j, oj)


def test_no_gpu_context_fails_cleanly(M):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(M.MeshSddError) as e:
        M.mesh_sdd_ctx_create(0)
    assert e.value.code in (M.E_DEVICE, M.E_INVAL)
