"""Host-side checks of the C ABI (no GPU needed).

The library must load and export every function include/femh.h declares;
descriptor and wave validation, and the device-footprint estimate, run on
the host and are checked against the exact counts of the mesh bookkeeping.
"""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_0704_2344_amd import femh as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "femh.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s+(femh_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(F.LIB_PATH):
        pytest.fail("libfemh.so is not built: run `python -m paper_0704_2344_amd.build`")
    return F.load()


def test_library_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), f"{n} declared in femh.h but not exported"
    # and the binding knows the signature of every one of them
    assert set(names) == set(F.SIGNATURES)


def test_library_targets_gfx950_only():
    data = open(F.LIB_PATH, "rb").read()
    assert b"gfx950" in data
    for other in (b"gfx942", b"gfx90a", b"gfx1100", b"gfx906"):
        assert other not in data


def _desc(prob):
    keep = F._Keep()
    return F.make_desc(prob, None, keep), keep


def _validate(lib, prob):
    d, keep = _desc(prob)
    buf = C.create_string_buffer(256)
    st = lib.femh_validate_desc(C.byref(d), buf, 256)
    return st, buf.value.decode()


def test_validation_accepts_workloads(lib):
    for name, make in W.WORKLOADS.items():
        if name == "pec_sphere_shell_60":
            continue  # big host scan; covered by the estimate test
        p, waves = make()
        st, msg = _validate(lib, p)
        assert st == F.FEMH_OK, msg
        w = F.make_waves(waves)
        buf = C.create_string_buffer(256)
        assert lib.femh_validate_waves(len(waves), w, buf, 256) == F.FEMH_OK


def test_validation_accepts_plane_faces(lib):
    """Symmetry (2) and antisymmetry (3) plane tags are valid outer faces."""
    for cut_x, cut_y in ((True, False), (False, True), (True, True)):
        p, _ = W.mirrored_pec_cube(6, cut_x=cut_x, cut_y=cut_y)
        st, msg = _validate(lib, p)
        assert st == F.FEMH_OK, msg
    p, _ = W.free_cube(3)
    p.faces = (F.FEMH_FACE_SYM, F.FEMH_FACE_ANTISYM, F.FEMH_FACE_NATURAL, F.FEMH_FACE_ABC, 2, 3)
    assert _validate(lib, p)[0] == F.FEMH_OK


def test_validation_rejects_bad_descriptors(lib):
    p, _ = W.free_cube(3)
    bad = []
    q = W._blank(0, 3, 3, (0.1,) * 3, (0, 0, 0), 1.0)
    bad.append((q, F.FEMH_E_INVALID))
    q, _ = W.free_cube(3)
    q.h = (0.1, -0.1, 0.1)
    bad.append((q, F.FEMH_E_INVALID))
    q, _ = W.free_cube(3)
    q.k0 = 0.0
    bad.append((q, F.FEMH_E_INVALID))
    q, _ = W.free_cube(3)
    q.k0 = float("nan")
    bad.append((q, F.FEMH_E_NONFINITE))
    q, _ = W.free_cube(3)
    q.eps_r[1, 1, 1] = np.nan
    bad.append((q, F.FEMH_E_NONFINITE))
    q, _ = W.free_cube(3)
    q.eps_r[0, 0, 0] = 0.0
    bad.append((q, F.FEMH_E_INVALID))
    q, _ = W.free_cube(3)
    q.pec[:] = 1
    bad.append((q, F.FEMH_E_INVALID))
    q, _ = W.free_cube(3)
    q.faces = (0, 0, 7, 0, 0, 0)
    bad.append((q, F.FEMH_E_INVALID))
    q, _ = W.free_cube(3)
    q.faces = (0, 0, 4, 0, 0, 0)
    bad.append((q, F.FEMH_E_INVALID))
    q, _ = W.free_cube(3)
    q.faces = (0, -1, 0, 0, 0, 0)
    bad.append((q, F.FEMH_E_INVALID))
    q, _ = W.free_cube(3)
    q.penalty_s = -1.0
    bad.append((q, F.FEMH_E_INVALID))
    for prob, want in bad:
        st, msg = _validate(lib, prob)
        assert st == want, (st, msg)
        assert msg
        assert F.last_error()


def test_wave_validation(lib):
    buf = C.create_string_buffer(256)
    good = W.PlaneWave(d=np.array([0.0, 0.0, 1.0]), p=np.array([1.0, 0.0, 0.0], np.complex128))
    assert lib.femh_validate_waves(1, F.make_waves([good]), buf, 256) == F.FEMH_OK
    not_unit = W.PlaneWave(d=np.array([0.0, 0.0, 2.0]), p=np.array([1.0, 0.0, 0.0], np.complex128))
    assert lib.femh_validate_waves(1, F.make_waves([not_unit]), buf, 256) == F.FEMH_E_INVALID
    not_perp = W.PlaneWave(d=np.array([0.0, 0.0, 1.0]), p=np.array([0.0, 0.3j, 1.0], np.complex128))
    assert lib.femh_validate_waves(1, F.make_waves([not_perp]), buf, 256) == F.FEMH_E_INVALID
    nan = W.PlaneWave(d=np.array([0.0, 0.0, 1.0]), p=np.array([np.nan, 0.0, 0.0], np.complex128))
    assert lib.femh_validate_waves(1, F.make_waves([nan]), buf, 256) == F.FEMH_E_NONFINITE
    assert lib.femh_validate_waves(0, F.make_waves([good]), buf, 256) == F.FEMH_E_INVALID


def _estimate(lib, prob, nrhs=1, prec=F.FEMH_FP64):
    d, keep = _desc(prob)
    out = C.c_int64()
    assert lib.femh_estimate_bytes(C.byref(d), nrhs, prec, C.byref(out)) == F.FEMH_OK
    return out.value


@pytest.mark.parametrize("name,nn,nnzb", [
    # active nodes and 3x3 blocks of the workloads (exact bookkeeping)
    ("free_cube_10", 1331, 29791),
    ("pec_cube_30", 29062, 729182),
])
def test_footprint_estimate_counts(lib, name, nn, nnzb):
    from oracle import fem
    p, _ = W.WORKLOADS[name]()
    mesh = fem.Mesh(p)
    assert mesh.n_nodes == nn
    est = _estimate(lib, p, nrhs=0)
    # matrix values dominate: 144 + 72 bytes per block (+ 4 for the column index)
    assert est >= 216 * nnzb
    ne = p.nx * p.ny * p.nz
    assert est <= 220 * nnzb + 100 * nn + 4 * mesh.node_active.size + 33 * ne + (2 << 20)
    # blocks = node pairs sharing an active element (oracle pattern)
    rp, ci = fem.block_pattern(p)
    assert len(ci) == nnzb


def test_footprint_estimate_grows_with_rhs_and_precision(lib):
    p, _ = W.free_cube(10)
    e1 = _estimate(lib, p, 1, F.FEMH_FP64)
    e4 = _estimate(lib, p, 4, F.FEMH_FP64)
    em = _estimate(lib, p, 1, F.FEMH_MIXED)
    # the mixed form's workspace (an FP64 residual, four complex64 vectors)
    # is three complex128 vectors, two fewer than FP64's, and it has three
    # fewer partial buffers
    v64 = (48 * 1331 + 255) // 256 * 256
    assert e4 > e1 and em >= e1 - 2 * v64 - 3 * 8 * 2048 * 4


def test_footprint_estimate_per_rhs_workspace(lib):
    """Per right-hand side the FP64 solver (single-reduction form) holds two
    more complex128 vectors (z = D^-1 r and s = A p) and three more partial
    buffers (two update buffers of 2048 x 8 doubles) than the matrix-mixed
    one, which keeps the textbook order."""
    p, _ = W.free_cube(10)
    nn = 1331
    v64 = (48 * nn + 255) // 256 * 256
    per = {}
    for prec in (F.FEMH_FP64, F.FEMH_MIXED_MATRIX):
        per[prec] = _estimate(lib, p, 3, prec) - _estimate(lib, p, 2, prec)
    d = per[F.FEMH_FP64] - per[F.FEMH_MIXED_MATRIX]
    assert d == 2 * v64 + 3 * 8 * 2048 * 4


def test_context_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = lib.femh_ctx_create(0, None, None, C.byref(h))
    assert st == F.FEMH_E_DEVICE
    assert "device" in F.last_error().lower()
    assert not h.value


def test_null_handles_are_safe(lib):
    lib.femh_ctx_destroy(None)
    lib.femh_problem_destroy(None)
    lib.femh_server_destroy(None)
    assert lib.femh_problem_get_info(None, None) == F.FEMH_E_INVALID


def test_struct_layouts_match_header(tmp_path):
    """Every public struct of include/femh.h has the size and field offsets
    the ctypes binding declares (a C program compiled against the header
    prints them)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    names = ["femh_allocator", "femh_problem_desc", "femh_plane_wave", "femh_solve_opts", "femh_solve_stats",
             "femh_problem_info", "femh_server_opts", "femh_server_report"]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "femh.h"', "int main(void) {"]
    for n in names:
        cls = getattr(F, n)
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{n} {fname} %zu\\n", offsetof({n}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for n in names:
        cls = getattr(F, n)
        assert got[(n, "size")] == C.sizeof(cls), n
        for fname, _ in cls._fields_:
            assert got[(n, fname)] == getattr(cls, fname).offset, (n, fname)


def _bare_problem(n_unknowns=12, grid_nodes=8):
    """A Problem wrapper with no device object behind it: the tensor checks
    must refuse bad buffers before anything reaches the library."""
    from types import SimpleNamespace

    P = F.Problem.__new__(F.Problem)
    P.handle = None
    P.lib = None
    P.ctx = SimpleNamespace(device=0)
    P.n_unknowns = n_unknowns
    P.grid_nodes = grid_nodes
    P.n_nodes = n_unknowns // 3
    P.spec = SimpleNamespace(nx=1, ny=1, nz=1)
    return P


def test_device_buffer_checks_refuse_host_tensors():
    import torch

    P = _bare_problem()
    x = torch.zeros(12, dtype=torch.complex128)
    for call in (lambda: P.spmv_dev(x, x), lambda: P.spmv_half_dev(x, x),
                 lambda: P.spmm_dev(x.reshape(12, 1), x.reshape(12, 1)),
                 lambda: P.solve_dev([], torch.zeros(0, dtype=torch.complex128))):
        with pytest.raises(F.FemhError) as e:
            call()
        assert e.value.status == F.FEMH_E_INVALID


def test_device_buffer_checks_refuse_bad_shapes_and_types():
    import torch

    P = _bare_problem()
    # wrong element type for the precision: complex64 vectors are FEMH_MIXED only
    with pytest.raises(F.FemhError, match="cuda"):
        P.spmv_dev(torch.zeros(12, dtype=torch.complex64), torch.zeros(12, dtype=torch.complex64))
    with pytest.raises(F.FemhError, match="unknown precision"):
        P.spmv_dev(torch.zeros(12, dtype=torch.complex128), torch.zeros(12, dtype=torch.complex128), precision=7)
    # SpMM blocks must be [n_unknowns, ncols], 1 <= ncols <= 64
    for shape in ((11, 2), (12, 65), (12,)):
        X = torch.zeros(shape, dtype=torch.complex128)
        with pytest.raises(F.FemhError, match="spmm_dev"):
            P.spmm_dev(X, X)
    # the checker itself, on each property in turn
    t = torch.zeros(12, dtype=torch.complex128)
    with pytest.raises(F.FemhError, match="cuda"):
        F.check_device_tensor(t, torch.complex128, 12, 0, "t")
    with pytest.raises(F.FemhError, match="torch tensor"):
        F.check_device_tensor(np.zeros(12, np.complex128), torch.complex128, 12, 0, "t")
