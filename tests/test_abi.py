"""The C ABI library loads on the host and exports every entry point that
include/lbm.h declares; host-only parameter validation (no device call)."""
import os
import re

import pytest

from paper_1802_01272_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_documented_calls():
    names = declared_functions()
    for n in ("lbm_init", "lbm_step", "lbm_moments", "lbm_reduce", "lbm_batch_step", "lbm_autotune"):
        assert n in names


def test_library_exports_every_declared_symbol():
    missing = [n for n in declared_functions() if not hasattr(lbm.LIB, n)]
    assert not missing, missing


def test_binding_struct_matches_header():
    """The ctypes mirror of lbm_params has the header's fields, in order and
    with the same C types."""
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\} lbm_params;", src, flags=re.S).group(1)
    fields = []
    for ctype, names in re.findall(r"(int32_t|double)\s+([^;]+);", body):
        fields += [(n.strip(), ctype) for n in names.split(",")]
    ct = {"int32_t": "c_int", "double": "c_double"}
    got = [(n, t.__name__) for n, t in lbm.CParams._fields_]
    assert got == [(n, ct[t]) for n, t in fields]
    assert [f for f, _ in got] == [f.name for f in lbm.fields(lbm.Params)]


def test_version_and_error_strings():
    assert "gfx950" in lbm.version()


def base():
    return lbm.Params(Lx=64, Ly=32)


def test_validate_accepts_paper_parameters():
    assert lbm.validate(base()) == lbm.LBM_OK
    assert lbm.workspace_bytes(base()) > 2 * 16 * 64 * 32 * 8


@pytest.mark.parametrize("field,value,status", [
    ("dt", 0.45, lbm.LBM_ECFL), ("Lx", 0, lbm.LBM_EINVAL), ("tau", 0.0, lbm.LBM_EINVAL),
    ("T", -1.0, lbm.LBM_EINVAL), ("scheme", 3, lbm.LBM_EINVAL), ("precision", 2, lbm.LBM_EINVAL),
    ("kappa", -1.0, lbm.LBM_EINVAL), ("ds", float("nan"), lbm.LBM_EINVAL), ("bc_y", 2, lbm.LBM_EINVAL),
    ("rounding", 2, lbm.LBM_EINVAL),
])
def test_validate_rejects(field, value, status):
    p = base()
    setattr(p, field, value)
    assert lbm.validate(p) == status
    assert lbm.workspace_bytes(p) == 0
    assert lbm.LIB.lbm_last_error().decode()


def test_cfl_limit_is_the_papers():
    """max_k |xi_k| dt <= ds with max |xi| = sqrt(3 + sqrt 6)."""
    lim = 1.0 / (3 + 6 ** 0.5) ** 0.5
    p = base()
    p.dt = lim * 0.999999
    assert lbm.validate(p) == lbm.LBM_OK
    p.dt = lim * 1.0001
    assert lbm.validate(p) == lbm.LBM_ECFL


def test_fp32_workspace_is_half_of_fp64():
    p = lbm.Params(Lx=1024, Ly=1024)
    a = lbm.workspace_bytes(p)
    p.precision = lbm.FP32_DEV
    b = lbm.workspace_bytes(p)
    assert abs((a - b) - 2 * 16 * 1024 * 1024 * 4) < 1 << 20


def test_size_limit_is_two_to_the_26_nodes():
    """A buffer descriptor spans eight distribution planes: with FP32 storage
    8192 x 8192 = 2^26 nodes is accepted and one row more is refused; with
    FP64 storage eight planes of 2^26 nodes would reach byte 2^32, one past
    the descriptor's range, so the limit is 2^26 - 1 (with walls, the two
    ghost rows count)."""
    p = lbm.Params(Lx=8192, Ly=8192, precision=lbm.FP32_DEV)
    assert lbm.validate(p) == lbm.LBM_OK
    p.Ly = 8193
    assert lbm.validate(p) == lbm.LBM_EINVAL
    p = lbm.Params(Lx=8192, Ly=8190, bc_y=lbm.SHEAR_WALLS, precision=lbm.FP32_DEV)
    assert lbm.validate(p) == lbm.LBM_OK
    p.Ly = 8191
    assert lbm.validate(p) == lbm.LBM_EINVAL
    p = lbm.Params(Lx=8192, Ly=8192, precision=lbm.FP64)
    assert lbm.validate(p) == lbm.LBM_EINVAL
    p.Ly = 8191
    assert lbm.validate(p) == lbm.LBM_OK
    p = lbm.Params(Lx=8191, Ly=8193, precision=lbm.FP64)    # 2^26 - 1 nodes
    assert lbm.validate(p) == lbm.LBM_OK
