"""The C ABI library loads on the host and exports every function include/enoao.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "enoao.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(enoao_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("enoao_plan_create", "enoao_plan_destroy", "enoao_rhs", "enoao_step", "enoao_solve",
                 "enoao_batch_create", "enoao_batch_step", "enoao_get_selection", "enoao_status_string"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2108_12742_amd import enoao as E
    lib = E.lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_problem_struct_layout_matches_header():
    from paper_2108_12742_amd import enoao as E
    assert ctypes.sizeof(E.Problem) == 96
    assert E.Problem.x_lo.offset == 24 and E.Problem.bc_x.offset == 56 and E.Problem.flags.offset == 88


def test_status_strings_and_workspace_query():
    from paper_2108_12742_amd import enoao as E
    assert "non-physical" in E.enoao_status_string(E.ENONPHYSICAL)
    p = E.make_problem("euler2d", 2048, 2048)
    assert E.enoao_workspace_bytes(p) > 3 * 4 * 2048 * 2048 * 8
    bad = E.make_problem("euler2d", 2048, 2048, order=6)
    assert E.enoao_workspace_bytes(bad) == 0


def test_size_limits():
    """Extents up to ENOAO_MAX_EXTENT (2^31 - 1024) and at most 2^31 nodes are accepted;
    anything larger is rejected before any device work."""
    from paper_2108_12742_amd import enoao as E
    src = open(os.path.join(ROOT, "include", "enoao.h")).read()
    limit = int(re.search(r"#define ENOAO_MAX_EXTENT (\d+)", src).group(1))
    assert limit == E.MAX_EXTENT == 2**31 - 1024
    ok = E.make_problem("advection", limit)
    assert E.enoao_workspace_bytes(ok) >= 2 * limit * 8
    assert E.enoao_workspace_bytes(E.make_problem("advection", limit + 1)) == 0
    assert E.enoao_workspace_bytes(E.make_problem("euler2d", 2, limit + 1)) == 0
    assert E.enoao_workspace_bytes(E.make_problem("euler2d", 2**16, 2**15)) > 0
    assert E.enoao_workspace_bytes(E.make_problem("euler2d", 2**16, 2**15 + 1)) == 0
    assert E.enoao_workspace_bytes(E.make_problem("euler1d", 0)) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises: there is no CPU fallback."""
    from paper_2108_12742_amd import enoao as E
    monkeypatch.setattr(E, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(E, "_lib", None)
    with pytest.raises(ImportError, match="no CPU fallback"):
        E.lib()
    with pytest.raises(ImportError):
        E.enoao_workspace_bytes(E.make_problem("advection", 64))
