"""The C-ABI library loads without a GPU and exports every symbol the header
declares; host-side argument validation fails cleanly."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2009_06725_amd", "libscvs.so")
HDR = os.path.join(ROOT, "include", "scvs.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(scvs_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported(lib):
    names = _declared()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (scvs_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_binding_covers_header(lib):
    from paper_2009_06725_amd import scvs
    assert sorted(scvs.EXPORTED) == _declared()


def test_version_and_errors_without_gpu(lib):
    import ctypes as C
    from paper_2009_06725_amd import scvs
    assert scvs.version().startswith("scvs-gfx950")
    # null out-pointer: rejected before touching any device
    assert lib.scvs_ctx_create(0, None, None) == -1
    assert b"null" in lib.scvs_last_error()
    assert lib.scvs_ctx_set_mem_cap(None, C.c_uint64(1 << 30)) == -1
    # null mesh: rejected by validation
    assert lib.scvs_mesh_info(None, None) == -1
    o = scvs.default_opts()
    assert o.restart == 200 and o.rtol == 1e-10 and o.cheb_vel == 12 and o.cheb_pres == 50
    assert lib.scvs_solve(None, 1, None, None, None, None, None, None, C.byref(o), None) == -1


def test_oracle_not_imported_by_product():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2009_06725_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp")):
                assert "oracle" not in open(os.path.join(dp, f)).read().replace("Oracle", ""), f


def test_host_hermitian_eigensolver(lib):
    """The POD's host eigen-decomposition (cyclic Jacobi) against numpy."""
    import numpy as np
    from paper_2009_06725_amd import scvs
    rng = np.random.default_rng(4)
    for n in (1, 2, 7, 40):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        A = A + A.conj().T
        w, v = scvs.herm_eig(A)
        assert np.allclose(w, np.linalg.eigvalsh(A)[::-1], atol=1e-12 * max(1.0, np.abs(w).max()))
        assert np.abs(A @ v - v * w).max() < 1e-11 * max(1.0, np.abs(w).max())
        assert np.abs(v.conj().T @ v - np.eye(n)).max() < 1e-12
